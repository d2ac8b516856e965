"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad configurations on the host before touching a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psweep.h")


def _lib_or_skip():
    from paper_1809_06132_amd import psweep
    if not os.path.exists(psweep.LIB_PATH):
        pytest.skip("libpsweep.so not built (run __graft_entry__.build())")
    return psweep


def _declared():
    import glob
    text = "".join(open(h).read() for h in glob.glob(os.path.join(ROOT, "include", "*.h")))
    return set(re.findall(r"\b(psweep_[a-z_]+)\s*\(", text))


def test_header_and_binding_agree():
    decl = _declared()
    from paper_1809_06132_amd import psweep
    assert decl == set(psweep.EXPORTS), decl ^ set(psweep.EXPORTS)


def test_library_exports_every_symbol():
    psweep = _lib_or_skip()
    L = psweep.lib()
    for name in psweep.EXPORTS:
        assert hasattr(L, name), name
    assert psweep.psweep_version().startswith("psweep-gfx950")


def _cfg(psweep, **kw):
    c = psweep.psweep_config()
    c.n_levels = 1
    L = c.level[0]
    L.n_fronto, L.near_m, L.far_m, L.window, L.downsample = 32, 0.5, 30.0, 7, 1
    c.ground_n[:] = [0.0, 1.0, 0.0]
    c.ground_d = 1.5
    c.best_k, c.var_floor, c.temperature = 1, 1.0, 0.1
    c.max_width, c.max_height, c.max_sources, c.max_frames, c.max_camera_sets = 320, 256, 1, 1, 1
    for k, v in kw.items():
        if "." in k:
            a, b = k.split(".")
            setattr(c.level[int(a)], b, v)
        else:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,status", [
    ({"0.window": 8}, -1),                # even window
    ({"0.window": 17}, -1),               # too large
    ({"0.n_fronto": 1}, -1),              # a family needs 2 planes
    ({"0.near_m": 40.0}, -1),             # near beyond far
    ({"best_k": 2}, -1),                  # more than max_sources
    ({"max_sources": 5}, -1),
    ({"n_levels": 3}, -1),
    ({"storage": 7}, -1),
    ({"0.n_ground": 4, "0.h_lo": -0.5, "0.h_hi": 0.5, "ground_d": 0.2}, -1),  # planes above the camera
    ({"mode": 1, "storage": 1}, -5),                                         # soft mode stages in FP32
    ({"mode": 1, "launch": 1}, -5),
    ({"launch": 1, "0.window": 5}, -5),
    ({"0.crop_w": 100, "0.crop_h": 100}, -5),
    ({"0.crop_w": 100, "0.crop_h": 0}, -1),                                 # crop with no height
    ({"image_format": 2}, -1),                                              # unknown pixel type
    ({"image_format": 1, "0.downsample": 2}, -5),                           # float images: full resolution
    ({"image_format": 1, "0.window": 9, "launch": 1}, -5),                  # float images: grid launch
    ({"image_format": 1, "storage": 1}, -5),                                # float images: FP32 staging
])
def test_create_rejects_bad_config(kw, status):
    psweep = _lib_or_skip()
    with pytest.raises(psweep.PsweepError) as ei:
        psweep.psweep_create(_cfg(psweep, **kw))
    assert ei.value.status == status
    assert psweep.psweep_last_error(None)


def test_null_arguments():
    psweep = _lib_or_skip()
    L = psweep.lib()
    assert L.psweep_create(None, None) == psweep.EINVAL
    assert L.psweep_workspace_size(None, None) == psweep.EINVAL
    assert L.psweep_run(None, None, 0, None, None) == psweep.EINVAL
    assert L.psweep_soft_depth_backward(None, None, None, None, None) == psweep.EINVAL
    assert L.psweep_mask_boxes(None, 0, None, None, 0, 0, None, None) == psweep.EINVAL


def test_product_path_is_independent_of_the_oracle():
    """The package never imports, loads or calls the oracle, and the oracle
    never includes the GPU sources: the two share no code."""
    pkg = os.path.join(ROOT, "paper_1809_06132_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "or_sweep" not in text, f
    otext = open(os.path.join(ROOT, "oracle", "psweep_oracle.c")).read()
    assert "#include \"" not in otext and "psw::" not in otext
    assert "paper_1809_06132_amd" not in open(os.path.join(ROOT, "oracle", "__init__.py")).read()


def test_tsdf_rejects_bad_config():
    psweep = _lib_or_skip()
    def cfg(**kw):
        c = psweep.psweep_tsdf_config(0.1, 0.3, (psweep._i32 * 3)(8, 4, 8), 100.0, 3, 320, 256)
        for k, v in kw.items():
            setattr(c, k, v)
        return c
    for kw in ({"voxel_m": 0.0}, {"mu_m": -1.0}, {"mu_m": 13.0}, {"w_max": 0.5}, {"max_width": 4},
               {"blocks": (psweep._i32 * 3)(0, 4, 4)}, {"blocks": (psweep._i32 * 3)(1024, 1024, 1024)}):
        with pytest.raises(psweep.PsweepError) as ei:
            psweep.psweep_tsdf_create(cfg(**kw))
        assert ei.value.status == psweep.EINVAL
    ts = psweep.psweep_tsdf_create(cfg())
    assert psweep.psweep_tsdf_workspace_size(ts) >= 8 * 4 * 8 * 4096
    L = psweep.lib()
    # integrating before the workspace is bound and the map reset is a state error
    cam = psweep.psweep_camera(0.9, 100.0, 100.0, 160.0, 128.0, 320, 256)
    pose = psweep.psweep_pose()
    c3 = (psweep._d * 3)(0.0, 0.0, 0.0)
    pose.R[:] = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    assert L.psweep_tsdf_integrate(ts, cam, pose, c3, 1, 0, None) == psweep.ESTATE
    assert L.psweep_tsdf_extract(ts, None, None, None, None) == psweep.ESTATE
    # arguments are checked before the state: non-finite or non-rotation poses,
    # and centres whose block coordinates leave the 21-bit key range
    bad = psweep.psweep_pose()
    bad.R[:] = [float("nan")] + [0.0] * 8
    assert L.psweep_tsdf_integrate(ts, cam, bad, c3, 1, 0, None) == psweep.EINVAL
    bad.R[:] = [2.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    assert L.psweep_tsdf_integrate(ts, cam, bad, c3, 1, 0, None) == psweep.EINVAL
    pose.t[:] = [0.0, float("inf"), 0.0]
    assert L.psweep_tsdf_integrate(ts, cam, pose, c3, 1, 0, None) == psweep.EINVAL
    pose.t[:] = [0.0, 0.0, 0.0]
    far = (psweep._d * 3)(0.0, 0.0, 9.0e5)
    assert L.psweep_tsdf_integrate(ts, cam, pose, far, 1, 0, None) == psweep.EINVAL
    assert psweep.psweep_tsdf_last_error(ts)
    psweep.psweep_tsdf_destroy(ts)
