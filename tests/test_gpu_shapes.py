"""GPU parity at the benchmark workloads' own shapes.

* Two levels at 1024x768 (low 512x384, 96 planes, 7x7; crop 512x384 at full
  resolution, 64 planes, 9x9), in FP32, FP16 and BF16 staging: every
  (pixel, plane) cost of seeded pixels of both levels against the oracle's,
  within the staging bound; index mismatches only at near ties; the merged
  map at full size against the oracle's.
* The batched form (16 frames of 1280x960, 1024x768 and 640x480, 4 sources,
  192 + 64 planes per level, both levels, one persistent launch in a HIP
  graph) against the oracle on one frame of each size.
* The 1024x768 single-level workload on 5,000 seeded pixels.
* Soft-argmin forward on the 640x480 frame and its backward on the 64x48
  crop at (288, 216) against the full-size sources.

Staging bound (FP16 / BF16 storage of a centred sample b - 128): rounding
moves a sample by at most eps (FP16 2^-5, BF16 2^-2), which moves the
unit-normalised centred window vector by at most 2 eps / sigma_b, so ZNCC
by at most 2 eps / sigma_b and the cost (1 - ZNCC) / 2 by at most
eps / sigma_b, sigma_b the standard deviation of the window's samples; the
mean of the best K source costs is 1-Lipschitz in the largest of them, so
the aggregated cost moves by at most max_s eps / sigma_b,s.  On top of it
the FP32 arithmetic of the window sums (FP32_COST)."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.parity import DEPTH_REL, INDEX_AGREE, assert_wta_parity, to_np, wta_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = {"f32": 0.0, "f16": 2.0 ** -5, "bf16": 2.0 ** -2}
# FP32 window sums: cost error measured at most a few 1e-5 on textured
# windows; the allowance also covers the weakest windows the variance floor
# lets through
FP32_COST = 2e-4


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    return PlaneSweep, frame_to_device


def _interior_sample(rng, w, h, hw, n):
    return np.stack([rng.integers(hw, w - hw, n), rng.integers(hw, h - hw, n)], 1).astype(np.int32)


def cost_bounds(ref, eps, var_floor=1.0):
    """Per (pixel, plane): the bound eps / min_s sigma_b,s + FP32_COST over the
    sources whose windows are usable, and whether the pair is marginal: a
    source window whose deviation lies within eps (+ FP32 slack) of the
    variance floor's, where rounding can make it usable in one form and not
    in the other and so change which sources the best-K mean takes."""
    sig = ref["srcsig"]                                                # [n, P, S], NaN: a sample unusable
    usable = np.isfinite(ref["srcvol"])                                # [n, P, S]
    with np.errstate(invalid="ignore", divide="ignore"):
        smin = np.nanmin(np.where(usable, sig, np.nan), axis=2)
        bound = eps / smin + FP32_COST
    bound = np.where(np.isfinite(bound), bound, FP32_COST)
    near = np.isfinite(sig) & (np.abs(sig - np.sqrt(var_floor)) <= eps + 1e-3)
    return bound, near.any(axis=2)


def check_costs(gvol, ref, eps, pix, label):
    """Every (pixel, plane) cost of the sampled pixels: GPU volume [P, h, w]
    against the oracle's volume, within the staging bound; usable in both
    forms except at marginal pairs."""
    g = gvol[:, pix[:, 1], pix[:, 0]].T.astype(np.float64)            # [n, P]
    o = ref["volume"]                                                  # [n, P], NaN = unusable
    ov, gv = np.isfinite(o), np.isfinite(g)
    bound, marginal = cost_bounds(ref, eps)
    both = ov & gv & ~marginal
    err = np.abs(g - o)
    flips = (ov != gv)
    ratio = np.where(both, err / bound, 0.0)
    print(f"{label}: pairs {both.sum()} (+{(marginal & ov & gv).sum()} marginal), validity flips "
          f"{flips.sum()} (marginal {(flips & marginal).sum()}), cost err max {err[both].max():.2e} "
          f"p99.9 {np.quantile(err[both], 0.999):.2e}, worst err/bound {ratio.max():.3f}")
    assert both.sum() > 0.3 * o.size
    assert np.all(err[both] <= bound[both]), label
    assert not np.any(flips & ~marginal), label
    assert marginal.sum() <= 0.02 * o.size, label
    return bound, marginal


def check_index(gidx, ref, bound, marginal, label):
    """Winning planes: identical, or a near tie within the two planes' bounds
    (the oracle's own costs of the two planes); pixels with a marginal pair
    on either plane are counted apart."""
    o = ref["volume"]
    oi = ref["index"]
    ok = oi >= 0
    gi = gidx
    n = np.arange(len(oi))
    same = ok & (gi == oi)
    mism = ok & (gi != oi) & (gi >= 0)
    gs = np.where(gi >= 0, gi, 0)
    os_ = np.where(oi >= 0, oi, 0)
    marg = marginal[n, gs] | marginal[n, os_]
    chk = mism & ~marg
    gap = o[n[chk], gi[chk]] - o[n[chk], oi[chk]]
    lim = bound[n[chk], gi[chk]] + bound[n[chk], oi[chk]]
    agree = same.sum() / ok.sum()
    print(f"{label}: index agreement {agree:.5f} ({chk.sum()} near ties, largest gap "
          f"{gap.max() if gap.size else 0:.2e}; {(mism & marg).sum()} at marginal pairs), "
          f"gpu-invalid/oracle-valid {(ok & (gi < 0)).sum()}")
    assert np.all(gap <= lim), label
    assert (ok & (gi < 0) & ~marginal.any(axis=1)).sum() == 0, label
    return same, agree


# ---------------------------------------------------------------------------
# two levels at 1024 x 768, every staging precision
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c3():
    wl = scenegen.workload("C3")
    fr, st = wl.frames[0], wl.settings
    full = oracle.run(fr, st)            # both levels at every pixel, then the merge
    return fr, st, full


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_two_levels_1024x768_every_cost(c3, storage):
    PlaneSweep, frame_to_device = _gpu()
    fr, st, full = c3
    ps = PlaneSweep(st, 1024, 768, 3, storage=storage)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs(level_maps=True)
    out["cost_volume"] = ps.alloc_cost_volumes()
    ps.run([frame_to_device(fr)], [out])
    torch.cuda.synchronize()
    gl = [to_np(m) for m in out["levels"]]
    vols = [v.cpu().numpy() for v in out["cost_volume"]]
    gm = to_np(out["merged"])
    ps.close()
    rng = np.random.default_rng(2024)
    eps = EPS[storage]
    for l, lv in enumerate(st.levels):
        rc, rimg, scs, simgs = oracle.level_inputs(fr, lv)
        h, w = rimg.shape
        pix = _interior_sample(rng, w, h, lv.window // 2, 2500)
        ref = oracle.sweep_level(lv, st, rc, rimg, scs, simgs, fr.poses, pixels=pix, volume=True, srcvol=True,
                                 srcsig=True)
        label = f"{storage} level {l}"
        bound, marginal = check_costs(vols[l], ref, eps, pix, label)
        gidx = gl[l]["index"][pix[:, 1], pix[:, 0]]
        same, agree = check_index(gidx, ref, bound, marginal, label)
        # the level map's winning cost is the volume's entry of its plane
        gi = np.where(gidx >= 0, gidx, 0)
        assert np.array_equal(gl[l]["cost1"][pix[:, 1], pix[:, 0]][gidx >= 0],
                              vols[l][gi, pix[:, 1], pix[:, 0]][gidx >= 0])
        if storage == "f32":
            assert agree >= INDEX_AGREE, label
    # merged map at full size against the oracle's merge of full levels
    rm = full["merged"]
    ov = rm["level"] != 255
    lev_agree = (gm["level"][ov] == rm["level"][ov]).mean()
    same = ov & (gm["level"] == rm["level"]) & (gm["index"] == rm["index"])
    rel = np.abs(gm["depth"][same] - rm["depth"][same]) / rm["depth"][same]
    p50, p999, mx = (float(v) for v in (np.quantile(rel, 0.5), np.quantile(rel, 0.999), rel.max()))
    print(f"{storage} merged 1024x768: level agreement {lev_agree:.5f}, index agreement "
          f"{same.sum() / ov.sum():.5f}, depth rel err p50 {p50:.2e} p99.9 {p999:.2e} max {mx:.2e}")
    assert lev_agree >= (INDEX_AGREE if storage == "f32" else 0.995)
    if storage == "f32":
        assert same.sum() / ov.sum() >= INDEX_AGREE and p999 <= DEPTH_REL


# ---------------------------------------------------------------------------
# the 1024 x 768 single-level workload on 5,000 pixels
# ---------------------------------------------------------------------------
def test_one_level_1024x768_5000_pixels():
    PlaneSweep, frame_to_device = _gpu()
    wl = scenegen.workload("C2")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, 1024, 768, 3)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    rng = np.random.default_rng(321)
    pix = _interior_sample(rng, 1024, 768, 4, 5000)
    ref = oracle.sweep_level(st.levels[0], st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses,
                             pixels=pix, volume=True)
    gs = {k: v[pix[:, 1], pix[:, 0]] for k, v in g.items()}
    s = wta_stats(gs, ref, ref["volume"])
    print("1024x768 on 5000 pixels", s)
    assert s["n_oracle_valid"] >= 3000
    assert_wta_parity(s)


# ---------------------------------------------------------------------------
# batched form: 16 frames of three sizes in one persistent launch (graph)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_batched_persistent_graph_against_oracle(storage):
    PlaneSweep, frame_to_device = _gpu()
    wl = scenegen.workload("C5")
    frames = wl.frames
    W, H = scenegen.C5_SIZES[0]
    st = scenegen.c5_settings(W, H)
    ps = PlaneSweep(st, W, H, 4, max_frames=len(frames), max_camera_sets=len(frames), storage=storage,
                    launch="persistent")
    dev = []
    for i, fr in enumerate(frames):
        ps.set_cameras(i, fr.ref_cam, fr.src_cams, fr.poses)
        w, h = fr.ref_cam.width, fr.ref_cam.height
        ps.set_crop(i, (w - w // 2) // 2, (h - h // 2) // 2, w // 2, h // 2)
        d = frame_to_device(fr)
        d["camera_set"] = i
        dev.append(d)
    outs = [ps.alloc_outputs(camera_set=i, level_maps=True) for i in range(len(frames))]
    ps.capture_graph(dev, outs)
    ps.launch_graph()
    ps.launch_graph()
    torch.cuda.synchronize()
    got = [[to_np(m) for m in o["levels"]] for o in outs]
    merged = [to_np(o["merged"]) for o in outs]
    ps.close()
    rng = np.random.default_rng(55)
    eps = EPS[storage]
    for f in (0, 1, 2):                    # one frame of each size
        fr = frames[f]
        w, h = fr.ref_cam.width, fr.ref_cam.height
        st_f = scenegen.c5_settings(w, h)
        for l, lv in enumerate(st_f.levels):
            rc, rimg, scs, simgs = oracle.level_inputs(fr, lv)
            lh, lw = rimg.shape
            pix = _interior_sample(rng, lw, lh, lv.window // 2, 600)
            ref = oracle.sweep_level(lv, st_f, rc, rimg, scs, simgs, fr.poses, pixels=pix, volume=True,
                                     srcvol=True, srcsig=True)
            g = got[f][l]
            gi = g["index"][pix[:, 1], pix[:, 0]]
            label = f"batched {storage} frame {f} ({w}x{h}) level {l}"
            # the GPU's winning cost against the oracle's cost of that plane
            n = np.arange(len(gi))
            bnd, marginal = cost_bounds(ref, eps)
            gs = np.where(gi >= 0, gi, 0)
            v = (gi >= 0) & (ref["index"] >= 0) & ~marginal[n, gs]
            c1 = g["cost1"][pix[:, 1], pix[:, 0]]
            err = np.abs(c1[v] - ref["volume"][n[v], gi[v]])
            assert np.all(err <= bnd[n[v], gi[v]]), label
            same, agree = check_index(gi, ref, bnd, marginal, label)
            if storage == "f32":
                assert agree >= 0.995, label
        assert (merged[f]["level"] != 255).mean() > 0.4


# ---------------------------------------------------------------------------
# soft-argmin at 640 x 480
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c4_run():
    PlaneSweep, frame_to_device = _gpu()
    wl = scenegen.workload("C4")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, 640, 480, 2)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    yield fr, st, ps, out
    ps.close()


def test_soft_forward_640x480_sampled(c4_run):
    fr, st, ps, out = c4_run
    torch.cuda.synchronize()
    rh = out["soft_invdepth"].cpu().numpy()
    rng = np.random.default_rng(77)
    pix = _interior_sample(rng, 640, 480, 3, 6000)
    rho, lse = oracle.soft_forward(st.levels[0], st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, pixels=pix)
    g = rh[pix[:, 1], pix[:, 0]]
    ok = np.isfinite(rho)
    assert ok.sum() >= 2000
    assert np.array_equal(ok, np.isfinite(g))
    rel = np.abs(g[ok] - rho[ok]) / rho[ok]
    print(f"soft rho 640x480 on {ok.sum()} pixels: rel err p99.9 {np.quantile(rel, 0.999):.2e} max {rel.max():.2e}")
    assert np.quantile(rel, 0.999) <= 1e-4


def test_soft_backward_crop_of_640x480(c4_run):
    """Gradient of sum(g * rho_hat) over the 64x48 crop at (288, 216) with
    respect to both full 640x480 source images and both poses."""
    fr, st, ps, out = c4_run
    rect = (288, 216, 64, 48)
    x0, y0, w, h = rect
    g = np.zeros((480, 640))
    g[y0:y0 + h, x0:x0 + w] = np.random.default_rng(0).normal(size=(h, w))
    gs, gp = ps.soft_backward(torch.from_numpy(g.astype(np.float32)).cuda(), [s.shape for s in fr.srcs])
    torch.cuda.synchronize()
    gs = [t.cpu().numpy() for t in gs]
    gp = gp.cpu().numpy()
    ogs, ogp = oracle.soft_backward(st.levels[0], st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, rect,
                                    g[y0:y0 + h, x0:x0 + w])
    rel_pose = np.linalg.norm(gp - ogp) / np.linalg.norm(ogp)
    rel_img = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(gs, ogs)) / sum(np.sum(b ** 2) for b in ogs))
    print(f"backward on the 64x48 crop: pose rel l2 {rel_pose:.2e}, image rel l2 {rel_img:.2e}")
    assert np.linalg.norm(ogp) > 0 and sum(np.sum(b ** 2) for b in ogs) > 0
    assert rel_pose <= 1e-3 and rel_img <= 1e-3
