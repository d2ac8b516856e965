"""GPU depth-map filtering against the oracle's filter, on the same input
maps (the GPU sweep's own output, so both sides filter identical values)."""
import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _near_ratio(m, ratio):
    """Pixels whose cost2 / cost1 sits on the ratio threshold (to FP32
    rounding); invalid pixels (costs +inf) are not near it."""
    c1, c2 = m["cost1"].astype(np.float64), m["cost2"].astype(np.float64)
    fin = np.isfinite(c1) & np.isfinite(c2)
    near = np.zeros(c1.shape, bool)
    near[fin] = np.abs(c2[fin] - ratio * c1[fin]) <= 1e-6 * np.abs(c2[fin])
    return near


@pytest.mark.parametrize("window,ratio", [(5, 1.05), (3, 1.2), (7, 1.0)])
def test_filter_matches_oracle(window, ratio):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    wl = scenegen.workload("C1")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, 320, 256, 1)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    d, c = ps.filter(out["merged"], ratio_min=ratio, window=window)
    torch.cuda.synchronize()
    m = {k: v.cpu().numpy() for k, v in out["merged"].items()}
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    ps.close()
    od, oc = oracle.depth_filter(fr.ref_cam, st.ground_n, m["depth"].astype(np.float64),
                                 m["cost1"].astype(np.float64), m["cost2"].astype(np.float64),
                                 ratio_min=ratio, window=window)
    # decisions can differ only where an FP32 comparison sits on its threshold
    near = _near_ratio(m, ratio)
    diff = (gc != oc) & ~near
    print("codes", np.bincount(gc.ravel(), minlength=256)[[0, 1, 2, 3, 255]], "mismatch", diff.sum())
    assert diff.sum() == 0
    keep = (gc == 0) & (oc == 0)
    assert np.array_equal(gd[keep], od[keep].astype(np.float32))
    assert np.all(np.isnan(gd[gc != 0]))


def test_mask_boxes_after_filter():
    """Detected boxes (some partly outside the image, overlapping, empty, and
    more than one launch holds) masked out of the filtered map, against the
    oracle's filter and mask."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    wl = scenegen.workload("C1")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, 320, 256, 1)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    d, c = ps.filter(out["merged"])
    rng = np.random.default_rng(5)
    boxes = [(-20, -10, 40, 30), (300, 200, 400, 300), (100, 100, 100, 140), (50, 60, 120, 90), (70, 70, 130, 160)]
    boxes += [tuple(int(v) for v in (x, y, x + rng.integers(1, 30), y + rng.integers(1, 30)))
              for x, y in zip(rng.integers(-10, 320, 80), rng.integers(-10, 256, 80))]
    ps.mask_boxes(d, boxes, code=c)
    torch.cuda.synchronize()
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    m = {k: v.cpu().numpy() for k, v in out["merged"].items()}
    ps.close()
    od, oc = oracle.depth_filter(fr.ref_cam, st.ground_n, m["depth"].astype(np.float64),
                                 m["cost1"].astype(np.float64), m["cost2"].astype(np.float64))
    od, oc = oracle.mask_boxes(od, boxes, oc)
    near = _near_ratio(m, 1.05)
    assert ((gc != oc) & ~near).sum() == 0
    assert np.all(gc[oc == 4] == 4)
    keep = (gc == 0) & (oc == 0)
    assert np.array_equal(gd[keep], od[keep].astype(np.float32))
    assert np.all(np.isnan(gd[gc != 0]))

def test_filter_c2_full_map():
    """The filter on the full C2 map (1024x768, three sources, both plane
    families) against the oracle's filter of the same maps."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    wl = scenegen.workload("C2")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, 1024, 768, 3)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    d, c = ps.filter(out["merged"])
    torch.cuda.synchronize()
    m = {k: v.cpu().numpy() for k, v in out["merged"].items()}
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    ps.close()
    od, oc = oracle.depth_filter(fr.ref_cam, st.ground_n, m["depth"].astype(np.float64),
                                 m["cost1"].astype(np.float64), m["cost2"].astype(np.float64))
    near = _near_ratio(m, 1.05)
    diff = (gc != oc) & ~near
    counts = np.bincount(gc.ravel(), minlength=256)[[0, 1, 2, 3, 255]]
    print("codes", counts, "mismatch", diff.sum())
    assert diff.sum() == 0
    assert counts[0] > 0.1 * gc.size and counts[1] > 0 and counts[3] > 0   # every filter acts
    keep = (gc == 0) & (oc == 0)
    assert np.array_equal(gd[keep], od[keep].astype(np.float32))
    assert np.all(np.isnan(gd[gc != 0]))
