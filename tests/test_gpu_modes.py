"""GPU checks of the other forms of the sweep: half-precision staging against
its stated bound, the batched persistent launch and its HIP graph against the
per-level launches, and the soft-argmin forward and backward against the
FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Level, Settings
from tests.parity import to_np, wta_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    return PlaneSweep, frame_to_device


# ---------------------------------------------------------------------------
# FP16 / BF16 staging of warped samples
# ---------------------------------------------------------------------------
# Rounding a centred sample b - 128 in [-128, 128) moves it by at most eps
# (FP16: 2^-5, BF16: 2^-2).  A perturbation of |e| <= eps per sample moves the
# unit-normalised centred window vector by at most 2 eps / sigma_b, so
# |dZNCC| <= 2 eps / sigma_b and |d cost| <= eps / sigma_b, with sigma_b the
# window's standard deviation; best-K means keep the bound (1-Lipschitz).
# Checked per pixel on the winning plane with sigma_b >= sqrt(var_floor).
EPS = {"f16": 2.0 ** -5, "bf16": 2.0 ** -2}


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_within_bound(storage):
    PlaneSweep, frame_to_device = _gpu()
    fr = scenegen.random_small_frame(w=130, h=96, n_src=3, seed=11, f=80.0)
    lv = Level(n_fronto=14, near=1.0, far=25.0, n_ground=6, h_lo=-0.4, h_hi=0.4, window=9)
    st = Settings(levels=[lv], best_k=2)
    ps = PlaneSweep(st, 130, 96, 3, storage=storage)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, volume=True,
                             srcvol=True)
    s = wta_stats(g, ref, ref["volume"])
    print(storage, s)
    ov = ref["index"] >= 0
    both = ov & (g["index"] >= 0)
    # bound on the GPU's winning cost against the oracle's cost of that plane
    eps = EPS[storage]
    ys, xs = np.nonzero(both)
    worst = 0.0
    for y, x in zip(ys[::7], xs[::7]):
        k = g["index"][y, x]
        sig = []
        for sidx in range(3):
            w = oracle.window_cost(lv, st, fr.ref_cam, fr.ref, fr.src_cams[sidx], fr.srcs[sidx], fr.poses[sidx],
                                   int(k), int(x), int(y))
            if w["valid"]:
                sig.append(np.sqrt(w["s_bb"] / lv.window ** 2))
        bound = eps / min(sig) + 2e-4 if sig else np.inf
        err = abs(g["cost1"][y, x] - ref["volume"][y, x, k])
        worst = max(worst, err / bound)
        assert err <= bound, (y, x, k, err, bound)
    print(storage, "worst err / bound", worst)
    assert s["index_agree"] >= (0.99 if storage == "f16" else 0.9)


# ---------------------------------------------------------------------------
# batched persistent launch and HIP graph == per-level launches
# ---------------------------------------------------------------------------
def _two_level_settings(w, h):
    cw, ch = w // 2, h // 2
    return Settings(levels=[
        Level(n_fronto=16, near=0.5, far=30.0, n_ground=6, window=7, downsample=2),
        Level(n_fronto=12, near=15.0, far=60.0, n_ground=4, window=9, crop=((w - cw) // 2, (h - ch) // 2, cw, ch)),
    ], best_k=2)


@pytest.mark.parametrize("storage,n_src,ptile", [("f32", 4, (4, 4)), ("f16", 4, (4, 4)), ("bf16", 4, (4, 4)),
                                                 ("f32", 3, (4, 4)), ("f32", 3, (4, 8)), ("bf16", 3, (4, 8)),
                                                 ("f16", 4, (4, 8))])
def test_persistent_and_graph_match_grid(storage, n_src, ptile):
    """Bitwise equal maps from the persistent launch, the graph replays of
    both launches and the per-level grid launches (default 4 x 4 tiles), for
    every persistent kernel the batched benchmarks use (three and four
    sources; FP32, FP16 and BF16 staging) and for persistent tiles of 8 waves
    of 4 rows (the same per-pixel sums in the same order)."""
    PlaneSweep, frame_to_device = _gpu()
    sizes = [(256, 192), (200, 150), (160, 120)]
    frames = [scenegen._street_frame(w, h, 0.3516 * w, 7000 + i, 8000 + i, ss=1, extra_right=True)
              for i, (w, h) in enumerate(sizes)]
    frames = [dataclasses.replace(f, srcs=f.srcs[:n_src], src_cams=f.src_cams[:n_src], poses=f.poses[:n_src])
              for f in frames]
    assert all(len(f.srcs) == n_src for f in frames)
    st = _two_level_settings(*sizes[0])
    outs = {}
    for launch in ("grid", "persistent"):
        ps = PlaneSweep(st, 256, 192, n_src, max_frames=3, max_camera_sets=3, storage=storage, launch=launch)
        dev = []
        for i, (fr, (w, h)) in enumerate(zip(frames, sizes)):
            ps.set_cameras(i, fr.ref_cam, fr.src_cams, fr.poses)
            cw, ch = w // 2, h // 2
            ps.set_crop(i, (w - cw) // 2, (h - ch) // 2, cw, ch)
            d = frame_to_device(fr)
            d["camera_set"] = i
            dev.append(d)
        if launch == "persistent":
            for lv in range(len(st.levels)):
                ps.set_tile(lv, *ptile)
        o = [ps.alloc_outputs(camera_set=i) for i in range(3)]
        ps.run(dev, o)
        torch.cuda.synchronize()
        outs[launch] = [to_np(x["merged"]) for x in o]
        # graph replays, with eager work in between, give the same maps (the
        # grid launch's graph holds its per-job grids on two streams)
        o2 = [ps.alloc_outputs(camera_set=i) for i in range(3)]
        ps.capture_graph(dev, o2)
        for rep in range(3):
            for x in o2:
                x["merged"]["depth"].fill_(-1.0)
            ps.launch_graph()
            torch.cuda.synchronize()
            ps.run(dev, o)          # eager work between replays
            torch.cuda.synchronize()
            outs[f"{launch}_graph{rep}"] = [to_np(x["merged"]) for x in o2]
        ps.close()
    for key in ("persistent", "grid_graph0", "grid_graph1", "grid_graph2", "persistent_graph0",
                "persistent_graph1", "persistent_graph2"):
        for a, b in zip(outs["grid"], outs[key]):
            for name in a:
                assert np.array_equal(a[name], b[name], equal_nan=True), (key, name)
    # and the batched maps agree with the oracle on the first frame
    ref = oracle.run(frames[2], _two_level_settings(*sizes[2]))["merged"]
    g = outs["persistent"][2]
    assert (g["level"] == ref["level"]).mean() >= 0.99


# ---------------------------------------------------------------------------
# soft-argmin forward and backward
# ---------------------------------------------------------------------------
def _soft_case(n_ground=0):
    fr = scenegen.random_small_frame(w=64, h=48, n_src=2, seed=4, f=40.0)
    lv = Level(n_fronto=16, near=1.0, far=15.0, window=5, n_ground=n_ground, h_lo=-0.4, h_hi=0.4)
    st = Settings(levels=[lv], best_k=2, mode="soft", temperature=0.1, var_floor=1.0)
    return fr, lv, st


@pytest.mark.parametrize("n_ground", [0, 8])
def test_soft_forward_matches_oracle(n_ground):
    """rho_hat against the oracle, fronto planes alone and with ground
    planes (each standing for the inverse z-depth of the pixel's ray at it)."""
    PlaneSweep, frame_to_device = _gpu()
    fr, lv, st = _soft_case(n_ground)
    ps = PlaneSweep(st, 64, 48, 2)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    torch.cuda.synchronize()
    rh = out["soft_invdepth"].cpu().numpy()
    ps.close()
    rho, lse = oracle.soft_forward(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses)
    ok = np.isfinite(rho)
    assert ok.sum() > 500
    assert np.array_equal(ok, np.isfinite(rh))
    rel = np.abs(rh[ok] - rho[ok]) / np.maximum(np.abs(rho[ok]), 1e-2)
    if n_ground:
        # the ground planes take part: rho_hat differs from the fronto-only one
        rho_f, _ = oracle.soft_forward(*_soft_case(0)[1:], fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses)
        both = ok & np.isfinite(rho_f)
        assert (np.abs(rho_f[both] - rho[both]) > 1e-3 * np.abs(rho[both])).mean() > 0.2
    print("soft rho rel err max", rel.max(), "p99.9", np.quantile(rel, 0.999))
    assert np.quantile(rel, 0.999) <= 1e-4 and rel.max() <= 1e-3


BWD_CASES = [
    # (window, n_src, best_k, w, h, n_fronto, seed, var_floor[, n_ground])
    (5, 2, 2, 64, 48, 16, 4, 1.0),
    # fronto and ground planes
    (7, 2, 2, 80, 60, 10, 9, 1.0, 8),
    (7, 3, 2, 90, 70, 12, 5, 1.0),
    (9, 1, 1, 100, 60, 10, 6, 1.0),
    # a variance floor below 1/16: the image-gradient taps skip the
    # fixed-point LDS patch and go to the gradient images directly
    (7, 2, 2, 80, 60, 12, 7, 0.05),
    # four sources (one workgroup per CU: its patches fill the LDS)
    (9, 4, 2, 80, 60, 8, 8, 1.0),
    # ground planes with three and with four sources
    (5, 3, 2, 90, 70, 10, 10, 1.0, 6),
    (9, 4, 2, 80, 60, 8, 11, 1.0, 6),
]


@pytest.mark.parametrize("case", BWD_CASES,
                         ids=lambda c: f"w{c[0]}_S{c[1]}_K{c[2]}_{c[3]}x{c[4]}_vf{c[7]}_g{c[8] if len(c) > 8 else 0}")
def test_soft_backward_matches_oracle_gradient(case):
    """The GPU gradient of sum(g * rho_hat) against the oracle's FP64
    analytic gradient (itself pinned by central differences), for a dense
    random g over a rectangle spanning several tiles.  The forward is run
    on a temporary device copy of the frame, followed by allocations: the
    wrapper holds the reference image that the backward reads again."""
    PlaneSweep, frame_to_device = _gpu()
    win, S, K, W, H, nf, seed, vfloor = case[:8]
    ng = case[8] if len(case) > 8 else 0
    fr = scenegen.random_small_frame(w=W, h=H, n_src=S, seed=seed, f=0.62 * W)
    lv = Level(n_fronto=nf, near=1.0, far=15.0, window=win, n_ground=ng, h_lo=-0.4, h_hi=0.4)
    st = Settings(levels=[lv], best_k=K, mode="soft", temperature=0.1, var_floor=vfloor)
    ps = PlaneSweep(st, W, H, S)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    rng = np.random.default_rng(seed)
    filler = [torch.full((H, W), 7, dtype=torch.uint8, device="cuda") for _ in range(4)]
    g = np.zeros((H, W))
    x0, y0, w, h = 6, 5, W - 14, H - 11
    g[y0:y0 + h, x0:x0 + w] = rng.normal(size=(h, w))
    gs, gp = ps.soft_backward(torch.from_numpy(g.astype(np.float32)).cuda(), [s.shape for s in fr.srcs])
    torch.cuda.synchronize()
    del filler
    gs = [t.cpu().numpy() for t in gs]
    gp = gp.cpu().numpy()
    ps.close()
    ogs, ogp = oracle.soft_backward(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses,
                                    (x0, y0, w, h), g[y0:y0 + h, x0:x0 + w])
    rel_pose = np.linalg.norm(gp - ogp) / np.linalg.norm(ogp)
    rel_img = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(gs, ogs)) / sum(np.sum(b ** 2) for b in ogs))
    print(case, "pose", gp, ogp, "rel", rel_pose, "img rel", rel_img)
    assert np.linalg.norm(ogp) > 0
    assert rel_pose <= 1e-3 and rel_img <= 1e-3


@pytest.mark.parametrize("n_ground", [0, 8])
def test_soft_backward_pose_only_matches_full(n_ground):
    """Skipping the image gradients (NULL source-gradient pointers) leaves the
    pose gradient unchanged, with fronto planes alone and with ground planes."""
    PlaneSweep, frame_to_device = _gpu()
    fr, lv, st = _soft_case(n_ground)
    ps = PlaneSweep(st, 64, 48, 2)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    g = torch.from_numpy(np.random.default_rng(2).normal(size=(48, 64)).astype(np.float32)).cuda()
    shapes = [s.shape for s in fr.srcs]
    gs, gp = ps.soft_backward(g, shapes)
    gs0, gp0 = ps.soft_backward(g, shapes, image_grads=False)
    gs1, gp1 = ps.soft_backward(g, shapes, image_grads=[False, True])
    torch.cuda.synchronize()
    ps.close()
    assert gs0 == [None, None] and gs1[0] is None
    a, b, c = gp.cpu().numpy(), gp0.cpu().numpy(), gp1.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max() + 1e-12
    assert np.abs(a - c).max() <= 1e-9 * np.abs(a).max() + 1e-12
    assert torch.allclose(gs[1], gs1[1], rtol=1e-5, atol=1e-7)
