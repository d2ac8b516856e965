"""GPU sweep of float frame images (four-float quad texels, FP64 reference
statistics) against the FP64 oracle, which takes the same float values."""
import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Level, Settings
from tests.parity import assert_wta_parity, to_np, wta_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep
    return PlaneSweep


def _float_frame(fr, seed):
    """The frame's images as float32 with a fractional offset per pixel (not
    integers any more), clipped to [0, 255]."""
    rng = np.random.default_rng(seed)
    f = lambda a: np.clip(a.astype(np.float32) + rng.uniform(-0.5, 0.5, a.shape).astype(np.float32), 0, 255)
    return scenegen.Frame(ref=f(fr.ref), srcs=[f(s) for s in fr.srcs], ref_cam=fr.ref_cam,
                          src_cams=fr.src_cams, poses=fr.poses, gt_range=fr.gt_range, gt_z=fr.gt_z)


def _dev(fr):
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return {"ref": up(fr.ref), "srcs": [up(s) for s in fr.srcs], "camera_set": 0}


CASES = [
    # (w, h, n_src, window, n_fronto, n_ground, best_k, seed)
    (96, 72, 1, 3, 12, 0, 1, 21),
    (100, 70, 2, 7, 10, 6, 2, 22),
    (130, 75, 3, 9, 12, 8, 2, 23),
    (90, 66, 4, 15, 8, 4, 3, 24),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}_S{c[2]}_w{c[3]}")
def test_float_images_match_oracle(case):
    PlaneSweep = _gpu()
    w, h, S, win, nf, ng, k, seed = case
    fr = _float_frame(scenegen.random_small_frame(w=w, h=h, n_src=S, seed=seed, f=0.62 * w), seed)
    lv = Level(n_fronto=nf, near=1.0, far=25.0, n_ground=ng, h_lo=-0.4, h_hi=0.4, window=win)
    st = Settings(levels=[lv], best_k=k)
    ps = PlaneSweep(st, w, h, S, image_format="f32")
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    d = _dev(fr)
    ps.run([d], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, volume=True)
    s = wta_stats(g, ref, ref["volume"])
    print(case, s)
    assert_wta_parity(s)


def test_integer_valued_float_images_match_u8_path():
    """Float images holding the 8-bit values give the 8-bit path's maps: the
    warped samples are bitwise equal, the reference statistics agree to an
    ulp."""
    PlaneSweep = _gpu()
    fr = scenegen.random_small_frame(w=150, h=90, n_src=3, seed=8, f=90.0)
    lv = Level(n_fronto=10, near=1.0, far=25.0, n_ground=6, h_lo=-0.4, h_hi=0.4, window=9)
    st = Settings(levels=[lv], best_k=2)
    maps = {}
    for fmt, dt in (("u8", torch.uint8), ("f32", torch.float32)):
        ps = PlaneSweep(st, 150, 90, 3, image_format=fmt)
        ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
        out = ps.alloc_outputs()
        d = _dev(fr)
        d = {"ref": d["ref"].to(dt), "srcs": [x.to(dt) for x in d["srcs"]], "camera_set": 0}
        ps.run([d], [out])
        torch.cuda.synchronize()
        maps[fmt] = to_np(out["merged"])
        ps.close()
    a, b = maps["u8"], maps["f32"]
    same = a["index"] == b["index"]
    assert same.mean() >= 0.9999
    both = same & (a["index"] >= 0)
    assert np.abs(a["cost1"][both] - b["cost1"][both]).max() <= 1e-5


@pytest.mark.parametrize("n_ground", [0, 6])
def test_float_images_soft_forward_and_backward(n_ground):
    """Soft forward and backward on float images, with fronto planes alone
    and with ground planes beside them."""
    PlaneSweep = _gpu()
    W, H, S = 64, 48, 2
    fr = _float_frame(scenegen.random_small_frame(w=W, h=H, n_src=S, seed=4, f=40.0), 5)
    lv = Level(n_fronto=16, near=1.0, far=15.0, window=5, n_ground=n_ground, h_lo=-0.4, h_hi=0.4)
    st = Settings(levels=[lv], best_k=2, mode="soft", temperature=0.1, var_floor=1.0)
    ps = PlaneSweep(st, W, H, S, image_format="f32")
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([_dev(fr)], [out])
    rng = np.random.default_rng(9)
    g = np.zeros((H, W))
    x0, y0, w, h = 6, 5, W - 14, H - 11
    g[y0:y0 + h, x0:x0 + w] = rng.normal(size=(h, w))
    gs, gp = ps.soft_backward(torch.from_numpy(g.astype(np.float32)).cuda(), [s.shape for s in fr.srcs])
    torch.cuda.synchronize()
    rh = out["soft_invdepth"].cpu().numpy()
    gs = [t.cpu().numpy() for t in gs]
    gp = gp.cpu().numpy()
    ps.close()
    rho, _ = oracle.soft_forward(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses)
    ok = np.isfinite(rho)
    assert ok.sum() > 500 and np.array_equal(ok, np.isfinite(rh))
    assert np.quantile(np.abs(rh[ok] - rho[ok]) / rho[ok], 0.999) <= 1e-4
    ogs, ogp = oracle.soft_backward(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses,
                                    (x0, y0, w, h), g[y0:y0 + h, x0:x0 + w])
    rel_pose = np.linalg.norm(gp - ogp) / np.linalg.norm(ogp)
    rel_img = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(gs, ogs)) / sum(np.sum(b ** 2) for b in ogs))
    print("float images, ground planes", n_ground, ": pose rel", rel_pose, "img rel", rel_img)
    assert rel_pose <= 1e-3 and rel_img <= 1e-3


@pytest.mark.parametrize("n_ground", [0, 6])
def test_autograd_float_sources_get_exact_gradients(n_ground):
    """Through torch.autograd: float sources of an f32-image sweep receive the
    library's backward gradient, and the pose gradient matches it too (fronto
    planes alone, and with ground planes)."""
    _gpu()
    from paper_1809_06132_amd.autograd import SoftDepthSweep
    W, H, S = 64, 48, 2
    fr = _float_frame(scenegen.random_small_frame(w=W, h=H, n_src=S, seed=4, f=40.0), 6)
    lv = Level(n_fronto=16, near=1.0, far=15.0, window=5, n_ground=n_ground, h_lo=-0.4, h_hi=0.4)
    st = Settings(levels=[lv], best_k=2, mode="soft", temperature=0.1, var_floor=1.0)
    sw = SoftDepthSweep(st, fr.ref_cam, fr.src_cams, fr.poses, image_format="f32")
    d = _dev(fr)
    srcs = [s.clone().requires_grad_(True) for s in d["srcs"]]
    xi = torch.zeros((S, 6), dtype=torch.float64, requires_grad=True)
    rho, _ = sw(d["ref"], srcs, xi)
    g = torch.randn(rho.shape, device=rho.device, generator=torch.Generator(device=rho.device).manual_seed(1))
    loss = (torch.nan_to_num(rho) * g).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert all(s.grad is not None and torch.isfinite(s.grad).all() for s in srcs)
    ogs, ogp = oracle.soft_backward(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses,
                                    (0, 0, W, H), np.where(np.isfinite(rho.detach().cpu().numpy()),
                                                           g.cpu().numpy(), 0.0))
    gp = xi.grad.cpu().numpy()
    assert np.linalg.norm(gp - ogp) / np.linalg.norm(ogp) <= 1e-3
    num = sum(float(((s.grad.cpu().numpy() - o) ** 2).sum()) for s, o in zip(srcs, ogs))
    den = sum(float((o ** 2).sum()) for o in ogs)
    assert (num / den) ** 0.5 <= 1e-3
    sw.close()
