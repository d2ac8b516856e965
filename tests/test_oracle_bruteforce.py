"""Brute-force pin of the whole single-level sweep on tiny inputs.

An independent NumPy/SciPy enumeration (camera rays by numerical inversion of
the polar projection formula, bilinear sampling by scipy.ndimage
map_coordinates, ZNCC by numpy.corrcoef, subpixel vertex by numpy.polyfit)
must reproduce the oracle's cost volume, winner, costs, subpixel offset and
range on every pixel."""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates
from scipy.optimize import brentq

import oracle
import scenegen
from scenegen import Level, Settings


def _rays(cam):
    H, W = cam.height, cam.width
    R = np.zeros((H, W, 3))
    for j in range(H):
        for i in range(W):
            x, y = (i - cam.cx) / cam.fx, (j - cam.cy) / cam.fy
            m = math.hypot(x, y)
            if m == 0:
                R[j, i] = (0, 0, 1)
                continue
            if cam.xi == 0:
                th = math.atan(m)
            else:
                th = brentq(lambda t: math.sin(t) / (math.cos(t) + cam.xi) - m, 0.0,
                            math.acos(-min(cam.xi, 1.0)) - 1e-12, xtol=1e-15)
            R[j, i] = (math.sin(th) * x / m, math.sin(th) * y / m, math.cos(th))
    return R


def _project_polar(cam, X):
    nrm = np.linalg.norm(X, axis=-1)
    cos_t = X[..., 2] / nrm
    sin_t = np.linalg.norm(X[..., :2], axis=-1) / nrm
    ph = np.arctan2(X[..., 1], X[..., 0])
    den = cos_t + cam.xi
    ok = den > 1e-12
    m = np.where(ok, sin_t / np.where(ok, den, 1.0), 0.0)
    return cam.cx + cam.fx * m * np.cos(ph), cam.cy + cam.fy * m * np.sin(ph), ok


def _planes(level, st):
    out = []
    for k in range(level.n_fronto):
        rho = 1 / level.far + k * (1 / level.near - 1 / level.far) / (level.n_fronto - 1)
        out.append((np.array([0, 0, 1.0]), 1 / rho, 0, rho))
    for j in range(level.n_ground):
        h = level.h_lo + j * (level.h_hi - level.h_lo) / (level.n_ground - 1)
        out.append((np.asarray(st.ground_n, float), st.ground_d - h, 1, h))
    return out


def brute(frame, level, st):
    cam = frame.ref_cam
    H, W = cam.height, cam.width
    rays = _rays(cam)
    ref = frame.ref.astype(np.float64)
    hw, N = level.window // 2, level.window ** 2
    planes = _planes(level, st)
    P, S = len(planes), len(frame.srcs)
    vol = np.full((H, W, P), np.nan)
    for k, (n, d, fam, prm) in enumerate(planes):
        t = rays @ n
        hit = t > 0
        lam = np.where(hit, d / np.where(hit, t, 1.0), 0.0)
        X = rays * lam[..., None]
        costs = np.full((S, H, W), np.nan)
        for s in range(S):
            ps, sc = frame.poses[s], frame.src_cams[s]
            Xs = X @ ps.R.T + ps.t
            u, v, ok = _project_polar(sc, Xs)
            ok &= hit & (u >= 0) & (u <= sc.width - 1) & (v >= 0) & (v <= sc.height - 1)
            b = map_coordinates(frame.srcs[s].astype(np.float64), [np.where(ok, v, 0), np.where(ok, u, 0)],
                                order=1, mode="nearest")
            for j in range(hw, H - hw):
                for i in range(hw, W - hw):
                    win = (slice(j - hw, j + hw + 1), slice(i - hw, i + hw + 1))
                    if not ok[win].all():
                        continue
                    a_w, b_w = ref[win].ravel(), b[win].ravel()
                    if a_w.var() * N <= N * st.var_floor or b_w.var() * N <= N * st.var_floor:
                        continue
                    z = np.clip(np.corrcoef(a_w, b_w)[0, 1], -1, 1)
                    costs[s, j, i] = (1 - z) / 2
        srt = np.sort(np.where(np.isnan(costs), np.inf, costs), axis=0)
        nvalid = (~np.isnan(costs)).sum(axis=0)
        kk = np.minimum(st.best_k, nvalid)
        acc = np.zeros((H, W))
        for q in range(min(st.best_k, S)):
            acc += np.where(q < kk, srt[q], 0.0)
        vol[..., k] = np.where(nvalid > 0, acc / np.maximum(kk, 1), np.nan)
    return vol, rays, planes


def _compare(frame, level, st):
    vol, rays, planes = brute(frame, level, st)
    res = oracle.sweep_level(level, st, frame.ref_cam, frame.ref, frame.src_cams, frame.srcs, frame.poses,
                             volume=True)
    both_nan = np.isnan(vol) & np.isnan(res["volume"])
    assert np.array_equal(np.isnan(vol), np.isnan(res["volume"]))
    assert np.nanmax(np.abs(np.where(both_nan, 0, vol - res["volume"]))) < 1e-10
    H, W, P = vol.shape
    F = level.n_fronto
    filled = np.where(np.isnan(vol), np.inf, vol)
    kbest = np.argmin(filled, axis=-1)
    any_valid = np.isfinite(filled).any(axis=-1)
    exp_idx = np.where(any_valid, kbest, -1)
    assert np.array_equal(exp_idx, res["index"])
    n_par = 0
    for j in range(H):
        for i in range(W):
            k = exp_idx[j, i]
            if k < 0:
                assert np.isnan(res["depth"][j, i])
                continue
            c = filled[j, i]
            srt = np.sort(np.delete(c, k))
            assert abs(res["cost1"][j, i] - c[k]) < 1e-12
            want2, got2 = (srt[0] if srt.size else np.inf), res["cost2"][j, i]
            assert (np.isinf(want2) and np.isinf(got2)) or abs(got2 - want2) < 1e-12
            lo, hi = (0, F - 1) if k < F else (F, P - 1)
            delta = 0.0
            if lo <= k - 1 and k + 1 <= hi and np.isfinite(c[k - 1]) and np.isfinite(c[k + 1]):
                a2, b2, _ = np.polyfit([-1.0, 0.0, 1.0], [c[k - 1], c[k], c[k + 1]], 2)
                if a2 > 1e-15:
                    delta = float(np.clip(-b2 / (2 * a2), -0.5, 0.5))
                    n_par += 1
            assert abs(res["delta"][j, i] - delta) < 1e-8
            n, d, fam, prm = planes[k]
            step = planes[1][3] - planes[0][3] if fam == 0 else planes[F + 1][3] - planes[F][3]
            prm_ref = prm + delta * step
            r = rays[j, i]
            lam = 1 / (prm_ref * r[2]) if fam == 0 else (st.ground_d - prm_ref) / (n @ r)
            assert abs(res["depth"][j, i] - lam) < 1e-8 * max(1.0, lam)
            assert abs(res["z"][j, i] - lam * r[2]) < 1e-8 * max(1.0, lam)
    assert n_par > 20


@pytest.mark.parametrize("xi,n_src,k", [(0.9, 2, 2), (0.9, 3, 1), (0.0, 2, 2)])
def test_bruteforce_tiny(xi, n_src, k):
    fr = scenegen.random_small_frame(w=40, h=32, n_src=n_src, seed=int(10 * xi) + n_src, f=28.0 if xi else 20.0,
                                     xi=xi)
    level = Level(n_fronto=6, near=1.0, far=15.0, n_ground=4, h_lo=-0.3, h_hi=0.3, window=5)
    st = Settings(levels=[level], best_k=k, var_floor=1.0)
    _compare(fr, level, st)
