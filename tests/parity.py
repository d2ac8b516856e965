"""Parity statistics between the GPU maps and the FP64 oracle's maps.

The bar (winner-take-all, FP32 GPU arithmetic):
  * winning plane identical on >= 99.9% of the oracle-valid pixels, and every
    other oracle-valid pixel a near tie: the oracle's own cost of the GPU's
    plane within NEAR_TIE of the oracle's best cost (several answers are then
    correct to FP32 precision);
  * range within 1e-3 relative on >= 99.9% of the index-matching pixels;
  * GPU-valid / oracle-invalid pixels counted separately (only possible where
    a window sits exactly on a validity boundary).
"""
from __future__ import annotations

import numpy as np

INDEX_AGREE = 0.999
DEPTH_REL = 1e-3
DEPTH_QUANTILE = 0.999
NEAR_TIE = 2e-4
COST_ABS = 2e-4


def to_np(maps: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in maps.items()}


def wta_stats(gpu: dict, ref: dict, volume=None) -> dict:
    gi = np.asarray(gpu["index"]).ravel()
    ri = np.asarray(ref["index"]).ravel()
    ov, gv = ri >= 0, gi >= 0
    st = {"n_oracle_valid": int(ov.sum()), "n_gpu_valid": int(gv.sum()),
          "gpu_valid_oracle_invalid": int((gv & ~ov).sum()),
          "oracle_valid_gpu_invalid": int((ov & ~gv).sum())}
    same = ov & (gi == ri)
    st["index_agree"] = float(same.sum() / max(ov.sum(), 1))
    gd, rd = np.asarray(gpu["depth"]).ravel(), np.asarray(ref["depth"]).ravel()
    rel = np.abs(gd[same] - rd[same]) / np.abs(rd[same])
    st["depth_rel_max"] = float(rel.max()) if rel.size else 0.0
    st["depth_rel_q"] = float(np.quantile(rel, DEPTH_QUANTILE)) if rel.size else 0.0
    st["depth_rel_frac_ok"] = float((rel <= DEPTH_REL).mean()) if rel.size else 1.0
    c1g, c1r = np.asarray(gpu["cost1"]).ravel(), np.asarray(ref["cost1"]).ravel()
    st["cost1_abs_max"] = float(np.abs(c1g[same] - c1r[same]).max()) if same.any() else 0.0
    if volume is not None:
        vol = np.asarray(volume).reshape(ri.size, -1)
        mism = np.where(ov & gv & (gi != ri))[0]
        gap = [vol[e, gi[e]] - vol[e, ri[e]] for e in mism]
        st["mismatch_cost_gap_max"] = float(np.nanmax(gap)) if gap else 0.0
        st["n_mismatch"] = int(mism.size)
    return st


def assert_wta_parity(st: dict, allow_gpu_extra: float = 1e-3):
    msg = str(st)
    assert st["n_oracle_valid"] > 0, msg
    assert st["index_agree"] >= INDEX_AGREE, msg
    assert st["depth_rel_frac_ok"] >= DEPTH_QUANTILE, msg
    assert st["cost1_abs_max"] <= COST_ABS, msg
    assert st["gpu_valid_oracle_invalid"] <= allow_gpu_extra * st["n_oracle_valid"] + 2, msg
    assert st["oracle_valid_gpu_invalid"] <= allow_gpu_extra * st["n_oracle_valid"] + 2, msg
    if "mismatch_cost_gap_max" in st:
        assert st["mismatch_cost_gap_max"] <= NEAR_TIE, msg
