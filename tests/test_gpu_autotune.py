"""The autotuner picks a tile shape and a plane-chunk count per level from
timings; whatever it picks still matches the oracle, and its cache hands the
same choice to a later context without timing again."""
import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Level, Settings
from tests.parity import assert_wta_parity, to_np, wta_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_choice_matches_oracle_and_is_cached(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.autotune import tune
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    fr = scenegen.random_small_frame(w=200, h=140, n_src=3, seed=31, f=120.0)
    lv = Level(n_fronto=16, near=1.0, far=25.0, n_ground=8, h_lo=-0.4, h_hi=0.4, window=9)
    st = Settings(levels=[lv], best_k=2)
    cache = str(tmp_path / "tiles.json")
    d = frame_to_device(fr)

    ps = PlaneSweep(st, 200, 140, 3)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    choice = tune(ps, [d], [out], reps=2, cache_path=cache, candidates=[(4, 4), (8, 4)],
                  chunk_candidates=[0, 1, 4])
    assert choice["tiles"][0] in ([4, 4], [8, 4]) and choice["chunks"][0] in (0, 1, 4)
    ps.run([d], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, volume=True)
    s = wta_stats(g, ref, ref["volume"])
    print(choice["tiles"], choice["chunks"], s)
    assert_wta_parity(s)

    ps2 = PlaneSweep(st, 200, 140, 3)
    ps2.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out2 = ps2.alloc_outputs()
    again = tune(ps2, [d], [out2], cache_path=cache)
    assert again["tiles"] == choice["tiles"] and again["chunks"] == choice["chunks"]
    ps2.run([d], [out2])
    torch.cuda.synchronize()
    g2 = to_np(out2["merged"])
    ps2.close()
    for k in g:
        assert np.array_equal(g[k], g2[k], equal_nan=True), k
