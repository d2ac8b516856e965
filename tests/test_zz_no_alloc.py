"""psweep_run_noalloc (the entry point for callers that cannot allocate:
its scratch is the library's static device array) gives the maps of
psweep_run bitwise, on two calls in a row, the second with a smaller frame;
contexts whose scratch would not fit are refused."""
import numpy as np
import pytest

import scenegen
from scenegen import Level, Settings
from tests.parity import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    return PlaneSweep, frame_to_device


def _same(a, b):
    for name in a:
        assert np.array_equal(a[name], b[name], equal_nan=True), name


def test_noalloc_matches_run_two_calls_second_smaller():
    PlaneSweep, frame_to_device = _gpu()
    big = scenegen.random_small_frame(w=320, h=240, n_src=3, seed=61, f=200.0)
    small = scenegen.random_small_frame(w=200, h=136, n_src=3, seed=62, f=125.0)
    lv = Level(n_fronto=24, near=1.0, far=25.0, n_ground=12, h_lo=-0.4, h_hi=0.4, window=9)
    st = Settings(levels=[lv], best_k=2)
    ps = PlaneSweep(st, 320, 240, 3, max_camera_sets=2)
    ps.set_cameras(0, big.ref_cam, big.src_cams, big.poses)
    ps.set_cameras(1, small.ref_cam, small.src_cams, small.poses)
    db, ds = frame_to_device(big), frame_to_device(small)
    ds["camera_set"] = 1
    # the workspace path (plane chunks as chosen automatically)
    ref_b, ref_s = ps.alloc_outputs(0), ps.alloc_outputs(1)
    ps.run([db], [ref_b])
    ps.run([ds], [ref_s])
    torch.cuda.synchronize()
    want_b, want_s = to_np(ref_b["merged"]), to_np(ref_s["merged"])
    # the static-scratch path, twice in a row: the large frame, then the small one
    out_b, out_s = ps.alloc_outputs(0), ps.alloc_outputs(1)
    for o in (out_b, out_s):
        for t in o["merged"].values():
            t.fill_(7)
    ps.run_noalloc([db], [out_b])
    ps.run_noalloc([ds], [out_s])
    torch.cuda.synchronize()
    got_b, got_s = to_np(out_b["merged"]), to_np(out_s["merged"])
    # and the workspace path again after it (its tables are set up afresh)
    again = ps.alloc_outputs(0)
    ps.run([db], [again])
    torch.cuda.synchronize()
    ps.close()
    assert (want_b["index"] >= 0).sum() > 10000 and (want_s["index"] >= 0).sum() > 4000
    _same(want_b, got_b)
    _same(want_s, got_s)
    _same(want_b, to_np(again["merged"]))


def test_noalloc_two_levels_matches_run():
    PlaneSweep, frame_to_device = _gpu()
    fr = scenegen.random_small_frame(w=256, h=192, n_src=2, seed=63, f=160.0)
    st = Settings(levels=[Level(n_fronto=16, near=1.0, far=25.0, window=7, downsample=2),
                          Level(n_fronto=12, near=8.0, far=40.0, window=9, crop=(64, 48, 128, 96))], best_k=2)
    ps = PlaneSweep(st, 256, 192, 2)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    d = frame_to_device(fr)
    a, b = ps.alloc_outputs(), ps.alloc_outputs()
    ps.run([d], [a])
    ps.run_noalloc([d], [b])
    torch.cuda.synchronize()
    ps.close()
    _same(to_np(a["merged"]), to_np(b["merged"]))


def test_noalloc_refuses_contexts_beyond_its_scratch():
    PlaneSweep, _ = _gpu()
    from paper_1809_06132_amd import psweep
    fr = scenegen.random_small_frame(w=64, h=48, n_src=2, seed=64, f=40.0)
    st = Settings(levels=[Level(n_fronto=8, near=1.0, far=20.0, window=7)], best_k=2)
    ps = PlaneSweep(st, 4096, 4096, 4)      # textures alone: 4 x 128 MiB
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    from paper_1809_06132_amd.sweep import frame_to_device
    with pytest.raises(psweep.PsweepError) as ei:
        ps.run_noalloc([frame_to_device(fr)], [out])
    assert ei.value.status == psweep.EINVAL and "static" in str(ei.value)
    ps.close()
