"""GPU TSDF fusion (through the C ABI) against the FP64 oracle on a seeded
depth sequence of a street scene seen from a moving, turning vehicle."""
import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VOX, MU = 0.1, 0.3


def _pen_tol(blocks):
    """Depth below which a segment's reach into a block is within FP32 error:
    4 x 8 u L with u = 2^-24 and L twice the box's diagonal (metres)."""
    L = 2.0 * np.linalg.norm(np.asarray(blocks, float) * 8 * VOX)
    return 4.0 * 8.0 * 2.0 ** -24 * L


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.tsdf import TsdfMap
    return TsdfMap


def _margin_masks(infos, pen_tol):
    """Voxels whose oracle decisions sit on an FP32-sensitive boundary in any
    fused frame: grazed blocks, corner projections on the image border,
    nearest-pixel ties and eta at -mu.  The flags of earlier frames move with
    the box, as the map does."""
    bad_blk = bad_vox = b0 = None
    for inf in infos:
        if bad_blk is None:
            bad_blk = np.zeros(inf["touched"].shape, bool)
            bad_vox = np.zeros(inf["voxel_edge"].shape, bool)
        else:
            sh = inf["b0"] - b0
            bad_blk = oracle.tsdf_shift(bad_blk, sh, 1, False)
            bad_vox = oracle.tsdf_shift(bad_vox, sh, 8, False)
        b0 = inf["b0"]
        # a segment that reaches into a block no deeper than the FP32 error of
        # the GPU's box-relative positions (8 u L per coordinate, u = 2^-24,
        # L = twice the box's diagonal; four times that) is taken either way
        bad_blk |= (inf["touched"] == 1) & (inf["pen"] < pen_tol)
        bad_blk |= inf["vis_edge"] == 1
        bad_vox |= inf["voxel_edge"] == 1
    up = np.repeat(np.repeat(np.repeat(bad_blk, 8, 0), 8, 1), 8, 2)
    return bad_blk, bad_vox | up


@pytest.mark.parametrize("blocks,steps,shift", [((16, 4, 24), 0.5, False), ((12, 4, 16), 0.9, True)],
                         ids=["static_box", "moving_box"])
def test_tsdf_matches_oracle(blocks, steps, shift):
    TsdfMap = _gpu()
    seq = scenegen.depth_sequence(n_frames=5, w=160, h=120, step_m=steps, seed=1007)
    tm = TsdfMap(voxel=VOX, mu=MU, blocks=blocks, min_obs=2, max_width=160, max_height=120)
    o = oracle.TsdfOracle(VOX, MU, blocks, min_obs=2)
    infos = []
    for k, (P, c, d) in enumerate(zip(seq.poses, seq.centres, seq.depths)):
        centre = c if shift else seq.centres[0]
        centre = (centre[0], centre[1], centre[2] + 4.0)
        tm.integrate(seq.cam, P, centre, torch.from_numpy(d).cuda())
        inf = o.integrate(seq.cam, P, d, centre)
        inf["b0"] = o.b0.copy()
        infos.append(inf)
    out = tm.extract()
    torch.cuda.synchronize()
    g_d, g_w, g_c = out["tsdf"].cpu().numpy(), out["weight"].cpu().numpy(), out["count"].cpu().numpy()
    assert np.array_equal(out["first_block"], o.b0)
    bad_blk, bad_vox = _margin_masks(infos, _pen_tol(blocks))
    print("excluded blocks", bad_blk.mean(), "voxels", bad_vox.mean())
    # block observation counts
    ok = ~bad_blk
    assert np.array_equal(g_c[ok], o.count[ok]), (g_c[ok] != o.count[ok]).sum()
    # weights and values
    ok = ~bad_vox
    assert ok.mean() > 0.9
    assert np.array_equal(g_w[ok], o.W[ok].astype(np.float32)), (g_w[ok] != o.W[ok]).sum()
    od = o.extract()
    assert np.array_equal(np.isfinite(g_d[ok]), np.isfinite(od[ok]))
    fin = ok & np.isfinite(od)
    err = np.abs(g_d[fin] - od[fin])
    print(blocks, "voxels compared", ok.sum(), "finite", fin.sum(), "max |dD|", err.max())
    assert fin.sum() > 1000 and err.max() <= 1e-4
    a, v = tm.stats()
    assert a == int(o.alloc.sum()) or abs(a - int(o.alloc.sum())) <= int(bad_blk.sum())
    tm.close()


def test_tsdf_reset_and_far_move_empty_the_map():
    TsdfMap = _gpu()
    seq = scenegen.depth_sequence(n_frames=2, w=160, h=120, seed=1008)
    tm = TsdfMap(voxel=VOX, mu=MU, blocks=(12, 4, 16), min_obs=1, max_width=160, max_height=120)
    d = torch.from_numpy(seq.depths[0]).cuda()
    tm.integrate(seq.cam, seq.poses[0], (0.0, 0.0, 4.0), d)
    assert tm.stats()[0] > 0
    # the box moves 100 m away: every block leaves; nothing new is in view there
    tm.integrate(seq.cam, seq.poses[0], (0.0, 0.0, 104.0), d)
    out = tm.extract()
    assert tm.stats()[0] == 0 and int(out["count"].sum()) == 0 and not torch.isfinite(out["tsdf"]).any()
    tm.integrate(seq.cam, seq.poses[0], (0.0, 0.0, 4.0), d)
    tm.reset()
    tm.integrate(seq.cam, seq.poses[1], (0.0, 0.0, 4.0), torch.full_like(d, float("nan")))
    assert tm.stats()[0] == 0
    tm.close()
