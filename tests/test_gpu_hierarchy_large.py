"""Fine buffers above 4 GiB.  The band fine step addresses a fine state buffer
with 32-bit byte offsets, so when a buffer exceeds 4 GiB the hierarchy runs
the W x 8 x 8 tiles of 32 cells instead.  A float64 D3Q19 hierarchy of 13
patches of 128^3 fine cells (each fine buffer about 4.4 GB) on a 200^3 cavity
reports tile width 32 and gives the same bits as the same hierarchy with the
32-wide tiles chosen explicitly (LBM_HIER_TILES=32): coarse density and
velocity, fine block maxima and flags, and one patch's populations after two
coarse steps from a seeded velocity perturbation, the second with the
sensor."""
import numpy as np
import pytest

import lbm_inputs

pytestmark = pytest.mark.gpu

N = 200
EDGE = 64          # coarse cells per patch side (128 fine)
SPACING = 66


def _boxes():
    lows = [1 + SPACING * i for i in range(3)]
    boxes = [((x, y, z), (x + EDGE, y + EDGE, z + EDGE)) for z in lows for y in lows for x in lows]
    return boxes[:13]


def _run(torch, lbm, w, tau, u, boxes):
    desc = lbm.make_desc(19, w.n, w.bc, tau, storage=lbm.LBM_F64, wall_u=w.wall_u,
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
    blk.set_equilibrium(u=u)
    H = lbm.Hierarchy(blk, boxes, use_graph=True)
    tile_x = H.info()["tile_x"]
    fine_bytes = H._bufs[0].numel()
    H.step_n(1, 0)
    H.step_n(1, 1)
    rho, uu = blk.macros()
    bm, fl, _ = H.sensor()
    f0 = H.patch_fields(0)[2]
    H.close()
    blk.close()
    del H, blk
    torch.cuda.empty_cache()
    return tile_x, fine_bytes, rho, uu, bm, fl, f0


def test_bands_fall_back_to_tiles_above_4gib(monkeypatch):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1507_06767_amd as lbm
    w = lbm_inputs.cavity3d(n=N)
    st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    u = lbm_inputs.velocity_perturbation(w.n, 0.01, 9)
    boxes = _boxes()
    print(f"\n[case] float64 hierarchy, {len(boxes)} patches of {2 * EDGE}^3, default tiling", flush=True)
    monkeypatch.delenv("LBM_HIER_TILES", raising=False)
    a = _run(torch, lbm, w, tau, u, boxes)
    print(f"fine buffer {a[1] / 2 ** 30:.2f} GiB, tile width {a[0]}", flush=True)
    assert a[1] > 2 ** 32 and a[0] == 32
    print("[case] the same with LBM_HIER_TILES=32", flush=True)
    monkeypatch.setenv("LBM_HIER_TILES", "32")
    b = _run(torch, lbm, w, tau, u, boxes)
    assert b[0] == 32
    for x, y in zip(a[2:], b[2:]):
        assert np.array_equal(x, y)
    assert np.isfinite(a[6]).all() and np.abs(a[6] - a[6][:, :1, :1, :1]).max() > 0
