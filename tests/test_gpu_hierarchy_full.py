"""The two-level hierarchy at the size of the refined benchmark (256^3 D3Q19
lid-driven cavity, Re 1000, plain float32, 400 patches with fine edges
from {16, 24, 32, 48}), in the benchmark's launch configuration: autotuned
tiles and workgroups, coarse steps replayed from HIP graphs, the restriction
fused into the second fine step, the LDS-staged ghost fill.  The oracle of
the whole hierarchy is too slow at this size, so two properties that hold at
any size are checked instead, from a seeded velocity perturbation at
equilibrium (patches placed by the seeded generator on a seeded block mask
confined to z < 96):

  * an isolated patch (the last one, 20+ coarse cells from any other) and the
    coarse cells around it match the FP64 hierarchy oracle run on a 28^3
    region around it alone, away from the region's cut faces;
  * far from every patch the coarse level evolves as the plain single-grid
    BGK step: after 3 coarse steps, a 64 x 56 x 64 region under the lid (16+
    cells from any patch) matches the FP64 oracle run on that region alone,
    away from its cut faces (a cell depends only on cells within 3 of it);
    a stray write of a ghost fill or restriction would show here;
  * the production configuration and a plain one (launch by launch, default
    tiles, the list-driven ghost fill and the separate restriction kernel)
    give the same coarse and fine states to the rounding of the restriction
    sums, and the same fine sensor maxima.

Tolerances: float32 populations 1e-6 absolute (values <= 1/3 rounded to
2^-24 relative per step; the oracle region also starts from a float32
rounding of the same equilibrium); sensor maxima 2e-4 relative to
max(M, 1e-3), the plain float32 sensor floor."""
import numpy as np
import pytest

import lbm_inputs
from lbm_inputs import PERIODIC, WALL

pytestmark = pytest.mark.gpu

N = 256
STEPS = 3
REGION_LO, REGION_N = (96, 200, 168), (64, 56, 64)     # under the lid (+y face)
ISOLATED = ((128, 128, 136), (140, 140, 148))           # a patch 24 fine cells wide, far from the rest
MARGIN = 8                                              # coarse cells around it in the oracle's region


def _boxes():
    nb = N // 8
    mask = (lbm_inputs.uniform(11, nb ** 3) < 0.2).reshape(nb, nb, nb)
    mask[12:] = False                                    # blocks with z >= 96 stay unflagged
    return lbm_inputs.place_patches(mask, 8, (N, N, N), count=399, seed=7) + [ISOLATED]


def _run(torch, lbm, w, tau, u, boxes, production):
    desc = lbm.make_desc(19, w.n, w.bc, tau, storage=lbm.LBM_F32, wall_u=w.wall_u,
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
    blk.set_equilibrium(u=u)
    H = lbm.Hierarchy(blk, boxes, use_graph=production)
    if production:
        H.autotune(3)
    H.step_n(STEPS - 1, 0)
    H.step_n(1, 1)
    out = (blk.populations().astype(np.float32), [H.patch_fields(p)[2].astype(np.float32)
                                                  for p in range(len(boxes))], H.sensor()[0])
    H.close()
    blk.close()
    return out


def test_full_size_hierarchy(orc, monkeypatch):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1507_06767_amd as lbm
    w = lbm_inputs.cavity3d(n=N)
    st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    boxes = _boxes()
    assert len(boxes) == 400 and max(hi[2] for lo, hi in boxes[:-1]) < 120
    fine_cells = 8 * sum(int(np.prod([hi[a] - lo[a] for a in range(3)])) for lo, hi in boxes)
    assert fine_cells > 14e6
    u = lbm_inputs.velocity_perturbation(w.n, 0.01, 5)
    print(f"\n[case] full-size hierarchy: {len(boxes)} patches, production configuration", flush=True)
    monkeypatch.delenv("LBM_HIER_RESTRICT", raising=False)
    monkeypatch.delenv("LBM_HIER_GHOSTS", raising=False)
    pa = _run(torch, lbm, w, tau, u, boxes, True)
    print("[case] full-size hierarchy: plain configuration", flush=True)
    monkeypatch.setenv("LBM_HIER_RESTRICT", "separate")
    monkeypatch.setenv("LBM_HIER_GHOSTS", "plain")
    pb = _run(torch, lbm, w, tau, u, boxes, False)

    # far field against the oracle on the region alone (its cut faces periodic
    # or walls, which the compared cells are too far from to see)
    x0, y0, z0 = REGION_LO
    nx, ny, nz = REGION_N
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = w.lid_speed
    G = orc.Grid(q=19, n=REGION_N, bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC), wall_u=wall_u,
                 tau=tau)
    ur = np.ascontiguousarray(u[:, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx])
    S0 = G.equilibrium_state(u=ur).astype(np.float32).astype(np.float64)   # the stored float32 start
    S, _ = G.run(S0, 0, STEPS, 0)
    core = (slice(None), slice(STEPS + 1, nz - STEPS - 1), slice(STEPS + 1, ny), slice(STEPS + 1, nx - STEPS - 1))
    gpu = pa[0][:, z0:z0 + nz, y0:y0 + ny, x0:x0 + nx]
    e_far = np.abs(gpu[core] - S[core]).max()
    moved = np.abs(S[core] - S0[core]).max()
    print(f"far field vs oracle: max err {e_far:.2e} (populations moved by up to {moved:.2e})")
    assert moved > 1e-4 and e_far < 1e-6

    # the isolated patch against the hierarchy oracle on the region around it
    from oracle.hier import Hierarchy as OH
    lo, hi = ISOLATED
    sub_lo = [lo[a] - MARGIN for a in range(3)]
    sub_n = tuple(hi[a] - lo[a] + 2 * MARGIN for a in range(3))
    Gs = orc.Grid(q=19, n=sub_n, bc=(PERIODIC,) * 6, tau=tau)
    sl = tuple(slice(sub_lo[a], sub_lo[a] + sub_n[a]) for a in (2, 1, 0))
    us = np.ascontiguousarray(u[(slice(None),) + sl])
    Ss = Gs.equilibrium_state(u=us).astype(np.float32).astype(np.float64)
    O = OH(Gs, [((MARGIN,) * 3, tuple(MARGIN + hi[a] - lo[a] for a in range(3)))])
    O.init_from(Ss)
    for k in range(STEPS):
        Ss, bm_o = O.step(Ss, k, sensor=(k == STEPS - 1))
    e_patch = np.abs(pa[1][-1] - O.patch_fields(0)[2]).max()
    core = tuple(slice(STEPS + 1, sub_n[a] - STEPS - 1) for a in (2, 1, 0))
    e_near = np.abs(pa[0][(slice(None),) + sl][(slice(None),) + core] - Ss[(slice(None),) + core]).max()
    nb_before = sum(int(np.prod([2 * (b[1][a] - b[0][a]) // 8 for a in range(3)])) for b in boxes[:-1])
    bm_p = pa[2][nb_before:nb_before + bm_o[0].size]
    e_pb = float((np.abs(bm_p - bm_o[0].ravel()) / np.maximum(bm_o[0].ravel(), 1e-3)).max())
    print(f"isolated patch vs hierarchy oracle: fine {e_patch:.2e}, coarse around it {e_near:.2e}, "
          f"fine block max rel err {e_pb:.2e}")
    assert e_patch < 1e-6 and e_near < 1e-6 and e_pb < 2e-4

    e_coarse = np.abs(pa[0] - pb[0]).max()
    e_fine = max(np.abs(a - b).max() for a, b in zip(pa[1], pb[1]))
    e_sens = float((np.abs(pa[2] - pb[2]) / np.maximum(pb[2], 1e-3)).max())
    print(f"production vs plain configuration: coarse {e_coarse:.2e}, fine {e_fine:.2e}, "
          f"sensor {e_sens:.2e} (max M {pb[2].max():.3e})")
    assert e_coarse < 1e-6 and e_fine < 1e-6 and e_sens < 2e-4
