"""Pins of the patch-hierarchy oracle (oracle/hier.py) against what the
physics fixes: a uniform flow crosses the refinement interface unchanged, and
a plane Couette flow reaches the exact linear profile on both levels.  A
wrong rescaling of the non-equilibrium part (planted below) breaks the
shear-stress balance at the interface and fails the Couette pin."""
import numpy as np
import pytest

from lbm_inputs import PERIODIC, WALL


def _uniform_state(G, rho, u):
    N = G.cells
    return G.equilibrium_state(rho=np.full(N, rho), u=np.repeat(np.asarray(u, float)[:, None], N, axis=1))


@pytest.mark.parametrize("q", [19, 27])
def test_uniform_flow_crosses_the_interface(orc, q):
    from oracle.hier import Hierarchy
    G = orc.Grid(q=q, n=(16, 12, 12), bc=(PERIODIC,) * 6, tau=0.7)
    S = _uniform_state(G, 1.01, (0.03, -0.02, 0.01))
    H = Hierarchy(G, [((4, 2, 4), (8, 6, 8)), ((8, 2, 4), (12, 6, 8))])     # two abutting patches
    H.init_from(S)
    S0 = S.copy()
    for k in range(5):
        S, bm = H.step(S, k, sensor=(k == 4))
    assert np.abs(S - S0).max() < 1e-14
    f_ref = S0[:, 0, 0, 0]
    for p in range(2):
        rho, u, f = H.patch_fields(p)
        assert np.abs(f - f_ref[:, None, None, None]).max() < 1e-14
    assert max(b.max() for b in bm) < 1e-13


@pytest.mark.parametrize("kind", [0, 1], ids=["l2", "kkn"])
def test_fine_sensor_closed_form(orc, kind):
    """A uniform coarse state f^eq(rho, u) + delta, delta orthogonal to the
    mass and momentum sums: every fine cell, ghosts included, starts at
    f^eq + alpha delta (interpolation keeps it, the rescaling scales the
    non-equilibrium part by alpha), streaming leaves it, and the fine sensor
    takes the closed form of Sec. 3.2 on it: ||alpha delta|| / ||f^eq||
    (Eq. sensor) or (1/q) sum_i |alpha delta_i| / f^eq_i (Eq. kkn)."""
    from oracle.hier import Hierarchy
    G = orc.Grid(q=19, n=(12, 12, 12), bc=(PERIODIC,) * 6, tau=0.7, sensor_kind=kind)
    rho, u = 1.02, np.array([0.04, -0.01, 0.02])
    S = _uniform_state(G, rho, u)
    feq = S[:, 0, 0, 0].copy()
    c = np.asarray(orc.ABI_VELOCITIES[19], dtype=float)
    M = np.vstack([np.ones(19), c.T])                        # the mass and momentum sums
    r = np.random.default_rng(9).standard_normal(19) * 1e-3 * feq
    delta = r - M.T @ np.linalg.solve(M @ M.T, M @ r)        # orthogonal to them
    assert np.abs(M @ delta).max() < 1e-17
    S = S + delta[:, None, None, None]
    H = Hierarchy(G, [((3, 3, 3), (7, 7, 7)), ((7, 3, 3), (11, 7, 7))])
    H.init_from(S)
    H.fill_ghosts(S, S, 0.0)
    sens = H.fine_step(sensor=True)
    ad = H.alpha * delta
    want = (np.sqrt((ad * ad).sum()) / np.sqrt((feq * feq).sum()) if kind == 0
            else np.abs(ad / feq).sum() / 19)
    assert want > 1e-4
    for s in sens:
        assert s.shape == (8, 8, 8)
        assert np.abs(s / want - 1).max() < 1e-10


def _couette(orc, alpha=None, steps=1500):
    """Plane Couette flow between y walls (the +y wall moves at U in x),
    periodic in x and z, one patch across the middle of the gap, from the
    linear profile at equilibrium.  Returns (largest distance of the coarse
    and fine x-velocities of one column from their common best-fit line,
    fitted slope over the exact one, relative mass change, largest cross-flow
    velocity), velocities relative to U."""
    from oracle.hier import Hierarchy
    U, ny = 0.02, 16
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = U
    G = orc.Grid(q=19, n=(8, ny, 8), bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC), wall_u=wall_u,
                 tau=0.8)
    y = np.arange(ny)
    u = np.zeros((3, 8, ny, 8))
    u[0] = (U * (y + 0.5) / ny)[None, :, None]
    S = G.equilibrium_state(u=u)
    H = Hierarchy(G, [((2, 4, 2), (6, 12, 6))])
    if alpha is not None:
        H.alpha = alpha
    H.init_from(S)
    for k in range(steps):
        S, _ = H.step(S, k)
    rc, uc = G.macros(S)
    rf, uf, _ = H.patch_fields(0)
    Y = np.concatenate([y.astype(float), (np.arange(8, 24) + 0.5) / 2.0 - 0.5])   # coarse-index positions
    V = np.concatenate([uc[0][0, :, 0], uf[0][0, :, 0]])
    A = np.stack([Y, np.ones_like(Y)], axis=1)
    coef = np.linalg.lstsq(A, V, rcond=None)[0]
    mass = rc[H.cover < 0].sum() + rf.sum() / 8.0
    cross = max(np.abs(uc[1:]).max(), np.abs(uf[1:]).max())
    return np.abs(V - A @ coef).max() / U, coef[0] / (U / ny), mass / G.cells - 1.0, cross / U


def test_couette_profile_is_linear_across_the_interface(orc):
    """BGK with halfway bounce-back keeps the Couette profile exactly linear;
    so must the coupled levels, whose interface then carries the same shear
    stress on both sides.  The coupling does not conserve mass exactly (the
    populations the patch sends out and receives come from different
    interpolations): the slope follows the slow mass change, which is
    bounded here per coarse step."""
    res, slope, dm, cross = _couette(orc)
    print(f"Couette: line residual {res:.2e}, slope/exact {slope:.6f}, mass change {dm:.2e}, cross {cross:.1e}")
    assert res < 1e-5 and abs(slope - 1.0) < 1e-4 and abs(dm) < 1e-7 * 1500 and cross < 5e-5


def test_couette_bends_with_a_wrong_rescaling(orc):
    """Planted mistake in the oracle: non-equilibrium parts passed unscaled
    (alpha = 1 instead of -1/4 at tau = 0.8).  The interface then carries the
    wrong shear stress and the profile bends."""
    res, slope, _, _ = _couette(orc, alpha=1.0)
    print(f"Couette with alpha = 1: line residual {res:.2e}, slope/exact {slope:.4f}")
    assert res > 1e-3
