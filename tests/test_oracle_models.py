"""Pins of the oracle's model options: the Smagorinsky subgrid model the paper
adds to BGK at high Reynolds number (Sec. 4) and the smoothed lid velocity of
the 3D cavity (Sec. 5.1).  Each pin checks a defining property, not the
oracle's formula retyped."""
import numpy as np
import pytest

import lbm_inputs
from lbm_inputs import PERIODIC, WALL


def _near_eq_state(orc, G, seed, amp=0.02):
    """Equilibrium of a random (rho, u) plus a random perturbation."""
    n = G.cells
    rho = 1.0 + 0.05 * (2 * lbm_inputs.uniform(seed, n) - 1)
    u = 0.05 * (2 * lbm_inputs.uniform(seed + 1, 3 * n) - 1)
    f = G.equilibrium_state(rho, u.reshape(3, n))
    pert = amp * (2 * lbm_inputs.uniform(seed + 2, f.size) - 1).reshape(f.shape)
    return f * (1.0 + pert)


@pytest.mark.parametrize("q", [9, 19])
def test_smagorinsky_zero_constant_is_bgk(orc, q):
    n = (5, 4, 1) if q == 9 else (4, 3, 5)
    G0 = orc.Grid(q=q, n=n, tau=0.53)
    G1 = orc.Grid(q=q, n=n, tau=0.53, smagorinsky=0.0)
    f = _near_eq_state(orc, G0, 3)
    assert np.array_equal(G0.collide(f), G1.collide(f))
    # at equilibrium Pi^neq = 0: the model adds no viscosity
    Gs = orc.Grid(q=q, n=n, tau=0.53, smagorinsky=0.14)
    feq = G0.equilibrium_state()
    assert np.allclose(Gs.collide(feq), feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("C", [0.1, 0.14, 0.3])
def test_smagorinsky_eddy_viscosity_definition(orc, q, C):
    """From the collided state read back the relaxation time each cell used
    (all populations must share it) and check the model's definition:
    c_s^2 (tau_e - tau) = C^2 |S|, |S| = sqrt(2 S:S), with the strain rate
    S = -Pi / (2 rho c_s^2 tau_e) and Pi = sum_i xi_i xi_i (f_i - f^eq_i)."""
    n = (6, 5, 1) if q == 9 else (4, 5, 3)
    tau = 0.505
    G = orc.Grid(q=q, n=n, tau=tau, smagorinsky=C)
    f = _near_eq_state(orc, G, 17)
    S = G.collide(f)
    c = np.asarray(orc.ABI_VELOCITIES[q], dtype=np.float64)     # interface order, as f
    fi = f.reshape(q, -1)
    Si = S.reshape(q, -1)
    rho = fi.sum(axis=0)
    u = (c.T @ fi) / rho
    cs2 = 1.0 / 3.0
    for cell in range(fi.shape[1]):
        feq = orc.equilibrium(q, rho[cell], u[:, cell])
        fneq = fi[:, cell] - feq
        ratio = (Si[:, cell] - feq) / fneq
        big = np.abs(fneq) > 1e-6
        r = ratio[big]
        assert np.allclose(r, r[0], rtol=0, atol=1e-9), "one relaxation time per cell"
        tau_e = 1.0 / (1.0 - ratio[np.argmax(np.abs(fneq))])     # best-conditioned read-back
        Pi = np.einsum("ia,ib,i->ab", c, c, fneq)
        Sab = -Pi / (2.0 * rho[cell] * cs2 * tau_e)
        nu_t = C * C * np.sqrt(2.0 * np.sum(Sab * Sab))
        assert tau_e > tau
        assert np.isclose(cs2 * (tau_e - tau), nu_t, rtol=1e-6, atol=0), (cell, tau_e)


@pytest.mark.parametrize("q", [9, 19])
def test_smagorinsky_conserves_mass_and_momentum(orc, q):
    n = (6, 5, 1) if q == 9 else (4, 5, 3)
    G = orc.Grid(q=q, n=n, tau=0.51, smagorinsky=0.14)
    f = _near_eq_state(orc, G, 29, amp=0.05)
    S = G.collide(f)
    c = np.asarray(orc.ABI_VELOCITIES[q], dtype=np.float64)
    assert np.allclose(S.reshape(q, -1).sum(0), f.reshape(q, -1).sum(0), rtol=0, atol=1e-14)
    assert np.allclose(c.T @ S.reshape(q, -1), c.T @ f.reshape(q, -1), rtol=0, atol=1e-14)


def _lid_momentum(orc, q, n, profile):
    bc = (PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC) if q == 9 else (WALL,) * 6
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.05
    prof = [0] * 6
    prof[3] = profile
    G = orc.Grid(q=q, n=n, bc=bc, wall_u=wall_u, tau=0.6, wall_profile=prof)
    f = G.stream(G.equilibrium_state())
    c = np.asarray(orc.ABI_VELOCITIES[q], dtype=np.float64)
    return float(c[:, 0] @ f.reshape(q, -1).sum(axis=1))


def test_smoothed_lid_profile_mean():
    """One streaming step from rest: the x momentum the moving lid injects is
    proportional to its velocity summed over the lid cells, so smoothed over
    uniform is the mean of the profile (1 - s^18)^2 over the cell centres,
    which for many cells is half its integral over (-1, 1): (2 - 4/19 + 2/37) / 2.
    A wrong exponent, a missing square or a shifted coordinate fails this."""
    import oracle as orc
    n = 2048
    ratio = _lid_momentum(orc, 9, (n, 3, 1), 1) / _lid_momentum(orc, 9, (n, 3, 1), 0)
    assert abs(ratio - (2.0 - 4.0 / 19.0 + 2.0 / 37.0) / 2.0) < 1e-6


def test_smoothed_lid_profile_is_a_product_over_the_lid_axes(orc):
    """In 3D the lid factor is the product of the profile along x and along z:
    the injected-momentum ratio of a 3D lid equals the product of the 2D
    ratios for the same x and z extents."""
    nx, nz = 24, 16
    r3 = _lid_momentum(orc, 19, (nx, 5, nz), 1) / _lid_momentum(orc, 19, (nx, 5, nz), 0)
    rx = _lid_momentum(orc, 9, (nx, 3, 1), 1) / _lid_momentum(orc, 9, (nx, 3, 1), 0)
    rz = _lid_momentum(orc, 9, (nz, 3, 1), 1) / _lid_momentum(orc, 9, (nz, 3, 1), 0)
    assert np.isclose(r3, rx * rz, rtol=1e-12)
    assert 0.5 < rx < 0.95 and 0.5 < rz < 0.95


def test_smoothed_lid_profile_symmetry(orc):
    """The profile is symmetric about the lid centre: a smoothed-lid cavity
    keeps the mirror symmetry z -> nz - 1 - z of the uniform one."""
    n = (12, 10, 9)
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.05
    G = orc.Grid(q=19, n=n, bc=(WALL,) * 6, wall_u=wall_u, tau=0.6, wall_profile=(0, 0, 0, 1, 0, 0))
    S, _ = G.run(G.equilibrium_state(), 0, 20, 0)
    rho, u = G.macros(S)
    assert np.allclose(u[0], u[0][::-1], rtol=0, atol=1e-15)
    assert np.allclose(u[2], -u[2][::-1], rtol=0, atol=1e-15)
