"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property and the passage behind it.  Together they are
meant to catch a plausible mistake anywhere in the oracle: a wrong weight or
velocity (lattice identities), a dropped or mis-scaled equilibrium term
(moment identities, Poiseuille, shear-wave viscosity), a sign or index slip in
streaming or bounce-back (conservation, Poiseuille, symmetry, rotation,
brute-force cross-check), a wrong force term (momentum growth, Poiseuille),
and a wrong sensor (ghost-mode closed forms, Chapman-Enskog estimate).
"""
from fractions import Fraction

import numpy as np
import pytest

import lbm_inputs
from lbm_inputs import PERIODIC, WALL


def _frac_tables(orc, q):
    c, w, opp, d = orc.lattice_tables(q)
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    for a, b in zip(w, wf):
        assert abs(float(b) - a) < 1e-16
    return c, wf, opp, d


# ---------------------------------------------------------------- P1, P2 -----
@pytest.mark.parametrize("q", [9, 19, 27])
def test_lattice_isotropy_exact(orc, q):
    """Sec. 2.2: the velocity set must reproduce the Maxwellian moments up to
    fourth order with c_s^2 = 1/3: sum w = 1, sum w c_a = 0, sum w c_a c_b =
    c_s^2 d_ab, odd third moments 0, sum w c_a c_b c_c c_d = c_s^4 (d d + d d + d d)."""
    c, w, opp, d = _frac_tables(orc, q)
    cs2 = Fraction(1, 3)
    assert sum(w) == 1
    dims = range(d)
    for a in dims:
        assert sum(w[i] * c[i][a] for i in range(q)) == 0
        for b in dims:
            m2 = sum(w[i] * c[i][a] * c[i][b] for i in range(q))
            assert m2 == (cs2 if a == b else 0)
            for g in dims:
                assert sum(w[i] * c[i][a] * c[i][b] * c[i][g] for i in range(q)) == 0
                for e in dims:
                    m4 = sum(w[i] * c[i][a] * c[i][b] * c[i][g] * c[i][e] for i in range(q))
                    dd = (a == b) * (g == e) + (a == g) * (b == e) + (a == e) * (b == g)
                    assert m4 == cs2 * cs2 * dd
    for i in range(q):
        assert (c[opp[i]] == -c[i]).all()
    assert len({tuple(v) for v in c}) == q


@pytest.mark.parametrize("q,expected", [(9, 0.5), (19, np.sqrt(5) / 6), (27, 1 / (2 * np.sqrt(2)))])
def test_weight_norm(orc, q, expected):
    """||f^eq||_2 at rest with rho = 1 is ||w||_2, the L2 sensor's denominator."""
    _, w, _, _ = orc.lattice_tables(q)
    assert abs(np.sqrt((w * w).sum()) - expected) < 1e-15


# ---------------------------------------------------------------- P3 ---------
@pytest.mark.parametrize("q", [9, 19, 27])
def test_equilibrium_moments(orc, q):
    """Eqs. rho and u: sum_i f^eq_i = rho and sum_i xi_i f^eq_i = rho u; and the
    second-order equilibrium's momentum flux sum_i xi xi f^eq = rho (u u + c_s^2 I)."""
    c = np.array(orc.ABI_VELOCITIES[q], dtype=float)
    d = 2 if q == 9 else 3
    rng = lbm_inputs.uniform(7, 40)
    for k in range(10):
        rho = 0.8 + 0.4 * rng[4 * k]
        u = np.zeros(3)
        u[:d] = 0.2 * (rng[4 * k + 1:4 * k + 1 + d] - 0.5)
        feq = orc.equilibrium(q, rho, u)
        assert abs(feq.sum() - rho) < 1e-15
        assert np.abs(c.T @ feq - rho * u).max() < 1e-15
        Pi = np.einsum("ia,ib,i->ab", c, c, feq)
        exp = rho * (np.outer(u, u) + np.eye(3) / 3.0)
        if d == 2:
            exp[2, 2] = 0.0
        assert np.abs(Pi - exp).max() < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("kind", [0, 1])
def test_sensor_ghost_mode_closed_form(orc, q, kind):
    """Sec. 3.2: a perturbation h with sum h = 0 and sum xi h = 0 leaves rho and
    u unchanged, so f^neq = h exactly.  On f = f^eq(rho, u) + h the L2 sensor is
    ||h|| / ||f^eq|| and Eq. kkn gives (1/q) sum |h_i / f^eq_i|.  At rest with
    rho = 1 and h = eps on the +-x links, -eps on the +-y links:
    D2Q9 L2 = 2 eps / (1/2) = 4 eps, K_Kn = (1/9) * 4 eps * 9 = 4 eps."""
    eps = 1e-4
    G = orc.Grid(q=q, n=(1, 1, 1), sensor_kind=kind)
    vel = orc.ABI_VELOCITIES[q]
    h = np.zeros(q)
    h[vel.index((1, 0, 0))] = h[vel.index((-1, 0, 0))] = eps
    h[vel.index((0, 1, 0))] = h[vel.index((0, -1, 0))] = -eps
    for rho, u in ((1.0, (0.0, 0.0, 0.0)), (1.1, (0.03, -0.02, 0.01 if q != 9 else 0.0))):
        feq = orc.equilibrium(q, rho, u)
        f = (feq + h).reshape(q, 1, 1, 1)
        s = G.sensor(f)[0, 0, 0]
        if kind == 0:
            exp = np.sqrt((h * h).sum()) / np.sqrt((feq * feq).sum())
        else:
            exp = np.abs(h / feq).sum() / q
        assert abs(s - exp) < 1e-12 * exp
    if q == 9:
        f = (orc.equilibrium(9, 1.0, (0, 0, 0)) + h).reshape(9, 1, 1, 1)
        assert abs(G.sensor(f)[0, 0, 0] - 4 * eps) < 1e-15


@pytest.mark.parametrize("q", [9, 19, 27])
def test_sensor_zero_at_equilibrium(orc, q):
    """The sensor is 0 when the populations are at local equilibrium."""
    n = (5, 4, 1 if q == 9 else 3)
    u = lbm_inputs.velocity_perturbation(n, 0.05, seed=3, dims=2 if q == 9 else 3)
    rho = 1.0 + 0.1 * lbm_inputs.uniform(4, n[0] * n[1] * n[2])
    for kind in (0, 1):
        G = orc.Grid(q=q, n=n, sensor_kind=kind)
        f = G.equilibrium_state(rho=rho, u=u)
        assert np.abs(G.sensor(f)).max() < 1e-14


@pytest.mark.parametrize("q", [9, 19, 27])
def test_uniform_flow_is_a_fixed_point(orc, q):
    """A uniform (rho0, u0) state at equilibrium in a periodic box stays so,
    with a vanishing sensor."""
    n = (6, 5, 1 if q == 9 else 4)
    N = n[0] * n[1] * n[2]
    u0 = np.array([0.04, -0.03, 0.02 if q != 9 else 0.0])
    G = orc.Grid(q=q, n=n, tau=0.7)
    S0 = G.equilibrium_state(rho=np.full(N, 1.02), u=np.repeat(u0[:, None], N, axis=1))
    S, hist = G.run(S0, 0, 50, 10)
    assert np.abs(S - S0).max() < 1e-15
    for _, bm, fl in hist:
        assert np.nanmax(bm) < 1e-14
        assert (fl == -1).all()


def test_cavity_at_rest_stays_at_rest(orc):
    """Walls with zero velocity and a state at rest: no flow is created and
    every block is flagged for coarsening."""
    G = orc.Grid(q=19, n=(10, 9, 8), bc=(WALL,) * 6, tau=0.6)
    S0 = G.equilibrium_state()
    S, hist = G.run(S0, 0, 20, 5)
    assert np.abs(S - S0).max() < 1e-15
    for _, bm, fl in hist:
        assert bm.max() < 1e-15 and (fl == -1).all()


# ---------------------------------------------------------------- P4, P5 -----
@pytest.mark.parametrize("q", [9, 19, 27])
def test_periodic_box_conservation(orc, q):
    """Eqs. ns1 and ns2 stem from exact mass and momentum conservation by the
    collision and the streaming: in a periodic box the totals stay constant to
    round-off."""
    n = (24, 20, 1) if q == 9 else (12, 10, 8)
    u = lbm_inputs.velocity_perturbation(n, 0.01, seed=1, dims=2 if q == 9 else 3)
    G = orc.Grid(q=q, n=n, tau=0.8)
    S0 = G.equilibrium_state(u=u)
    c0 = G.conservation(S0)
    S, _ = G.run(S0, 0, 300, 0)
    c1 = G.conservation(S)
    N = G.cells
    assert abs(c1[0] - c0[0]) < 1e-13 * N
    assert np.abs(c1[1:] - c0[1:]).max() < 1e-14 * N
    assert np.abs(S - S0).max() > 1e-4          # the state really evolved


@pytest.mark.parametrize("q", [9, 19, 27])
def test_body_force_momentum_growth(orc, q):
    """Guo's source adds exactly F per cell and step to the momentum while
    leaving the mass unchanged."""
    n = (8, 6, 1) if q == 9 else (6, 5, 4)
    F = (2e-5, -1e-5, 3e-6 if q != 9 else 0.0)
    u = lbm_inputs.velocity_perturbation(n, 0.01, seed=2, dims=2 if q == 9 else 3)
    G = orc.Grid(q=q, n=n, tau=0.9, force=F)
    S0 = G.equilibrium_state(u=u)
    c0 = G.conservation(S0)
    steps = 100
    S, _ = G.run(S0, 0, steps, 0)
    c1 = G.conservation(S)
    N = G.cells
    assert abs(c1[0] - c0[0]) < 1e-13 * N
    assert np.abs(c1[1:] - c0[1:] - steps * N * np.array(F)).max() < 1e-13 * N


@pytest.mark.parametrize("q,n", [(9, (16, 16, 1)), (19, (8, 8, 8)), (27, (8, 8, 8))])
def test_cavity_mass_conservation(orc, q, n):
    """The moving bounce-back terms cancel pairwise when every link through
    the lid, its edges and its corners uses the lid velocity, so the cavity
    conserves mass to round-off."""
    bc = (WALL, WALL, WALL, WALL, PERIODIC, PERIODIC) if q == 9 else (WALL,) * 6
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.1
    G = orc.Grid(q=q, n=n, bc=bc, wall_u=wall_u, tau=0.7)
    S0 = G.equilibrium_state()
    m0 = G.conservation(S0)[0]
    S, _ = G.run(S0, 0, 400, 0)
    assert abs(G.conservation(S)[0] - m0) < 1e-13 * G.cells
    _, u = G.macros(S)
    assert u[0].max() > 1e-3                   # the lid drives a flow


# ---------------------------------------------------------------- P6, P7 -----
def _poiseuille(orc, q, tau, axes=(0, 1), H=32, steps=40000, umax=1e-3):
    """Channel along axes[0], walls normal to axes[1]; returns (G, S, y, g)."""
    nu = (tau - 0.5) / 3.0
    g = umax * 8.0 * nu / H ** 2
    n = [1, 1, 1]
    n[axes[1]] = H
    bc = [PERIODIC] * 6
    bc[2 * axes[1]] = bc[2 * axes[1] + 1] = WALL
    F = [0.0, 0.0, 0.0]
    F[axes[0]] = g
    G = orc.Grid(q=q, n=tuple(n), bc=tuple(bc), tau=tau, force=tuple(F))
    S, _ = G.run(G.equilibrium_state(), 0, steps, 0)
    return G, S, np.arange(H) + 0.5, g


@pytest.mark.parametrize("q,axes", [(9, (0, 1)), (9, (1, 0)), (19, (0, 1)), (19, (2, 0)), (19, (1, 2))])
@pytest.mark.parametrize("tau", [0.8, 1.0, 0.5 + np.sqrt(3.0) / 4.0])
def test_poiseuille_closed_form(orc, q, axes, tau):
    """Steady force-driven channel with halfway bounce-back and Guo forcing.
    The discrete BGK steady state is exactly
        u(y) = g / (2 nu) [ y (H - y) + (16 tau^2 - 16 tau + 1) / 12 ],
    y = j + 1/2, nu = c_s^2 (tau - 1/2) (Eq. nu_omega); the slip term vanishes
    at (tau - 1/2)^2 = 3/16, where halfway bounce-back is exact."""
    if q == 9 and 2 in axes:
        pytest.skip("2D")
    H = 32
    G, S, y, g = _poiseuille(orc, q, tau, axes, H=H)
    nu = (tau - 0.5) / 3.0
    rho, u = G.macros(S)
    prof = u[axes[0]].reshape(-1)
    exact = g / (2 * nu) * (y * (H - y) + (16 * tau ** 2 - 16 * tau + 1) / 12.0)
    assert np.abs(prof - exact).max() < 1e-8 * exact.max()
    other = [a for a in range(3) if a != axes[0]]
    assert np.abs(u[other]).max() < 1e-10 * exact.max()
    assert np.abs(rho - 1.0).max() < 1e-10


@pytest.mark.parametrize("q", [9, 19])
def test_poiseuille_nonequilibrium_and_sensor(orc, q):
    """Chapman-Enskog (Eqs. generalf0, generalf1): f^neq ~ -tau w_i rho Q_i:S / c_s^2,
    i.e. -3 w tau c_x c_y u' on the diagonal links of a shear flow.  On the
    discrete Poiseuille state the x-odd part of f^neq on the (+-1, +1) and
    (+-1, -1) links is exactly -+(tau u' + G)/12 and +-(tau u' - G)/12 with
    G = (4 tau + 1) g / 2, whose leading term is the CE estimate.  Hence the
    L2 sensor is sqrt(tau^2 u'^2 + G^2) / ||w||, up to O(u) relative."""
    tau, H = 0.8, 32
    G, S, y, g = _poiseuille(orc, q, tau, (0, 1), H=H)
    nu = (tau - 0.5) / 3.0
    f = G.stream(S)
    rho, u = G.macros(f, post_collision=False)
    up = g / nu * (H / 2.0 - y)
    Gc = (4 * tau + 1) * g / 2.0
    feq = np.stack([orc.equilibrium(q, rho.ravel()[j], u[:, 0, j, 0]) for j in range(H)], axis=1)
    fneq = f.reshape(q, H) - feq
    vel = orc.ABI_VELOCITIES[q]
    for cy in (1, -1):
        ip, im = vel.index((1, cy, 0)), vel.index((-1, cy, 0))
        odd = 0.5 * (fneq[ip] - fneq[im])
        exact = -(tau * up + Gc) / 12.0 if cy == 1 else (tau * up - Gc) / 12.0
        assert np.abs(odd - exact).max() < 1e-9 * np.abs(exact).max()
        ce = -3.0 * (1.0 / 36.0) * tau * cy * up       # c_x = +1
        wall = slice(0, 4)
        assert np.all(np.abs(odd[wall] - ce[wall]) < 0.05 * np.abs(ce[wall]))
    s = G.sensor(f).ravel()
    wnorm = np.sqrt(5.0) / 6.0 if q == 19 else 0.5
    pred = np.sqrt(tau ** 2 * up ** 2 + Gc ** 2) / 6.0 / wnorm
    assert np.abs(s - pred).max() < 2e-3 * pred.max()


# ---------------------------------------------------------------- P8 ---------
@pytest.mark.parametrize("q,n", [(9, (1, 64, 1)), (19, (1, 64, 1)), (19, (64, 1, 1)), (27, (1, 64, 1)),
                                 (27, (64, 1, 1))])
def test_shear_wave_viscosity(orc, q, n):
    """Eq. nu_omega: a periodic shear wave u = A sin(k y) decays as
    exp(-nu k^2 t) with nu = c_s^2 (tau - 1/2), up to O(k^2) lattice effects.
    The rate is taken between two late times to skip the start-up transient."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    axis_k = 1 if n[1] > 1 else 0
    axis_u = 0 if axis_k == 1 else 2 if q != 9 else 1
    G = orc.Grid(q=q, n=n, tau=tau)
    S = G.equilibrium_state(u=lbm_inputs.shear_wave(n, 1e-4, axis_u=axis_u, axis_k=axis_k))
    k = 2 * np.pi / n[axis_k]
    S1, _ = G.run(S, 0, 200, 0)
    S2, _ = G.run(S1, 200, 500, 0)
    a1 = np.abs(G.macros(S1)[1][axis_u]).max()
    a2 = np.abs(G.macros(S2)[1][axis_u]).max()
    rate = np.log(a1 / a2) / 500.0
    assert abs(rate / k ** 2 / nu - 1.0) < 2e-3


# ---------------------------------------------------------------- P9 ---------
def test_translation_invariance_reduces_channel(orc):
    """A state uniform in x and z stays uniform: the 3D channel equals its 1D
    reduction column by column, bit for bit."""
    H = 24
    bc = (PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC)
    G3 = orc.Grid(q=19, n=(5, H, 3), bc=bc, tau=0.8, force=(1e-6, 0, 0))
    G1 = orc.Grid(q=19, n=(1, H, 1), bc=bc, tau=0.8, force=(1e-6, 0, 0))
    S3, h3 = G3.run(G3.equilibrium_state(), 0, 300, 100)
    S1, h1 = G1.run(G1.equilibrium_state(), 0, 300, 100)
    assert (S3 == S1.reshape(19, 1, H, 1)).all()


# ---------------------------------------------------------------- P10 --------
_BRUTE_CASES = [
    ("cavity2d", 9, (10, 12, 1), (WALL, WALL, WALL, WALL, PERIODIC, PERIODIC), 0.1, (0, 0, 0)),
    ("box2d_force", 9, (9, 7, 1), (PERIODIC,) * 6, 0.0, (1e-5, 2e-5, 0)),
    ("channel2d", 9, (6, 11, 1), (PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC), 0.0, (1e-5, 0, 0)),
    ("cavity3d", 19, (9, 10, 11), (WALL,) * 6, 0.1, (0, 0, 0)),
    ("box3d_force", 19, (7, 6, 5), (PERIODIC,) * 6, 0.0, (1e-5, -2e-5, 3e-5)),
    ("mixed3d", 19, (6, 9, 10), (WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), 0.0, (0, 1e-5, 0)),
    ("cavity3d_q27", 27, (9, 8, 10), (WALL,) * 6, 0.1, (0, 0, 0)),
    ("mixed3d_q27", 27, (6, 9, 7), (WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), 0.0, (1e-5, 0, -1e-5)),
]


@pytest.mark.parametrize("case", _BRUTE_CASES, ids=[c[0] for c in _BRUTE_CASES])
@pytest.mark.parametrize("kind", [0, 1])
def test_brute_force_cross_check(orc, case, kind):
    """orc.c (push, AoS, enumerated order, tensor equilibrium) against brute.py
    (pull, SoA, interface order, expanded equilibrium) on tiny grids."""
    from oracle import brute
    name, q, n, bc, lid, F = case
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = lid
    if name.startswith("mixed3d"):           # two moving walls meeting at edges
        wall_u[0] = [0.0, 0.02, -0.01]
        wall_u[5] = [0.05, 0.02, 0.0]
    G = orc.Grid(q=q, n=n, bc=bc, wall_u=wall_u, tau=0.75, force=F, sensor_kind=kind)
    u = lbm_inputs.velocity_perturbation(n, 0.02, seed=5, dims=2 if q == 9 else 3)
    S0 = G.equilibrium_state(u=u)
    S_o, h_o = G.run(S0, 0, 25, 5)
    S_b, h_b = brute.run(S0.copy(), q, n, bc, wall_u, 0.75, 1.0, F, kind, G.block, 0, 25, 5)
    assert np.abs(S_o - S_b).max() < 1e-14
    assert [k for k, _, _ in h_o] == [k for k, _ in h_b]
    for (_, bo, _), (_, bb) in zip(h_o, h_b):
        assert np.abs(bo - bb).max() < 1e-12 * np.abs(bb).max()


# ---------------------------------------------------------------- P11 --------
def test_block_max_and_flags_planted(orc):
    """Block maxima over 8x8 blocks with ragged edge blocks, NaN propagation,
    and the thresholds: refine iff M > theta_r (a tie keeps), coarsen iff
    M < theta_c, non-finite gives 2."""
    G = orc.Grid(q=9, n=(20, 10, 1), theta_refine=1e-3, theta_coarsen=5e-4)
    s = np.zeros((1, 10, 20))
    s[0, 3, 4] = 2e-3            # block (0,0): refine
    s[0, 9, 9] = 1e-3            # block (1,1): tie with theta_r -> keep
    s[0, 2, 17] = 7e-4           # block (2,0): keep
    s[0, 8, 19] = np.nan         # block (2,1): non-finite
    s[0, 0, 10] = np.inf         # block (1,0): non-finite
    bm = G.block_max(s)
    assert bm.shape == (1, 2, 3)
    assert bm[0, 0, 0] == 2e-3 and bm[0, 1, 1] == 1e-3 and bm[0, 0, 2] == 7e-4
    assert np.isnan(bm[0, 1, 2]) and bm[0, 0, 1] == np.inf and bm[0, 1, 0] == 0.0
    fl = G.flags(bm)
    assert fl.tolist() == [[[1, 2, 0], [-1, 0, 2]]]


# ---------------------------------------------------------------- P12 --------
def test_cavity3d_mirror_symmetry(orc):
    """The 3D cavity (lid +y moving +x) is symmetric under z -> n-1-z: s, rho,
    u_x, u_y even and u_z odd."""
    n = (10, 10, 10)
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.1
    G = orc.Grid(q=19, n=n, bc=(WALL,) * 6, wall_u=wall_u, tau=0.6)
    S, _ = G.run(G.equilibrium_state(), 0, 150, 0)
    rho, u = G.macros(S)
    s = G.sensor(G.stream(S))
    m = lambda a: a[::-1, :, :]
    assert np.abs(rho - m(rho)).max() < 1e-14
    assert np.abs(u[0] - m(u[0])).max() < 1e-14 and np.abs(u[1] - m(u[1])).max() < 1e-14
    assert np.abs(u[2] + m(u[2])).max() < 1e-14
    assert np.abs(s - m(s)).max() < 1e-13
    assert np.abs(u[2]).max() > 1e-5


def test_cavity2d_reflection(orc):
    """Reflecting x -> n-1-x maps the cavity with lid +U onto the one with lid
    -U, with u_x -> -u_x."""
    n = (12, 12, 1)
    bc = (WALL, WALL, WALL, WALL, PERIODIC, PERIODIC)
    res = []
    for U in (0.1, -0.1):
        wall_u = [[0.0] * 3 for _ in range(6)]
        wall_u[3][0] = U
        G = orc.Grid(q=9, n=n, bc=bc, wall_u=wall_u, tau=0.7)
        S, _ = G.run(G.equilibrium_state(), 0, 200, 0)
        res.append(G.macros(S))
    (r1, u1), (r2, u2) = res
    fl = lambda a: a[:, :, ::-1]
    assert np.abs(r1 - fl(r2)).max() < 1e-14
    assert np.abs(u1[0] + fl(u2[0])).max() < 1e-14
    assert np.abs(u1[1] - fl(u2[1])).max() < 1e-14


def test_cavity3d_axis_rotation(orc):
    """Relabelling the axes (x, y, z) -> (y, z, x) maps a cavity with its lid on
    +y moving +x onto one with its lid on +z moving +y."""
    n = 8
    wa = [[0.0] * 3 for _ in range(6)]
    wa[3][0] = 0.1
    wb = [[0.0] * 3 for _ in range(6)]
    wb[5][1] = 0.1
    out = []
    for wall_u in (wa, wb):
        G = orc.Grid(q=19, n=(n, n, n), bc=(WALL,) * 6, wall_u=wall_u, tau=0.6)
        S, hist = G.run(G.equilibrium_state(), 0, 60, 60)
        out.append((G.macros(S), G.sensor(G.stream(S))))
    ((ra, ua), sa), ((rb, ub), sb) = out
    t = lambda a: np.transpose(a, (1, 2, 0))
    assert np.abs(t(ra) - rb).max() < 1e-14
    assert np.abs(t(ua[0]) - ub[1]).max() < 1e-14
    assert np.abs(t(ua[1]) - ub[2]).max() < 1e-14
    assert np.abs(t(ua[2]) - ub[0]).max() < 1e-14
    assert np.abs(t(sa) - sb).max() < 1e-13


def test_tau_from_reynolds(orc):
    """nu = U N / Re and tau = nu / c_s^2 + 1/2 (Eq. nu_omega): the 64^2
    cavity at U = 0.1, Re = 100 has tau = 0.692; the 128^3 one at U = 0.05,
    Re = 1000 has tau = 0.5192."""
    assert abs(orc.tau_from_reynolds(0.1, 64, 100) - 0.692) < 1e-15
    assert abs(orc.tau_from_reynolds(0.05, 128, 1000) - 0.5192) < 1e-15


# ---------------------------------------------------------------- level map --
def test_level_map_closed_form(orc):
    """Sec. 3.4: l = clamp([a log2 K + b], l_min, l_max) with [.] = floor;
    non-finite K refines to l_max, K = 0 coarsens to l_min."""
    G = orc.Grid(q=9, n=(48, 8, 1))
    K = np.array([[[2.0 ** -12, 2.0 ** -10, 2.0 ** -9.5, 2.0 ** -8, np.nan, 0.0]]])
    lev = G.levels(K, a=1.0, b=10.0, lmin=0, lmax=1)
    assert lev.tolist() == [[[0, 0, 0, 1, 1, 0]]]
    lev = G.levels(K, a=2.0, b=24.0, lmin=-1, lmax=6)
    # 2*(-12)+24=0, -20+24=4, -19+24=5, -16+24=8->6, nan->6, 0->-1
    assert lev.tolist() == [[[0, 4, 5, 6, 6, -1]]]


def test_level_map_buffer_layer(orc):
    """Sec. 5.2: one layer of buffer blocks around tagged blocks: each block
    takes the largest level within Chebyshev distance 1 (26 neighbours in 3D),
    and distance 0 changes nothing."""
    G = orc.Grid(q=19, n=(40, 32, 24))
    nb = G.nblocks
    K = np.full((nb[2], nb[1], nb[0]), 1e-5)
    K[1, 2, 3] = 1e-2
    lev0 = G.levels(K, 1.0, 10.0, 0, 3, buffer=0)
    assert lev0.sum() == lev0[1, 2, 3] and lev0[1, 2, 3] == 3
    lev1 = G.levels(K, 1.0, 10.0, 0, 3, buffer=1)
    expected = np.zeros_like(lev0)
    expected[0:3, 1:4, 2:5] = 3
    assert (lev1 == expected).all()
    lev2 = G.levels(K, 1.0, 10.0, 0, 3, buffer=2)
    expected2 = np.zeros_like(lev0)
    expected2[0:3, 0:4, 1:5] = 3          # the grid has 5 x 4 x 3 blocks
    assert (lev2 == expected2).all()


@pytest.mark.parametrize("kind", [0, 1], ids=["L2", "KKn"])
def test_time_averaged_sensor_matches_brute_force(orc, kind):
    """Sec. 5.1 averages the cell sensor over time before building the mesh:
    the oracle's running mean over the sensor steps after `start` equals the
    mean of the sensors of brute.py (pull, SoA, its own equilibrium and
    sensor), summed step by step in numpy, on a moving-lid cavity with a body
    force (a skipped sample, an off-by-one in the window or a sum that is not
    divided by the count fails it)."""
    from oracle import brute
    n = (11, 9, 1)
    bc = (WALL, WALL, WALL, WALL, PERIODIC, PERIODIC)
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.08
    F = (1e-4, -5e-5, 0.0)
    G = orc.Grid(q=9, n=n, bc=bc, wall_u=wall_u, tau=0.66, force=F, sensor_kind=kind)
    S0 = G.equilibrium_state(u=lbm_inputs.velocity_perturbation(n, 0.02, seed=8, dims=2))
    # the window opens after step 9, itself a sensor step: samples 12, 15, ..., 39
    S, mean, cnt = G.sensor_history(S0, 0, 40, 3, start=9)
    assert cnt == 10
    acc, Sb = np.zeros(G.shape), S0.copy()
    for k in range(1, 41):
        f = brute.stream(Sb, 9, n, bc, wall_u, 1.0)
        if k % 3 == 0 and k > 9:
            acc += brute.sensor(f, 9, F, kind)
        Sb = brute.collide(f, 9, 0.66, F)
    assert np.abs(mean - acc / 10).max() <= 1e-12 * np.abs(acc / 10).max()
    assert np.abs(S - Sb).max() < 1e-14


def test_time_averaged_sensor_of_a_steady_flow(orc):
    """A flow that no longer changes has a time average equal to its
    instantaneous sensor: forced Poiseuille flow between walls started from
    its converged state, averaged over 50 steps, against the sensor of one
    step (and at rest with no force and no moving wall the average is 0)."""
    n = (4, 16, 1)
    bc = (PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC)
    F = (2e-6, 0.0, 0.0)
    G = orc.Grid(q=9, n=n, bc=bc, wall_u=[[0.0] * 3 for _ in range(6)], tau=0.8, force=F)
    S, _ = G.run(G.equilibrium_state(), 0, 6000, 0)
    one = G.sensor(G.stream(S))
    _, mean, cnt = G.sensor_history(S, 6000, 50, 1, start=6000)
    assert cnt == 50 and one.max() > 1e-7
    assert np.abs(mean - one).max() <= 1e-9 * one.max()
    R = orc.Grid(q=9, n=n, bc=bc, wall_u=[[0.0] * 3 for _ in range(6)], tau=0.8)
    _, mean0, _ = R.sensor_history(R.equilibrium_state(), 0, 12, 2, start=0)
    assert np.abs(mean0).max() < 1e-15


def test_time_averaged_sensor_matches_step_by_step(orc):
    """The running mean over sensor steps equals the mean of the per-step
    sensors recomputed from stored states (the same oracle, step by step)."""
    n = (12, 10, 1)
    bc = (WALL, WALL, WALL, WALL, PERIODIC, PERIODIC)
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.1
    G = orc.Grid(q=9, n=n, bc=bc, wall_u=wall_u, tau=0.7)
    S0 = G.equilibrium_state()
    S, mean, cnt = G.sensor_history(S0, 0, 30, 2, start=10)
    assert cnt == 10
    ref = np.zeros(G.shape)
    Sk = S0
    for k in range(1, 31):
        Sn, _ = G.run(Sk, k - 1, 1, 0)
        if k % 2 == 0 and k > 10:
            ref += G.sensor(G.stream(Sk))
        Sk = Sn
    assert np.abs(mean - ref / 10).max() < 1e-15
    assert np.abs(S - Sk).max() == 0.0
