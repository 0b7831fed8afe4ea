"""FP64 oracle of the two-level patch hierarchy (static refinement by a
factor 2, Sec. 5.1, coupled as in the AMR runs of Sec. 5.2 after Dupuis &
Chopard).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The coarse level is the C
oracle (``oracle.Grid``); the fine patches, the ghost layers, the
interpolation, the rescaling and the restriction are written here in plain
numpy, one step at a time, in the order of one coarse step:

  1. ghost layers of the fine state from the coarse state S_c(t);
  2. fine step (pull streaming, BGK with tau_f = 2 tau_c - 1/2);
  3. coarse step S_c(t) -> S_c(t+1) over every coarse cell;
  4. ghost layers from (S_c(t) + S_c(t+1)) / 2;
  5. fine step (sensor on sensor steps);
  6. restriction of the fine state onto the covered coarse cells of S_c(t+1).

Ghost cell with global fine index g: if the coarse cell g // 2 belongs to
another patch, copy that patch's value; else interpolate the coarse
post-collision populations trilinearly at the fine cell centre (coarse-index
position (g + 1/2)/2 - 1/2), and keep f^eq(rho, u) of the result while
scaling its non-equilibrium part by alpha = (tau_f - 1) / (2 (tau_c - 1)).
Restriction: mean of the 8 fine cells, non-equilibrium part scaled by
1/alpha.  (Readings: acoustic scaling of the refined level; pre-collision
f^neq scaled by tau_f / (2 tau_c), hence alpha for post-collision values.)

Pins (tests/test_oracle_hier.py): a uniform flow stays uniform through the
interface; a plane Couette flow across a patch converges to the exact linear
profile on both levels (a wrong alpha breaks the stress balance at the
interface and fails it); the fine sensor of both kinds takes its closed form
on a uniform state with a known non-equilibrium part; the single-level
reduction (no patch effect outside the stencil) is covered by comparing with
the plain coarse oracle.
"""
from __future__ import annotations

import numpy as np

from . import ABI_VELOCITIES, SENSOR_KKN, Grid, abi_permutation, lattice_tables


def _weights(q):
    _, w, _, _ = lattice_tables(q)
    return w[abi_permutation(q)]


class Hierarchy:
    """A coarse ``Grid`` and fine patches over boxes of coarse cells
    ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z))."""

    def __init__(self, G: Grid, boxes):
        self.G = G
        self.q = G.q
        self.c = np.asarray(ABI_VELOCITIES[self.q], dtype=np.int64)
        self.w = _weights(self.q)
        self.tau_c = G.tau
        self.tau_f = 2.0 * G.tau - 0.5
        self.alpha = (self.tau_f - 1.0) / (2.0 * (self.tau_c - 1.0))
        nx, ny, nz = G.n
        self.cover = -np.ones((nz, ny, nx), dtype=np.int64)
        self.boxes = [(tuple(lo), tuple(hi)) for lo, hi in boxes]
        self.o, self.e = [], []
        for p, (lo, hi) in enumerate(self.boxes):
            sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
            assert (self.cover[sl] < 0).all(), "boxes overlap"
            self.cover[sl] = p
            self.o.append(np.array([2 * lo[0], 2 * lo[1], 2 * lo[2]]))
            self.e.append(np.array([2 * (hi[0] - lo[0]), 2 * (hi[1] - lo[1]), 2 * (hi[2] - lo[2])]))
        self.F = [np.zeros((self.q, e[2] + 2, e[1] + 2, e[0] + 2)) for e in self.e]

    # -- equilibrium and rescaling ------------------------------------------------
    def feq(self, rho, u):
        """w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2) (Eq. feq_i), per column."""
        cu = self.c.astype(np.float64) @ u
        usq = (u * u).sum(axis=0)
        return self.w[:, None] * rho[None, :] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * usq[None, :])

    def rescale(self, S, factor):
        """Keep f^eq(rho, u) of populations S (q, N), scale the rest."""
        rho = S.sum(axis=0)
        u = (self.c.T.astype(np.float64) @ S) / rho
        eq = self.feq(rho, u)
        return eq + factor * (S - eq)

    # -- coarse -> fine -----------------------------------------------------------
    def interpolate(self, S0, S1, w1, g):
        """Coarse populations (q, nz, ny, nx) at fine global cells g (N, 3),
        trilinear in space, linear in time."""
        p = (g + 0.5) / 2.0 - 0.5
        base = np.floor(p).astype(np.int64)
        frac = p - base
        out = np.zeros((self.q, len(g)))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    wt = ((frac[:, 0] if dx else 1 - frac[:, 0]) * (frac[:, 1] if dy else 1 - frac[:, 1])
                          * (frac[:, 2] if dz else 1 - frac[:, 2]))
                    x, y, z = base[:, 0] + dx, base[:, 1] + dy, base[:, 2] + dz
                    val = S0[:, z, y, x] * (1 - w1) + S1[:, z, y, x] * w1
                    out += wt[None, :] * val
        return self.rescale(out, self.alpha)

    def init_from(self, S_c):
        """Every padded fine cell interpolated from the coarse state."""
        for p in range(len(self.F)):
            pz, py, px = self.F[p].shape[1:]
            zz, yy, xx = np.meshgrid(np.arange(pz), np.arange(py), np.arange(px), indexing="ij")
            g = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1) + self.o[p] - 1
            self.F[p] = self.interpolate(S_c, S_c, 0.0, g).reshape(self.F[p].shape)

    def fill_ghosts(self, S0, S1, w1):
        new = [F.copy() for F in self.F]
        for p, F in enumerate(self.F):
            pz, py, px = F.shape[1:]
            zz, yy, xx = np.meshgrid(np.arange(pz), np.arange(py), np.arange(px), indexing="ij")
            ghost = (xx == 0) | (yy == 0) | (zz == 0) | (xx == px - 1) | (yy == py - 1) | (zz == pz - 1)
            loc = np.stack([xx[ghost], yy[ghost], zz[ghost]], axis=1)
            g = loc + self.o[p] - 1
            owner = self.cover[g[:, 2] // 2, g[:, 1] // 2, g[:, 0] // 2]
            vals = np.empty((self.q, len(g)))
            own = owner >= 0
            for k in np.nonzero(own)[0]:
                r = owner[k]
                lx, ly, lz = g[k] - self.o[r] + 1
                vals[:, k] = self.F[r][:, lz, ly, lx]
            if (~own).any():
                vals[:, ~own] = self.interpolate(S0, S1, w1, g[~own])
            new[p][:, loc[:, 2], loc[:, 1], loc[:, 0]] = vals
        self.F = new

    # -- fine step ----------------------------------------------------------------
    def fine_step(self, sensor=False):
        """Pull streaming from the padded neighbours and BGK collision with
        tau_f; returns per patch the cell sensor of the pre-collision
        populations if sensor, of the coarse grid's kind (Sec. 3.2):
        ||f^neq|| / ||f^eq|| (Eq. sensor), or (1/q) sum_i |f^neq_i / f^eq_i|
        (Eq. kkn)."""
        sens = []
        for p, F in enumerate(self.F):
            ex, ey, ez = self.e[p]
            f = np.empty((self.q, ez, ey, ex))
            for i, (cx, cy, cz) in enumerate(self.c):
                f[i] = F[i, 1 - cz:1 - cz + ez, 1 - cy:1 - cy + ey, 1 - cx:1 - cx + ex]
            flat = f.reshape(self.q, -1)
            rho = flat.sum(axis=0)
            u = (self.c.T.astype(np.float64) @ flat) / rho
            eq = self.feq(rho, u)
            neq = flat - eq
            if sensor:
                if self.G.sensor_kind == SENSOR_KKN:
                    s = np.abs(neq / eq).sum(axis=0) / self.q
                else:
                    s = np.sqrt((neq * neq).sum(axis=0)) / np.sqrt((eq * eq).sum(axis=0))
                sens.append(s.reshape(ez, ey, ex))
            G = F.copy()
            G[:, 1:-1, 1:-1, 1:-1] = (flat - neq / self.tau_f).reshape(self.q, ez, ey, ex)
            self.F[p] = G
        return sens

    # -- fine -> coarse -----------------------------------------------------------
    def restrict_into(self, S_c):
        for p, (lo, hi) in enumerate(self.boxes):
            ex, ey, ez = self.e[p]
            inner = self.F[p][:, 1:-1, 1:-1, 1:-1]
            mean = inner.reshape(self.q, ez // 2, 2, ey // 2, 2, ex // 2, 2).mean(axis=(2, 4, 6))
            S_c[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = self.rescale(
                mean.reshape(self.q, -1), 1.0 / self.alpha).reshape(mean.shape)

    # -- one coarse step ----------------------------------------------------------
    def step(self, S_c, k, sensor=False):
        """Coarse step k -> k + 1 from S_c (interface layout); returns the new
        coarse state and, if sensor, the fine block maxima (one array per
        patch, [bz][by][bx] of 8^3 blocks)."""
        self.fill_ghosts(S_c, S_c, 0.0)
        self.fine_step()
        S_next, _ = self.G.run(S_c, k, 1, 0)
        self.fill_ghosts(S_c, S_next, 0.5)
        sens = self.fine_step(sensor)
        self.restrict_into(S_next)
        bmax = None
        if sensor:
            bmax = []
            for s in sens:
                ez, ey, ex = s.shape
                bmax.append(s.reshape(ez // 8, 8, ey // 8, 8, ex // 8, 8).max(axis=(1, 3, 5)))
        return S_next, bmax

    def patch_fields(self, p):
        """(rho, u (3, ...), f (q, ...)) of patch p's interior, [z][y][x]."""
        f = self.F[p][:, 1:-1, 1:-1, 1:-1]
        rho = f.sum(axis=0)
        u = np.tensordot(self.c.T.astype(np.float64), f, axes=(1, 0)) / rho
        return rho, u, f.copy()
