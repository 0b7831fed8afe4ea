"""Independent numpy implementation of the same step, for tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This second oracle
cross-checks ``orc.c``: it works directly in the interface velocity order with
an explicitly written table, stores populations field-major ``(q, nz, ny, nx)``,
streams by PULLING from x - xi_i with index arithmetic done by numpy fancy
indexing, and writes the equilibrium in its expanded polynomial form
``w_i rho [1 + 3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u]`` (Eq. feq_i with c_s^2 = 1/3).
``orc.c`` instead enumerates its velocities, pushes, and contracts Q_i : uu.
Agreement of the two to round-off therefore checks the velocity order, the
boundary handling and the equilibrium of each against the other.
"""
from __future__ import annotations

import numpy as np

from . import ABI_VELOCITIES, PERIODIC

# Weights by squared velocity length (Sec. 2.2; standard DdQq weights).
_WEIGHTS = {9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36},
            19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36},
            27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}}


def tables(q):
    c = np.array(ABI_VELOCITIES[q], dtype=np.int64)
    w = np.array([_WEIGHTS[q][int((v * v).sum())] for v in c])
    opp = np.array([next(j for j in range(q) if (c[j] == -c[i]).all()) for i in range(q)])
    return c, w, opp


def stream(S, q, n, bc, wall_u, rho0):
    """Pull form: f_i(x) = S_i(x - xi_i), or the bounced S_opp(i)(x) plus the
    moving-wall term 6 w_i rho0 xi_i.u_w when x - xi_i is beyond a wall."""
    c, w, opp = tables(q)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = (x, y, z)
    f = np.empty_like(S)
    for i in range(q):
        src = []
        solid = np.zeros(x.shape, dtype=bool)
        uw = np.zeros((3,) + x.shape)
        for a in range(3):
            s = coords[a] - c[i, a]
            lo, hi = s < 0, s >= n[a]
            for mask, face in ((lo, 2 * a), (hi, 2 * a + 1)):
                if bc[face] == PERIODIC:
                    continue
                solid |= mask
                for b in range(3):
                    uw[b] += np.where(mask, wall_u[face][b], 0.0)
            src.append(np.mod(s, n[a]))
        pulled = S[i][src[2], src[1], src[0]]
        cu_w = sum(c[i, b] * uw[b] for b in range(3))
        bounced = S[opp[i]] + 6.0 * w[i] * rho0 * cu_w
        f[i] = np.where(solid, bounced, pulled)
    return f


def moments(f, q, force, sign=+1.0):
    c, _, _ = tables(q)
    rho = f.sum(axis=0)
    u = np.stack([(np.tensordot(c[:, a].astype(float), f, axes=(0, 0)) + sign * 0.5 * force[a]) / rho
                  for a in range(3)])
    return rho, u


def equilibrium(rho, u, q):
    c, w, _ = tables(q)
    usq = (u * u).sum(axis=0)
    out = np.empty((q,) + rho.shape)
    for i in range(q):
        cu = sum(c[i, a] * u[a] for a in range(3))
        out[i] = w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
    return out


def sensor(f, q, force, kind):
    rho, u = moments(f, q, force)
    feq = equilibrium(rho, u, q)
    fneq = f - feq
    if kind == 1:
        return np.abs(fneq / feq).sum(axis=0) / q
    return np.sqrt((fneq * fneq).sum(axis=0)) / np.sqrt((feq * feq).sum(axis=0))


def collide(f, q, tau, force):
    c, w, _ = tables(q)
    rho, u = moments(f, q, force)
    feq = equilibrium(rho, u, q)
    out = f - (f - feq) / tau
    if any(force):
        for i in range(q):
            cu = sum(c[i, a] * u[a] for a in range(3))
            Fi = sum((3.0 * (c[i, a] - u[a]) + 9.0 * cu * c[i, a]) * force[a] for a in range(3))
            out[i] += (1.0 - 0.5 / tau) * w[i] * Fi
    return out


def block_max(s, block):
    nz, ny, nx = s.shape
    bx, by, bz = block
    nb = ((nz + bz - 1) // bz, (ny + by - 1) // by, (nx + bx - 1) // bx)
    out = np.full(nb, -np.inf)
    for k in range(nb[0]):
        for j in range(nb[1]):
            for i in range(nb[2]):
                blk = s[k * bz:(k + 1) * bz, j * by:(j + 1) * by, i * bx:(i + 1) * bx]
                out[k, j, i] = np.nan if np.isnan(blk).any() else blk.max()
    return out


def run(S, q, n, bc, wall_u, tau, rho0, force, kind, block, k0, nsteps, sensor_every):
    """Returns (S_final, [(k, block_max), ...])."""
    hist = []
    for k in range(k0 + 1, k0 + nsteps + 1):
        f = stream(S, q, n, bc, wall_u, rho0)
        if sensor_every > 0 and k % sensor_every == 0:
            hist.append((k, block_max(sensor(f, q, force, kind), block)))
        S = collide(f, q, tau, force)
    return S, hist
