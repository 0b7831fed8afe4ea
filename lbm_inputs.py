"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it draws random numbers and
describes workloads (sizes, boundary types, wall speeds, Reynolds numbers).
Everything the method computes from these inputs (relaxation times,
equilibria, steps) is done separately by the HIP library and by the oracle.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: value k of stream ``seed`` is mix64(seed + (k + 1) * gamma).  A
uniform double in [0, 1) takes the top 53 bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` consecutive SplitMix64 outputs of stream ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def velocity_perturbation(n, amplitude: float, seed: int, dims: int = 3) -> np.ndarray:
    """u of shape (3, nz, ny, nx): each of the first ``dims`` components iid
    uniform in [-amplitude, amplitude], component a drawn from offset a*cells."""
    nx, ny, nz = n
    cells = nx * ny * nz
    u = np.zeros((3, cells))
    for a in range(dims):
        u[a] = amplitude * (2.0 * uniform(seed, cells, offset=a * cells) - 1.0)
    return u.reshape(3, nz, ny, nx)


def random_populations(q: int, n, seed: int, lo: float = 0.01, hi: float = 0.2) -> np.ndarray:
    """Arbitrary positive populations (q, nz, ny, nx) uniform in [lo, hi): a
    generic, far-from-equilibrium state for single-step checks."""
    nx, ny, nz = n
    cells = nx * ny * nz
    return (lo + (hi - lo) * uniform(seed, q * cells)).reshape(q, nz, ny, nx)


def shear_wave(n, amplitude: float, axis_u: int = 0, axis_k: int = 1, periods: int = 1) -> np.ndarray:
    """u of shape (3, nz, ny, nx) with u[axis_u] = A sin(2 pi m j / L) along
    axis_k (node index j, box length L, m periods)."""
    nx, ny, nz = n
    L = n[axis_k]
    j = np.arange(L)
    prof = amplitude * np.sin(2.0 * np.pi * periods * j / L)
    shape = [1, 1, 1]
    shape[2 - axis_k] = L
    u = np.zeros((3, nz, ny, nx))
    u[axis_u] = np.broadcast_to(prof.reshape(shape), (nz, ny, nx))
    return u


# ---------------------------------------------------------------------------
# Workloads.  Face order -x,+x,-y,+y,-z,+z; 0 periodic, 1 wall.
# ---------------------------------------------------------------------------
PERIODIC, WALL = 0, 1


@dataclass
class Workload:
    name: str
    q: int
    n: tuple
    bc: tuple
    wall_u: tuple = ((0.0, 0.0, 0.0),) * 6
    reynolds: float = None        # with lid_speed and n_across, fixes tau
    lid_speed: float = 0.0
    n_across: int = 0
    tau: float = None             # given directly when reynolds is None
    force: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    sensor_every: int = 1
    theta_refine: float = 1e-3
    theta_coarsen: float = 5e-4
    storage: str = "f32"
    init: str = "rest"            # "rest" or "perturbed"
    perturb_amp: float = 0.0
    seed: int = 1
    block: tuple = None
    notes: str = ""

    def __post_init__(self):
        if self.block is None:
            self.block = (8, 8, 1) if self.q == 9 else (8, 8, 8)

    @property
    def cells(self):
        return self.n[0] * self.n[1] * self.n[2]


def _lid(speed):
    wu = [[0.0, 0.0, 0.0] for _ in range(6)]
    wu[3][0] = speed          # +y face moves in +x
    return tuple(tuple(v) for v in wu)


def cavity2d(n=64, lid=0.1, re=100.0, steps=2000, sensor_every=100):
    return Workload(name=f"cavity2d_d2q9_{n}x{n}_f64", q=9, n=(n, n, 1),
                    bc=(WALL, WALL, WALL, WALL, PERIODIC, PERIODIC), wall_u=_lid(lid),
                    reynolds=re, lid_speed=lid, n_across=n, steps=steps,
                    sensor_every=sensor_every, storage="f64")


def cavity3d(n=128, lid=0.05, re=1000.0, steps=5000, sensor_every=1, storage="f32"):
    return Workload(name=f"cavity3d_d3q19_{n}^3_{storage}", q=19, n=(n, n, n), bc=(WALL,) * 6,
                    wall_u=_lid(lid), reynolds=re, lid_speed=lid, n_across=n, steps=steps,
                    sensor_every=sensor_every, storage=storage)


def periodic_box(n=64, amp=0.01, tau=0.8, steps=5000, seed=1, storage="f32"):
    return Workload(name=f"box_d3q19_{n}^3_{storage}", q=19, n=(n, n, n), bc=(PERIODIC,) * 6,
                    tau=tau, steps=steps, storage=storage, init="perturbed", perturb_amp=amp,
                    seed=seed)


def channel3d(n=256, g=1e-6, tau=0.8, steps=10000, storage="f32", nx=None, nz=None):
    nx = n if nx is None else nx
    nz = n if nz is None else nz
    return Workload(name=f"channel_d3q19_{nx}x{n}x{nz}_{storage}", q=19, n=(nx, n, nz),
                    bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC), tau=tau,
                    force=(g, 0.0, 0.0), steps=steps, storage=storage)


def predictor_cavities(count: int, seed: int, n: int = 128, re_range=(1000.0, 5000.0), lid_range=(0.03, 0.08),
                       storage: str = "f32s"):
    """``count`` lid-driven 3D cavities for training and testing the flag
    predictor: Reynolds number and lid speed of cavity k drawn uniformly from
    the ranges (values 2k and 2k+1 of stream ``seed``)."""
    r = uniform(seed, 2 * count)
    out = []
    for k in range(count):
        re = re_range[0] + (re_range[1] - re_range[0]) * r[2 * k]
        lid = lid_range[0] + (lid_range[1] - lid_range[0]) * r[2 * k + 1]
        out.append(cavity3d(n=n, lid=lid, re=re, sensor_every=64, storage=storage))
    return out


def place_patches(flagged, block, n, count=400, edges=(16, 24, 32, 48), seed=7, margin=1):
    """``count`` non-overlapping cubic patch boxes for a two-level run,
    placed where a coarse run's sensor flags refinement.  ``flagged`` is the
    boolean block mask [nbz][nby][nbx] of the coarse grid (blocks of edge
    ``block``, grid extent ``n`` = (nx, ny, nz)).  Patch k has fine edge
    edges[r_k] (r_k from the stream ``seed``), i.e. a coarse edge ce of half
    that, with its origin on a multiple of 4 coarse cells and at least
    ``margin`` cells from the domain faces.  It goes on the flagged blocks in
    a seeded order, starting after the block of the previous patch: on the
    first block where a free position exists, at the free origin whose box
    overlaps that block and whose centre lies nearest the block's centre
    (ties: lowest z, then y, then x).  When no flagged block has room left,
    the mask grows by one block in every direction (the buffer layer around
    tagged cells of Sec. 5.2) and the search goes on.  Raises ValueError if
    the grid cannot hold ``count`` boxes.  Returns
    [((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z))] in coarse cells."""
    flagged = np.asarray(flagged, dtype=bool)
    if count == 0:
        return []
    if not flagged.any():
        raise ValueError("no flagged block to place patches on")
    assert block % 4 == 0 and all(e % 8 == 0 for e in edges)
    pick = (uniform(seed + 1, count) * len(edges)).astype(np.int64)
    # occupancy in units of 4 coarse cells (every box is 4-aligned); a box is
    # free when its sum over the summed-volume table is zero
    lo4_min = (margin + 3) // 4
    hi4_max = [(n[a] - margin) // 4 for a in range(3)]
    occ = np.zeros((n[2] // 4 + 1, n[1] // 4 + 1, n[0] // 4 + 1), dtype=np.int32)   # [z][y][x]
    b4 = block // 4

    def table():
        t = np.zeros(tuple(d + 1 for d in occ.shape), dtype=np.int32)
        t[1:, 1:, 1:] = occ.cumsum(0).cumsum(1).cumsum(2)
        return t

    def box_sums(t, lo, e):            # lo: (k, 3) in x, y, z units of 4 cells
        x0, y0, z0 = lo[:, 0], lo[:, 1], lo[:, 2]
        x1, y1, z1 = x0 + e, y0 + e, z0 + e
        return (t[z1, y1, x1] - t[z0, y1, x1] - t[z1, y0, x1] - t[z1, y1, x0]
                + t[z0, y0, x1] + t[z0, y1, x0] + t[z1, y0, x0] - t[z0, y0, x0])

    def candidates(b, e4):             # b: block (x, y, z); origins whose box overlaps it, nearest first
        rng = []
        for a in range(3):
            lo = max(b[a] * b4 - e4 + 1, lo4_min)
            hi = min(b[a] * b4 + b4 - 1, hi4_max[a] - e4)
            if hi < lo:
                return None
            rng.append(np.arange(lo, hi + 1))
        gz, gy, gx = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        c = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        centre = 2 * np.asarray(b) * b4 + b4            # twice the block centre, units of 4 cells
        d2 = ((2 * c + e4 - centre) ** 2).sum(axis=1)
        return c[np.lexsort((c[:, 0], c[:, 1], c[:, 2], d2))]

    masks = [flagged]
    orders, cursors, failed = [], [], [set()]
    boxes = []
    t = table()
    k = 0
    p = 0
    while k < count:
        if p == len(orders):
            blocks = np.argwhere(masks[p])[:, ::-1]            # (x, y, z) block indices
            orders.append(blocks[np.argsort(uniform(seed + 2 + p, len(blocks)), kind="stable")])
            cursors.append(0)
        e4 = edges[pick[k]] // 8                                # coarse edge / 4
        order = orders[p]
        placed = False
        for j in range(len(order)):
            idx = (cursors[p] + j) % len(order)
            b = tuple(int(v) for v in order[idx])
            if any((b, e) in failed[p] for e in range(1, e4 + 1)):
                continue
            c = candidates(b, e4)
            free = None if c is None else np.flatnonzero(box_sums(t, c, e4) == 0)
            if free is None or len(free) == 0:
                failed[p].add((b, e4))
                continue
            lo = c[free[0]]
            occ[lo[2]:lo[2] + e4, lo[1]:lo[1] + e4, lo[0]:lo[0] + e4] = 1
            t = table()
            boxes.append((tuple(int(4 * v) for v in lo), tuple(int(4 * (v + e4)) for v in lo)))
            cursors[p] = (idx + 1) % len(order)
            placed = True
            break
        if placed:
            k += 1
            p = 0
            continue
        p += 1
        if p == len(masks):
            grown = masks[-1].copy()
            for ax in range(3):                             # one block in every direction
                g = grown.copy()
                sl_lo = [slice(None)] * 3
                sl_hi = [slice(None)] * 3
                sl_lo[ax], sl_hi[ax] = slice(1, None), slice(None, -1)
                g[tuple(sl_lo)] |= grown[tuple(sl_hi)]
                g[tuple(sl_hi)] |= grown[tuple(sl_lo)]
                grown = g
            if grown.sum() == masks[-1].sum():
                raise ValueError(f"only {len(boxes)} of {count} patches fit on the grid")
            masks.append(grown)
            failed.append(set())
    return boxes
