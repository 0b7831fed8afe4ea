"""FP64 CPU oracle for the BGK step and the kinetic refinement sensor.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It is the plain,
slow reference the HIP library is checked against and shares nothing with it:
the arithmetic lives in ``orc.c`` (push streaming, cell-major storage, its own
enumerated velocity order) and in ``brute.py`` (an independent numpy pull
implementation used to cross-check ``orc.c`` on tiny grids).

Populations cross this wrapper in the library's interface layout: float64
arrays of shape ``(q, nz, ny, nx)`` (x fastest) in the interface velocity
order, which ``ABI_VELOCITIES`` lists.  Internally ``orc.c`` keeps
``(cells, q)`` in its own order; the permutation between the two is found by
matching velocity vectors.

Parts with "parity unpinned": none of the functions here lacks a pin; the
pins are listed in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

# Interface velocity order (the library header fixes it; it is an interface
# table, restated here, not shared).  Opposite of index i: i+1 for odd i,
# i-1 for even i > 0.
ABI_VELOCITIES = {
    9: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)],
    19: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
    27: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
         (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
         (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)],
}

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")
PERIODIC, WALL = 0, 1
SENSOR_L2, SENSOR_KKN = 0, 1


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("sensor_kind", ctypes.c_int32),
        ("block", ctypes.c_int32 * 3),
        ("theta_refine", ctypes.c_double),
        ("theta_coarsen", ctypes.c_double),
        ("smagorinsky", ctypes.c_double),
        ("wall_profile", ctypes.c_int32 * 6),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Params)
        lib.orc_lattice_tables.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp,
                                           ctypes.POINTER(ctypes.c_int)]
        lib.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        for name in ("orc_stream", "orc_sensor", "orc_collide", "orc_block_max"):
            getattr(lib, name).argtypes = [P, dp, dp]
        lib.orc_moments.argtypes = [P, dp, ctypes.c_double, dp, dp]
        lib.orc_flags.argtypes = [P, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int8)]
        lib.orc_step.argtypes = [P, dp, dp, dp, dp]
        lib.orc_run.argtypes = [P, dp, dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, dp]
        lib.orc_run.restype = ctypes.c_int64
        lib.orc_conservation.argtypes = [P, dp, dp]
        lib.orc_equilibrium_field.argtypes = [P, dp, dp, dp]
        lib.orc_levels.argtypes = [P, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int8)]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice_tables(q: int):
    """(c[q,3] int, w[q] float64, opp[q] int, d) in the oracle's own order."""
    lib = _load()
    c = (ctypes.c_int * (3 * q))()
    w = np.zeros(q)
    opp = (ctypes.c_int * q)()
    d = lib.orc_lattice_tables(q, c, _dp(w), opp)
    if d < 0:
        raise ValueError(f"unsupported lattice q={q}")
    return np.array(list(c)).reshape(q, 3), w, np.array(list(opp)), d


def abi_permutation(q: int) -> np.ndarray:
    """perm[j] = oracle index of interface velocity j."""
    c, _, _, _ = lattice_tables(q)
    perm = []
    for v in ABI_VELOCITIES[q]:
        hits = [i for i in range(q) if tuple(c[i]) == v]
        assert len(hits) == 1
        perm.append(hits[0])
    return np.array(perm)


def equilibrium(q: int, rho: float, u) -> np.ndarray:
    """f^eq in interface order for one cell (Eq. feq_i)."""
    lib = _load()
    feq = np.zeros(q)
    uu = np.ascontiguousarray(np.asarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64))
    lib.orc_equilibrium(q, float(rho), _dp(uu), _dp(feq))
    return feq[abi_permutation(q)]


@dataclass
class Grid:
    """One uniform grid with its boundary conditions and method parameters."""
    q: int
    n: tuple                      # (nx, ny, nz)
    bc: tuple = (PERIODIC,) * 6   # -x,+x,-y,+y,-z,+z
    wall_u: tuple = ((0.0, 0.0, 0.0),) * 6
    tau: float = 0.8
    rho0: float = 1.0
    force: tuple = (0.0, 0.0, 0.0)
    sensor_kind: int = SENSOR_L2
    block: tuple = None
    theta_refine: float = 1e-3
    theta_coarsen: float = 5e-4
    smagorinsky: float = 0.0
    wall_profile: tuple = (0,) * 6
    _p: _Params = field(default=None, init=False, repr=False)

    def __post_init__(self):
        if self.block is None:
            self.block = (8, 8, 1) if self.q == 9 else (8, 8, 8)
        p = _Params()
        p.q = self.q
        for a in range(3):
            p.n[a] = int(self.n[a])
            p.force[a] = float(self.force[a])
            p.block[a] = int(self.block[a])
        for k in range(6):
            p.bc[k] = int(self.bc[k])
            for a in range(3):
                p.wall_u[k][a] = float(self.wall_u[k][a])
        p.tau, p.rho0 = float(self.tau), float(self.rho0)
        p.sensor_kind = int(self.sensor_kind)
        p.theta_refine, p.theta_coarsen = float(self.theta_refine), float(self.theta_coarsen)
        p.smagorinsky = float(self.smagorinsky)
        for k in range(6):
            p.wall_profile[k] = int(self.wall_profile[k])
        self._p = p
        self._perm = abi_permutation(self.q)      # interface index -> oracle index
        self._inv = np.argsort(self._perm)         # oracle index -> interface index

    # -- layout -----------------------------------------------------------------
    @property
    def cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def nblocks(self):
        return tuple((self.n[a] + self.block[a] - 1) // self.block[a] for a in range(3))

    def to_internal(self, f_abi: np.ndarray) -> np.ndarray:
        """(q, nz, ny, nx) interface order -> (cells, q) oracle order."""
        f_abi = np.asarray(f_abi, dtype=np.float64).reshape(self.q, self.cells)
        return np.ascontiguousarray(f_abi[self._inv].T)

    def to_abi(self, f_int: np.ndarray) -> np.ndarray:
        """(cells, q) oracle order -> (q, nz, ny, nx) interface order."""
        return np.ascontiguousarray(f_int[:, self._perm].T).reshape((self.q,) + self.shape)

    # -- states -----------------------------------------------------------------
    def equilibrium_state(self, rho=None, u=None) -> np.ndarray:
        """Interface-layout f^eq(rho, u) per cell; rho (cells) and u (3, cells)
        default to rho0 and 0."""
        N = self.cells
        rho = np.full(N, self.rho0) if rho is None else np.asarray(rho, dtype=np.float64).reshape(N)
        u = np.zeros((3, N)) if u is None else np.asarray(u, dtype=np.float64).reshape(-1, N)
        if u.shape[0] < 3:
            u = np.vstack([u, np.zeros((3 - u.shape[0], N))])
        rho = np.ascontiguousarray(rho)
        uc = np.ascontiguousarray(u[:3].T)
        out = np.empty((N, self.q))
        assert _load().orc_equilibrium_field(ctypes.byref(self._p), _dp(rho), _dp(uc), _dp(out)) == 0
        return self.to_abi(out)

    # -- the step ---------------------------------------------------------------
    def stream(self, S_abi):
        S = self.to_internal(S_abi)
        f = np.empty_like(S)
        assert _load().orc_stream(ctypes.byref(self._p), _dp(S), _dp(f)) == 0
        return self.to_abi(f)

    def collide(self, f_abi):
        f = self.to_internal(f_abi)
        S = np.empty_like(f)
        assert _load().orc_collide(ctypes.byref(self._p), _dp(f), _dp(S)) == 0
        return self.to_abi(S)

    def sensor(self, f_abi):
        """Cell sensor on pre-collision populations, shape (nz, ny, nx)."""
        f = self.to_internal(f_abi)
        s = np.empty(self.cells)
        assert _load().orc_sensor(ctypes.byref(self._p), _dp(f), _dp(s)) == 0
        return s.reshape(self.shape)

    def block_max(self, s):
        s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(self.cells))
        nb = self.nblocks
        out = np.empty(nb[0] * nb[1] * nb[2])
        assert _load().orc_block_max(ctypes.byref(self._p), _dp(s), _dp(out)) == 0
        return out.reshape(nb[2], nb[1], nb[0])

    def flags(self, bmax):
        bmax = np.ascontiguousarray(np.asarray(bmax, dtype=np.float64).ravel())
        out = np.empty(bmax.size, dtype=np.int8)
        _load().orc_flags(ctypes.byref(self._p), _dp(bmax), bmax.size,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        return out.reshape(self.nblocks[::-1])

    def levels(self, bmax, a, b, lmin, lmax, buffer=0):
        """Refinement level per block from block maxima (Sec. 3.4), dilated by
        `buffer` blocks (the buffer layer of Sec. 5.2)."""
        bmax = np.ascontiguousarray(np.asarray(bmax, dtype=np.float64).ravel())
        out = np.empty(bmax.size, dtype=np.int8)
        assert _load().orc_levels(ctypes.byref(self._p), _dp(bmax), float(a), float(b), int(lmin),
                                  int(lmax), int(buffer),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))) == 0
        return out.reshape(self.nblocks[::-1])

    def sensor_history(self, S_abi, k0, n, every, start):
        """Runs n steps from S_{k0}; returns (S, mean cell sensor over the
        sensor steps k > start, number of samples): the time average of the
        sensor that Sec. 5.1 builds its mesh from."""
        S = S_abi
        acc, cnt = None, 0
        for k in range(k0 + 1, k0 + n + 1):
            f = self.stream(S)
            if every > 0 and k % every == 0 and k > start:
                s = self.sensor(f)
                acc = s if acc is None else acc + s
                cnt += 1
            S = self.collide(f)
        return S, (acc / cnt if cnt else None), cnt

    def macros(self, f_abi, post_collision=True):
        """(rho (nz,ny,nx), u (3,nz,ny,nx)); u of the stored post-collision
        state carries -F/2, of pre-collision populations +F/2."""
        f = self.to_internal(f_abi)
        rho = np.empty(self.cells)
        u = np.empty((self.cells, 3))
        _load().orc_moments(ctypes.byref(self._p), _dp(f), -1.0 if post_collision else 1.0,
                            _dp(rho), _dp(u))
        return rho.reshape(self.shape), np.ascontiguousarray(u.T).reshape((3,) + self.shape)

    def conservation(self, S_abi):
        S = self.to_internal(S_abi)
        out = np.zeros(4)
        _load().orc_conservation(ctypes.byref(self._p), _dp(S), _dp(out))
        return out

    def run(self, S_abi, k0: int, n: int, sensor_every: int, keep_history: bool = True):
        """Advance n steps from state S_{k0}.  Returns (S_{k0+n}, history),
        history = list of (k, block_max, flags) for each sensor step."""
        S = self.to_internal(S_abi)
        work = np.empty(2 * S.size + self.cells)
        sens_steps = [k for k in range(k0 + 1, k0 + n + 1)
                      if sensor_every > 0 and k % sensor_every == 0]
        nb = self.nblocks
        NB = nb[0] * nb[1] * nb[2]
        hist = np.empty(max(1, len(sens_steps)) * NB) if keep_history else None
        got = _load().orc_run(ctypes.byref(self._p), _dp(S), _dp(work), k0, n, sensor_every,
                              _dp(hist) if keep_history else None)
        assert got == len(sens_steps), (got, sens_steps)
        history = []
        if keep_history:
            for j, k in enumerate(sens_steps):
                bm = hist[j * NB:(j + 1) * NB].reshape(nb[2], nb[1], nb[0]).copy()
                history.append((k, bm, self.flags(bm)))
        return self.to_abi(S), history


def threads() -> int:
    """Threads the oracle's OpenMP loops currently use."""
    return int(_load().orc_max_threads())


def set_threads(n: int) -> int:
    """Threads the oracle's OpenMP loops use from now on; returns the previous count."""
    lib = _load()
    prev = lib.orc_max_threads()
    assert lib.orc_set_threads(int(n)) == 0
    return prev


def tau_from_reynolds(u: float, n_cells: float, re: float) -> float:
    """tau = nu / c_s^2 + 1/2 with nu = u N / Re (Eq. nu_omega, c_s^2 = 1/3)."""
    nu = u * n_cells / re
    return nu / (1.0 / 3.0) + 0.5
