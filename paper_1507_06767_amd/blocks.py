"""``Blocks``: one lbm_blocks handle plus the torch tensors that back its
caller-owned device buffers.  Torch supplies device memory and the stream;
every computation is a call into liblbm.so."""
from __future__ import annotations

import numpy as np
import torch

from . import abi
from .abi import LbmError


def _check(st):
    if st != abi.LBM_OK:
        raise LbmError(st, abi.lbm_last_error())


class Blocks:
    """Owns the device buffers of one grid and the handle that steps it.

    desc: an ``abi.lbm_desc`` (see ``abi.make_desc``) whose buffer fields are
    filled here.  f0: optional float64 host state [q][nz][ny][nx].  The work is
    enqueued on ``stream`` (default: torch's current stream on ``device``).
    """

    def __init__(self, desc: abi.lbm_desc, f0=None, device="cuda", stream=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        st, sizes = abi.lbm_required_bytes(desc)
        _check(st)
        self._bufs = [torch.empty(int(n), dtype=torch.uint8, device=self.device) for n in sizes]
        for b, t in enumerate(self._bufs):
            desc.buf[b] = t.data_ptr()
            desc.buf_bytes[b] = t.numel()
        desc.stream = self.stream.cuda_stream
        self.desc = desc
        self.q = desc.lattice
        self.n = (desc.extent[0], desc.extent[1], desc.extent[2])
        self.cells, self.nblocks, self.dim = abi._counts(desc)
        self.nb = tuple((self.n[a] + desc.block[a] - 1) // desc.block[a] for a in range(3))
        if f0 is not None:
            f0 = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1)
        with torch.cuda.device(self.device):
            st, self.h = abi.lbm_create_blocks(desc, f0)
        _check(st)

    # ------------------------------------------------------------------
    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def step_n(self, n: int, sensor_every: int = 0):
        _check(abi.lbm_step_n(self.h, n, sensor_every))

    def sensor_flags(self):
        """(block_max [nbz,nby,nbx] float64, flags int8, step index, nonfinite)."""
        bm = np.empty(self.nblocks)
        fl = np.empty(self.nblocks, dtype=np.int8)
        st, step = abi.lbm_sensor_flags(self.h, self.nblocks, bm, fl)
        if st not in (abi.LBM_OK, abi.LBM_ENONFINITE):
            _check(st)
        shp = (self.nb[2], self.nb[1], self.nb[0])
        return bm.reshape(shp), fl.reshape(shp), step, st == abi.LBM_ENONFINITE

    def levels(self, a, b, lmin, lmax, buffer=0):
        """Refinement levels [nbz,nby,nbx] from the latest sensor step."""
        lev = np.empty(self.nblocks, dtype=np.int8)
        _check(abi.lbm_sensor_levels(self.h, self.nblocks, a, b, lmin, lmax, buffer, lev))
        return lev.reshape(self.nb[2], self.nb[1], self.nb[0])

    def average_begin(self):
        _check(abi.lbm_sensor_average_begin(self.h))

    def average(self):
        """(per-block max of the time-averaged cell sensor, samples)."""
        bm = np.empty(self.nblocks)
        st, n = abi.lbm_sensor_average(self.h, self.nblocks, bm)
        _check(st)
        return bm.reshape(self.nb[2], self.nb[1], self.nb[0]), n

    def average_end(self):
        _check(abi.lbm_sensor_average_end(self.h))

    def macros(self):
        rho = np.empty(self.cells)
        u = np.empty(3 * self.cells)
        _check(abi.lbm_get_macros(self.h, self.cells, rho, u))
        return rho.reshape(self.shape), u.reshape((3,) + self.shape)

    def block_means(self):
        """Per-block means of (rho - rho0, u_x, u_y, u_z), [nbz,nby,nbx,4]."""
        m = np.empty(4 * self.nblocks)
        _check(abi.lbm_block_means(self.h, self.nblocks, m))
        return m.reshape(self.nb[2], self.nb[1], self.nb[0], 4)

    def populations(self):
        f = np.empty(self.q * self.cells)
        _check(abi.lbm_get_populations(self.h, self.q, self.cells, f))
        return f.reshape((self.q,) + self.shape)

    def set_populations(self, f):
        _check(abi.lbm_set_populations(self.h, self.q, self.cells,
                                       np.ascontiguousarray(f, dtype=np.float64).reshape(-1)))

    def set_equilibrium(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        uu = None
        if u is not None:
            uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64)[:self.dim]).reshape(-1)
        _check(abi.lbm_set_equilibrium(self.h, self.cells, self.dim, r, uu))

    def conservation(self):
        st, out = abi.lbm_conservation(self.h)
        _check(st)
        return out

    @property
    def step(self):
        st, s = abi.lbm_get_step(self.h)
        _check(st)
        return s

    @step.setter
    def step(self, value: int):
        _check(abi.lbm_set_step(self.h, value))

    def use_graphs(self, chunk: int):
        """Replay runs of `chunk` (even) sensor-free steps from HIP graphs."""
        _check(abi.lbm_use_graphs(self.h, chunk))

    def autotune(self, reps: int = 5):
        """Times the tile widths of the step kernel and keeps the fastest."""
        st, tx = abi.lbm_autotune(self.h, reps)
        _check(st)
        return tx

    def scheme(self):
        """dict(inplace, next_is_gather, tile_x, multistep) of the handle."""
        st, ip, nxt, tx = abi.lbm_get_scheme(self.h)
        _check(st)
        st, ms = abi.lbm_get_multistep(self.h)
        _check(st)
        return {"inplace": bool(ip), "next_is_gather": bool(nxt), "tile_x": tx, "multistep": ms}

    def set_multistep(self, steps: int):
        """Most sensor-free steps per launch on small 2D grids (0: off)."""
        _check(abi.lbm_set_multistep(self.h, steps))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            abi.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
