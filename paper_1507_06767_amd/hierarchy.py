"""``Hierarchy``: fine patches (refinement factor 2) over the grid of a
``Blocks`` handle, with the caller-owned device buffers as torch tensors.
Every computation is a call into liblbm.so (lbm_create_hierarchy and
friends)."""
from __future__ import annotations

import numpy as np
import torch

from . import abi
from .abi import LbmError


def _check(st):
    if st != abi.LBM_OK:
        raise LbmError(st, abi.lbm_last_error())


class Hierarchy:
    """boxes: list of ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z)) in coarse
    cells.  The coarse ``Blocks`` must stream ping-pong; give it a non-default
    torch stream to replay steps from a HIP graph."""

    def __init__(self, coarse, boxes, use_graph=True):
        self.coarse = coarse
        self.boxes = [(tuple(int(v) for v in lo), tuple(int(v) for v in hi)) for lo, hi in boxes]
        st, sizes = abi.lbm_hierarchy_required_bytes(coarse.h, self.boxes)
        _check(st)
        self._bufs = [torch.empty(int(n), dtype=torch.uint8, device=coarse.device) for n in sizes]
        with torch.cuda.device(coarse.device):
            st, self.h = abi.lbm_create_hierarchy(coarse.h, self.boxes, [t.data_ptr() for t in self._bufs],
                                                  [t.numel() for t in self._bufs], use_graph)
        _check(st)
        self.q = coarse.q
        self.extents = [tuple(2 * (hi[a] - lo[a]) for a in range(3)) for lo, hi in self.boxes]
        st, self.fine_cells, self.nblocks, self.n_eff, self.tau_fine, _, _ = abi.lbm_hierarchy_info(self.h)
        _check(st)

    def step_n(self, n: int, sensor_every: int = 0):
        _check(abi.lbm_hierarchy_step(self.h, n, sensor_every))

    def sensor(self):
        """(fine block maxima, flags, coarse step index), blocks patch by
        patch, x fastest within a patch."""
        bm = np.empty(self.nblocks)
        fl = np.empty(self.nblocks, dtype=np.int8)
        st, step = abi.lbm_hierarchy_sensor(self.h, self.nblocks, bm, fl)
        _check(st)
        return bm, fl, step

    def patch_fields(self, p: int):
        """(rho, u, f) of patch p's interior: [z][y][x], [3][z][y][x], [q][z][y][x]."""
        ex, ey, ez = self.extents[p]
        n = ex * ey * ez
        rho, u, f = np.empty(n), np.empty(3 * n), np.empty(self.q * n)
        _check(abi.lbm_hierarchy_patch_fields(self.h, p, n, self.q, rho, u, f))
        shp = (ez, ey, ex)
        return rho.reshape(shp), u.reshape((3,) + shp), f.reshape((self.q,) + shp)

    def info(self):
        st, fc, fb, ne, tf, tz, wg = abi.lbm_hierarchy_info(self.h)
        _check(st)
        return {"fine_cells": fc, "fine_blocks": fb, "n_eff": ne, "tau_fine": tf, "tile_x": tz,
                "workgroups": wg}

    def autotune(self, reps: int = 5):
        """(widest tile, workgroups, microseconds per fine step) of the
        fastest fine-step configuration, which is kept."""
        st, tz, wg, us = abi.lbm_hierarchy_autotune(self.h, reps)
        _check(st)
        return tz, wg, us

    def profile(self, steps: int = 4):
        """Advances `steps` coarse steps launched one by one and returns mean
        microseconds, timed with HIP events in production order: "coarse"
        (the coarse step), "ghosts" (one ghost fill), "fine" (the first fine
        step) and "fine_restrict" (the second fine step, which also
        restricts to the coarse level)."""
        st, us = abi.lbm_hierarchy_profile(self.h, steps)
        _check(st)
        return dict(zip(("coarse", "ghosts", "fine", "fine_restrict"), us))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            abi.lbm_destroy_hierarchy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
