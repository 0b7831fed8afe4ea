"""ctypes binding of include/lbm.h: same names, argument marshalling only.

Every function returns the C status code (0 = LBM_OK, < 0 = error), plus any
output the C function writes through a pointer.  Host arrays are numpy
arrays; their dtype, contiguity and size are checked here before the call
so that the C side never writes past a host buffer.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_ABI_VERSION = 2
LBM_OK, LBM_EINVAL, LBM_ENOTSUP, LBM_EHIP, LBM_ESTATE, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5
LBM_D2Q9, LBM_D3Q19, LBM_D3Q27 = 9, 19, 27
LBM_F64, LBM_F32, LBM_F32_SHIFTED, LBM_F16_SHIFTED, LBM_BF16_SHIFTED = 0, 1, 2, 3, 4
LBM_F16_SHIFTED_SR, LBM_BF16_SHIFTED_SR = 5, 6
LBM_SENSOR_L2, LBM_SENSOR_KKN = 0, 1
LBM_BC_PERIODIC, LBM_BC_WALL = 0, 1
LBM_PROFILE_UNIFORM, LBM_PROFILE_SMOOTH = 0, 1
LBM_STREAMING_AUTO, LBM_STREAMING_PINGPONG, LBM_STREAMING_INPLACE = 0, 1, 2
LBM_NBUF = 5
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOTSUP", -3: "LBM_EHIP",
                -4: "LBM_ESTATE", -5: "LBM_ENONFINITE"}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lbm_desc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("lattice", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("sensor_kind", ctypes.c_int32),
        ("extent", ctypes.c_int32 * 3),
        ("block", ctypes.c_int32 * 3),
        ("face_bc", ctypes.c_int32 * 6),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("theta_refine", ctypes.c_double),
        ("theta_coarsen", ctypes.c_double),
        ("smagorinsky", ctypes.c_double),
        ("wall_profile", ctypes.c_int32 * 6),
        ("streaming", ctypes.c_int32),
        ("buf", ctypes.c_void_p * LBM_NBUF),
        ("buf_bytes", ctypes.c_size_t * LBM_NBUF),
        ("stream", ctypes.c_void_p),
    ]


LBM_NHBUF = 5


class lbm_box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


def library_path() -> str:
    return _LIB_PATH


def _load_library():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch loads its bundled HIP runtime by the file name libamdhip64.so; the
    # library asks for the soname libamdhip64.so.7, which that copy carries.
    # Loading torch first makes both use one runtime: loaded the other way
    # round, two runtimes would coexist and neither would know the other's
    # device pointers.
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    H = ctypes.c_void_p
    D = ctypes.POINTER(lbm_desc)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lbm_required_bytes": [D, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_create_blocks": [D, dp, ctypes.POINTER(H)],
        "lbm_step_n": [H, ctypes.c_int64, ctypes.c_int32],
        "lbm_sensor_flags": [H, dp, ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(ctypes.c_int64)],
        "lbm_get_macros": [H, dp, dp],
        "lbm_block_means": [H, dp],
        "lbm_get_populations": [H, dp],
        "lbm_set_populations": [H, dp],
        "lbm_set_equilibrium": [H, dp, dp],
        "lbm_get_step": [H, ctypes.POINTER(ctypes.c_int64)],
        "lbm_set_multistep": [H, ctypes.c_int32],
        "lbm_get_multistep": [H, ctypes.POINTER(ctypes.c_int32)],
        "lbm_get_scheme": [H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)],
        "lbm_set_step": [H, ctypes.c_int64],
        "lbm_sensor_levels": [H, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, ctypes.POINTER(ctypes.c_int8)],
        "lbm_sensor_average_begin": [H],
        "lbm_sensor_average": [H, dp, ctypes.POINTER(ctypes.c_int64)],
        "lbm_sensor_average_end": [H],
        "lbm_conservation": [H, dp],
        "lbm_conservation_noalloc": [H, dp],
        "lbm_tau_from_reynolds": [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp],
    }
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    BP = ctypes.POINTER(lbm_box)
    sig.update({
        "lbm_autotune": [H, ctypes.c_int32, i32p],
        "lbm_use_graphs": [H, ctypes.c_int32],
        "lbm_hierarchy_required_bytes": [H, ctypes.c_int32, BP, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_create_hierarchy": [H, ctypes.c_int32, BP, ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.POINTER(ctypes.c_size_t), ctypes.c_int32, ctypes.POINTER(H)],
        "lbm_hierarchy_step": [H, ctypes.c_int64, ctypes.c_int32],
        "lbm_hierarchy_sensor": [H, dp, ctypes.POINTER(ctypes.c_int8), i64p],
        "lbm_hierarchy_patch_fields": [H, ctypes.c_int32, dp, dp, dp],
        "lbm_hierarchy_info": [H, i64p, i64p, dp, dp, i32p, i32p],
        "lbm_hierarchy_autotune": [H, ctypes.c_int32, i32p, i32p, dp],
        "lbm_hierarchy_profile": [H, ctypes.c_int32, dp],
    })
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.lbm_destroy.argtypes = [H]
    lib.lbm_destroy.restype = None
    lib.lbm_destroy_hierarchy.argtypes = [H]
    lib.lbm_destroy_hierarchy.restype = None
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load_library()


def _dptr(a, n=None):
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError("host arrays must be C-contiguous float64 numpy arrays")
    if n is not None and a.size != n:
        raise ValueError(f"host array has {a.size} values, needs {n}")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _counts(desc: lbm_desc):
    cells = desc.extent[0] * desc.extent[1] * desc.extent[2]
    nb = [(desc.extent[a] + desc.block[a] - 1) // max(desc.block[a], 1) for a in range(3)]
    dim = 2 if desc.lattice == LBM_D2Q9 else 3
    return cells, nb[0] * nb[1] * nb[2], dim


def make_desc(lattice, extent, face_bc, tau, storage=LBM_F32, sensor_kind=LBM_SENSOR_L2,
              wall_u=None, rho0=1.0, force=(0.0, 0.0, 0.0), theta_refine=1e-3,
              theta_coarsen=5e-4, block=None, smagorinsky=0.0, wall_profile=None,
              streaming=LBM_STREAMING_AUTO) -> lbm_desc:
    """A descriptor with the buffers left empty."""
    d = lbm_desc()
    d.abi_version = LBM_ABI_VERSION
    d.lattice, d.storage, d.sensor_kind = lattice, storage, sensor_kind
    if block is None:
        block = (8, 8, 1) if lattice == LBM_D2Q9 else (8, 8, 8)
    for a in range(3):
        d.extent[a], d.block[a], d.force[a] = int(extent[a]), int(block[a]), float(force[a])
    for f in range(6):
        d.face_bc[f] = int(face_bc[f])
        for a in range(3):
            d.wall_u[f][a] = float(wall_u[f][a]) if wall_u is not None else 0.0
    d.tau, d.rho0 = float(tau), float(rho0)
    d.theta_refine, d.theta_coarsen = float(theta_refine), float(theta_coarsen)
    d.smagorinsky = float(smagorinsky)
    for f in range(6):
        d.wall_profile[f] = int(wall_profile[f]) if wall_profile is not None else LBM_PROFILE_UNIFORM
    d.streaming = int(streaming)
    return d


def lbm_last_error() -> str:
    return _lib.lbm_last_error().decode()


def lbm_required_bytes(desc: lbm_desc):
    out = (ctypes.c_size_t * LBM_NBUF)()
    st = _lib.lbm_required_bytes(ctypes.byref(desc), out)
    return st, list(out)


def lbm_create_blocks(desc: lbm_desc, f0=None):
    cells, _, _ = _counts(desc)
    h = ctypes.c_void_p()
    st = _lib.lbm_create_blocks(ctypes.byref(desc), _dptr(f0, desc.lattice * cells), ctypes.byref(h))
    return st, h


def lbm_step_n(h, n: int, sensor_every: int):
    return _lib.lbm_step_n(h, int(n), int(sensor_every))


def lbm_sensor_flags(h, nblocks: int, block_max=None, flags=None):
    """block_max: float64[nblocks] or None; flags: int8[nblocks] or None."""
    if flags is not None and not (isinstance(flags, np.ndarray) and flags.dtype == np.int8
                                  and flags.flags.c_contiguous and flags.size == nblocks):
        raise TypeError("flags must be a C-contiguous int8 array of nblocks values")
    step = ctypes.c_int64(-1)
    fp = flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)) if flags is not None else None
    st = _lib.lbm_sensor_flags(h, _dptr(block_max, nblocks), fp, ctypes.byref(step))
    return st, step.value


def lbm_get_macros(h, cells: int, rho=None, u=None):
    return _lib.lbm_get_macros(h, _dptr(rho, cells), _dptr(u, 3 * cells))


def lbm_block_means(h, nblocks: int, means):
    """means: float64[nblocks * 4] (rho - rho0, u_x, u_y, u_z per block)."""
    return _lib.lbm_block_means(h, _dptr(means, 4 * nblocks))


def lbm_get_populations(h, q: int, cells: int, f):
    return _lib.lbm_get_populations(h, _dptr(f, q * cells))


def lbm_set_populations(h, q: int, cells: int, f):
    return _lib.lbm_set_populations(h, _dptr(f, q * cells))


def lbm_set_equilibrium(h, cells: int, dim: int, rho=None, u=None):
    return _lib.lbm_set_equilibrium(h, _dptr(rho, cells), _dptr(u, dim * cells))


def lbm_get_step(h):
    s = ctypes.c_int64(0)
    st = _lib.lbm_get_step(h, ctypes.byref(s))
    return st, s.value


def lbm_set_multistep(h, steps: int):
    return _lib.lbm_set_multistep(h, steps)


def lbm_get_multistep(h):
    s = ctypes.c_int32(0)
    st = _lib.lbm_get_multistep(h, ctypes.byref(s))
    return st, s.value


def lbm_get_scheme(h):
    """(status, inplace, next_is_gather, tile_x)."""
    a, b, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    st = _lib.lbm_get_scheme(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return st, a.value, b.value, c.value


def lbm_sensor_levels(h, nblocks: int, a: float, b: float, lmin: int, lmax: int, buffer: int, levels):
    if not (isinstance(levels, np.ndarray) and levels.dtype == np.int8 and levels.flags.c_contiguous
            and levels.size == nblocks):
        raise TypeError("levels must be a C-contiguous int8 array of nblocks values")
    return _lib.lbm_sensor_levels(h, float(a), float(b), int(lmin), int(lmax), int(buffer),
                                  levels.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))


def lbm_sensor_average_begin(h):
    return _lib.lbm_sensor_average_begin(h)


def lbm_sensor_average(h, nblocks: int, block_max=None):
    n = ctypes.c_int64(0)
    st = _lib.lbm_sensor_average(h, _dptr(block_max, nblocks), ctypes.byref(n))
    return st, n.value


def lbm_sensor_average_end(h):
    return _lib.lbm_sensor_average_end(h)


def lbm_set_step(h, step: int):
    return _lib.lbm_set_step(h, int(step))


def lbm_conservation(h):
    out = np.zeros(4)
    st = _lib.lbm_conservation(h, _dptr(out))
    return st, out


def lbm_conservation_noalloc(h):
    out = np.zeros(4)
    st = _lib.lbm_conservation_noalloc(h, _dptr(out))
    return st, out


def lbm_tau_from_reynolds(u: float, n_across: float, re: float):
    t = ctypes.c_double(0.0)
    st = _lib.lbm_tau_from_reynolds(float(u), float(n_across), float(re), ctypes.byref(t))
    return st, t.value


def lbm_destroy(h):
    _lib.lbm_destroy(h)


def lbm_use_graphs(h, chunk: int):
    return _lib.lbm_use_graphs(h, int(chunk))


def lbm_autotune(h, reps: int):
    t = ctypes.c_int32(0)
    st = _lib.lbm_autotune(h, int(reps), ctypes.byref(t))
    return st, t.value


def _boxes(boxes):
    arr = (lbm_box * len(boxes))()
    for k, (lo, hi) in enumerate(boxes):
        for a in range(3):
            arr[k].lo[a], arr[k].hi[a] = int(lo[a]), int(hi[a])
    return arr


def lbm_hierarchy_required_bytes(h, boxes):
    out = (ctypes.c_size_t * LBM_NHBUF)()
    st = _lib.lbm_hierarchy_required_bytes(h, len(boxes), _boxes(boxes), out)
    return st, list(out)


def lbm_create_hierarchy(h, boxes, bufs, buf_bytes, use_graph: bool):
    """bufs: LBM_NHBUF device addresses; buf_bytes: their sizes."""
    pb = (ctypes.c_void_p * LBM_NHBUF)(*bufs)
    pn = (ctypes.c_size_t * LBM_NHBUF)(*buf_bytes)
    H = ctypes.c_void_p()
    st = _lib.lbm_create_hierarchy(h, len(boxes), _boxes(boxes), pb, pn, int(bool(use_graph)), ctypes.byref(H))
    return st, H


def lbm_hierarchy_step(H, n: int, sensor_every: int):
    return _lib.lbm_hierarchy_step(H, int(n), int(sensor_every))


def lbm_hierarchy_sensor(H, nblocks: int, block_max=None, flags=None):
    if flags is not None and not (isinstance(flags, np.ndarray) and flags.dtype == np.int8
                                  and flags.flags.c_contiguous and flags.size == nblocks):
        raise TypeError("flags must be a C-contiguous int8 array of nblocks values")
    step = ctypes.c_int64(-1)
    fp = flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)) if flags is not None else None
    st = _lib.lbm_hierarchy_sensor(H, _dptr(block_max, nblocks), fp, ctypes.byref(step))
    return st, step.value


def lbm_hierarchy_patch_fields(H, patch: int, cells: int, q: int, rho=None, u=None, f=None):
    return _lib.lbm_hierarchy_patch_fields(H, int(patch), _dptr(rho, cells), _dptr(u, 3 * cells),
                                           _dptr(f, q * cells))


def lbm_hierarchy_info(H):
    """(status, fine_cells, fine_blocks, n_eff, tau_fine, tile_z, workgroups)."""
    fc, fb = ctypes.c_int64(0), ctypes.c_int64(0)
    ne, tf = ctypes.c_double(0.0), ctypes.c_double(0.0)
    tz, wg = ctypes.c_int32(0), ctypes.c_int32(0)
    st = _lib.lbm_hierarchy_info(H, ctypes.byref(fc), ctypes.byref(fb), ctypes.byref(ne), ctypes.byref(tf),
                                 ctypes.byref(tz), ctypes.byref(wg))
    return st, fc.value, fb.value, ne.value, tf.value, tz.value, wg.value


def lbm_hierarchy_autotune(H, reps: int):
    """(status, tile_x, workgroups, fine step microseconds)."""
    tz, wg, us = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    st = _lib.lbm_hierarchy_autotune(H, int(reps), ctypes.byref(tz), ctypes.byref(wg), ctypes.byref(us))
    return st, tz.value, wg.value, us.value


def lbm_hierarchy_profile(H, steps: int):
    """(status, [coarse step, ghost fill, first fine step, second fine step with the
    restriction] microseconds)."""
    us = (ctypes.c_double * 4)()
    st = _lib.lbm_hierarchy_profile(H, int(steps), us)
    return st, list(us)


def lbm_destroy_hierarchy(H):
    _lib.lbm_destroy_hierarchy(H)
