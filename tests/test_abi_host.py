"""Host-side checks of the C interface: the library loads, exports every
function the header declares, and rejects bad descriptors before touching
the GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


@pytest.fixture(scope="module")
def lbm():
    import paper_1507_06767_amd as lbm
    return lbm


def _declared_functions(headers=None):
    names = set()
    for path in headers or HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names.update(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_interface():
    names = _declared_functions([HEADER])
    for required in ("lbm_create_blocks", "lbm_step_n", "lbm_sensor_flags", "lbm_get_macros",
                     "lbm_block_means"):
        assert required in names
    assert len(names) >= 14
    cnn = _declared_functions([os.path.join(ROOT, "include", "lbm_cnn.h")])
    assert {"lbm_cnn_conv3d_forward", "lbm_cnn_conv3d_wgrad", "lbm_cnn_adam", "lbm_cnn_mse"} <= set(cnn)


def test_cnn_sizes_and_argument_checks(lbm):
    """Sizes of packed weights and the weight-gradient workspace, and the
    argument checks that return before any launch."""
    lib = ctypes.CDLL(lbm.library_path())
    lib.lbm_cnn_packed_size.restype = ctypes.c_int64
    lib.lbm_cnn_wgrad_workspace.restype = ctypes.c_int64
    # Co16 x pad16(27 * Ci4): (16, 5) -> 16 x pad16(216) = 16 x 224
    assert lib.lbm_cnn_packed_size(16, 5) == 16 * 224
    assert lib.lbm_cnn_packed_size(1, 16) == 16 * 432
    assert lib.lbm_cnn_packed_size(0, 4) == -1
    # chunks of 512 voxels x Co16 x (K16 + 1) floats (the extra column: bias sums)
    assert lib.lbm_cnn_wgrad_workspace(2, 16, 16, 16, 16, 16) == 16 * 16 * 433 * 4
    assert lib.lbm_cnn_wgrad_workspace(1, 16, 16, 17, 16, 1) == 9 * 16 * 433 * 4
    f = lib.lbm_cnn_conv3d_forward
    f.argtypes = [ctypes.c_void_p] + [ctypes.c_int32] * 5 + [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                             ctypes.c_void_p]
    assert f(None, 1, 2, 2, 2, 4, None, 4, None, 0, None, None, None) == -1
    assert f(16, 0, 2, 2, 2, 4, 16, 4, None, 0, None, 16, None) == -1
    assert f(20, 1, 2, 2, 2, 4, 16, 4, None, 0, None, 16, None) == -1       # x not 16-byte aligned
    lib.lbm_cnn_adam.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] + [ctypes.c_float] * 4 + \
        [ctypes.c_int32, ctypes.c_void_p]
    assert lib.lbm_cnn_adam(16, 16, 16, 16, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1   # t < 1
    lib.lbm_cnn_adam_begin.argtypes = [ctypes.c_void_p] + [ctypes.c_float] * 4 + [ctypes.c_void_p]
    assert lib.lbm_cnn_adam_begin(None, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert lib.lbm_cnn_adam_begin(16, 1e-3, 1.0, 0.999, 1e-8, None) == -1                # beta1 = 1
    assert lib.lbm_cnn_adam_begin(16, 1e-3, 0.9, 0.999, 0.0, None) == -1                 # eps = 0
    lib.lbm_cnn_adam_dev.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lbm_cnn_adam_dev(16, 16, 16, 16, 10, None, None) == -1                    # no hyper
    assert lib.lbm_cnn_adam_dev(16, 16, 16, 16, -1, 16, None) == -1
    lib.lbm_cnn_adam_layer.argtypes = [ctypes.c_void_p] * 8 + [ctypes.c_int32] * 2 + [ctypes.c_void_p] * 4
    ok = [16] * 8
    assert lib.lbm_cnn_adam_layer(*ok, 16, 6, 16, 16, None, None) == -1                 # no hyper
    assert lib.lbm_cnn_adam_layer(*ok, 0, 6, 16, 16, 16, None) == -1                    # co < 1
    assert lib.lbm_cnn_adam_layer(*([None] + ok[1:]), 16, 6, 16, 16, 16, None) == -1    # no w


def test_library_exports_every_declared_symbol(lbm):
    lib = ctypes.CDLL(lbm.library_path())
    for name in _declared_functions():
        assert hasattr(lib, name), name


def _cavity_desc(lbm, **kw):
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.05
    args = dict(lattice=lbm.LBM_D3Q19, extent=(128, 128, 128), face_bc=(1,) * 6, tau=0.5192,
                storage=lbm.LBM_F32, wall_u=wall_u)
    args.update(kw)
    return lbm.make_desc(**args)


def test_required_bytes_layout(lbm):
    st, b = lbm.lbm_required_bytes(_cavity_desc(lbm))
    assert st == lbm.LBM_OK
    cells = 128 ** 3
    assert b[0] == b[1] and b[0] >= 19 * cells * 4 and b[0] % 256 == 0
    assert b[0] < 19 * (cells * 4 + 65536)
    assert b[2] >= 4096 * 4 and b[3] >= 4096
    assert b[4] >= 4 * cells * 8
    st, b64 = lbm.lbm_required_bytes(_cavity_desc(lbm, storage=lbm.LBM_F64))
    assert b64[0] >= 19 * cells * 8 and b64[2] >= 4096 * 8
    st, b2 = lbm.lbm_required_bytes(lbm.make_desc(lbm.LBM_D2Q9, (64, 64, 1), (1, 1, 1, 1, 0, 0), 0.692,
                                                   storage=lbm.LBM_F64))
    assert st == lbm.LBM_OK and b2[0] >= 9 * 4096 * 8 and b2[3] >= 64


@pytest.mark.parametrize("bad,code", [
    (dict(tau=0.5), "LBM_EINVAL"),
    (dict(tau=float("nan")), "LBM_EINVAL"),
    (dict(extent=(0, 8, 8)), "LBM_EINVAL"),
    (dict(face_bc=(0, 1, 1, 1, 1, 1)), "LBM_EINVAL"),
    (dict(lattice=15), "LBM_ENOTSUP"),
    (dict(smagorinsky=-0.1), "LBM_EINVAL"),
    (dict(smagorinsky=float("inf")), "LBM_EINVAL"),
    (dict(wall_profile=(0, 0, 0, 2, 0, 0)), "LBM_EINVAL"),
    (dict(storage=7), "LBM_ENOTSUP"),
    (dict(block=(4, 4, 4)), "LBM_ENOTSUP"),
    (dict(rho0=-1.0), "LBM_EINVAL"),
    (dict(theta_refine=1e-4, theta_coarsen=1e-3), "LBM_EINVAL"),
    (dict(extent=(2048, 2048, 1024)), "LBM_ENOTSUP"),
])
def test_bad_descriptors_rejected(lbm, bad, code):
    d = _cavity_desc(lbm, **bad)
    st, _ = lbm.lbm_required_bytes(d)
    assert st == getattr(lbm, code)
    assert lbm.lbm_last_error() != ""
    # create fails the same way before any device work
    st2, h = lbm.lbm_create_blocks(d)
    assert st2 == st and not h.value


def test_d2q9_descriptor_rules(lbm):
    ok = lbm.make_desc(lbm.LBM_D2Q9, (10, 10, 1), (1, 1, 1, 1, 0, 0), 0.7)
    assert lbm.lbm_required_bytes(ok)[0] == lbm.LBM_OK
    for kw in (dict(extent=(10, 10, 2)), dict(face_bc=(1, 1, 1, 1, 1, 1)), dict(force=(0, 0, 1e-5))):
        args = dict(lattice=lbm.LBM_D2Q9, extent=(10, 10, 1), face_bc=(1, 1, 1, 1, 0, 0), tau=0.7)
        args.update(kw)
        assert lbm.lbm_required_bytes(lbm.make_desc(**args))[0] == lbm.LBM_EINVAL


def test_create_rejects_missing_buffers(lbm):
    d = _cavity_desc(lbm, extent=(16, 16, 16))
    st, h = lbm.lbm_create_blocks(d)          # buffers left NULL
    assert st == lbm.LBM_EINVAL and "NULL" in lbm.lbm_last_error()


def test_tau_from_reynolds(lbm):
    st, tau = lbm.lbm_tau_from_reynolds(0.1, 64, 100)
    assert st == 0 and abs(tau - 0.692) < 1e-15
    st, tau = lbm.lbm_tau_from_reynolds(0.05, 128, 1000)
    assert st == 0 and abs(tau - 0.5192) < 1e-15
    assert lbm.lbm_tau_from_reynolds(0.1, 64, 0.0)[0] == lbm.LBM_EINVAL


def test_null_handle_calls_fail_cleanly(lbm):
    assert lbm.lbm_step_n(None, 1, 1) == lbm.LBM_EINVAL
    assert lbm.lbm_get_step(None)[0] == lbm.LBM_EINVAL
    lbm.lbm_destroy(None)


def test_product_package_does_not_reach_the_oracle():
    """The HIP binding must not import, load or call anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_1507_06767_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liborc" not in text and "orc_" not in text, fn
