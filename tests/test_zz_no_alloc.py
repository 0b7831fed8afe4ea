"""The allocation-free conservation entry point against lbm_conservation.

lbm_conservation_noalloc keeps its partial sums and totals in the library's
own static device array instead of the handle's scratch buffer, with the
same kernels and summation order: its totals must be the same bits.  Two
calls in a row, the second on a smaller grid (so the array holds the first
call's larger set of partial sums when the second starts), in both
streaming schemes and in float64 and float32 storage."""
import numpy as np
import pytest

from paper_1507_06767_amd import abi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1507_06767_amd as lbm
    return lbm


def _cavity(lbm, n, storage, streaming):
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3][0] = 0.08
    desc = lbm.make_desc(lbm.LBM_D3Q19, n, (1,) * 6, 0.6, storage=storage, wall_u=wall_u,
                         streaming=streaming)
    return lbm.Blocks(desc, device="cuda:0")


@pytest.mark.parametrize("streaming", [abi.LBM_STREAMING_PINGPONG, abi.LBM_STREAMING_INPLACE],
                         ids=["pingpong", "inplace"])
@pytest.mark.parametrize("storage", [abi.LBM_F64, abi.LBM_F32], ids=["f64", "f32"])
def test_noalloc_conservation_matches(lbm, storage, streaming):
    if storage == abi.LBM_F64 and streaming == abi.LBM_STREAMING_INPLACE:
        pytest.skip("3D float64 streams ping-pong only")
    # 96 x 80 x 72 cells use 1024 partial sums (the cap); 20 x 12 x 9 use 9
    for n, steps in (((96, 80, 72), 7), ((20, 12, 9), 5)):
        print(f"\n[case] noalloc conservation n={n} storage={storage} streaming={streaming}", flush=True)
        blk = _cavity(lbm, n, storage, streaming)
        blk.step_n(steps, 0)
        st, ref = abi.lbm_conservation(blk.h)
        assert st == abi.LBM_OK, abi.lbm_last_error()
        st, got = abi.lbm_conservation_noalloc(blk.h)
        assert st == abi.LBM_OK, abi.lbm_last_error()
        print(f"totals {got.tolist()} vs {ref.tolist()}")
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (got, ref)
        # the state is left as it was: stepping on gives the same totals again
        blk.step_n(1, 0)
        st, ref2 = abi.lbm_conservation(blk.h)
        st2, got2 = abi.lbm_conservation_noalloc(blk.h)
        assert st == st2 == abi.LBM_OK
        assert np.array_equal(got2.view(np.uint64), ref2.view(np.uint64))
        assert abs(got2[0] - np.prod(n)) < 1e-6 * np.prod(n)     # mass of the cavity
        blk.close()


def test_noalloc_conservation_rejects_null(lbm):
    assert abi._lib.lbm_conservation_noalloc(None, None) == abi.LBM_EINVAL
