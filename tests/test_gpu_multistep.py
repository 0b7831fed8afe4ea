"""Several steps per launch on small 2D grids (lbm_set_multistep, the
temporal-blocking kernel step_multi).  The same runs with the multi-step
launches on and off give the same bits: populations after runs whose lengths
are not multiples of the steps per launch, with sensor steps in between (so
the runs are cut at the cadence), block maxima and flags of the last sensor
step, and step counters; eagerly and replayed from HIP graphs.  Cases cover
walls with a moving lid, periodic axes (the halo wraps, on grids narrower
than the halo too), a body force, the Smagorinsky model, every storage the
path takes and ragged tiles.  Against the oracle the path is covered by the
2D cases of test_gpu_parity.py, whose ping-pong handles take it by default.
Each case prints what it runs before the GPU work."""
import numpy as np
import pytest

from lbm_inputs import PERIODIC, WALL
import lbm_inputs

pytestmark = pytest.mark.gpu

_P2 = (PERIODIC, PERIODIC)


def _wall(lid=0.0, face=3, comp=0):
    w = [[0.0] * 3 for _ in range(6)]
    w[face][comp] = lid
    return w


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1507_06767_amd as lbm
    return lbm


# name, extent, face_bc, wall_u, storage, force, smagorinsky
_CASES = [
    ("cavity64_f64", (64, 64, 1), (WALL,) * 4 + _P2, _wall(0.1), 0, (0, 0, 0), 0.0),
    ("ragged37x23_f32", (37, 23, 1), (WALL,) * 4 + _P2, _wall(0.08), 1, (0, 0, 0), 0.0),
    ("channel50x20_force_f32s", (50, 20, 1), (PERIODIC, PERIODIC, WALL, WALL) + _P2, _wall(), 2, (2e-5, 0, 0), 0.0),
    ("cavity40_smag_f64", (40, 40, 1), (WALL,) * 4 + _P2, _wall(0.1), 0, (0, 0, 0), 0.14),
    ("periodic5x3_f64", (5, 3, 1), (PERIODIC,) * 6, _wall(), 0, (1e-4, -2e-4, 0), 0.0),
    ("walls2x2_f64", (2, 2, 1), (WALL,) * 4 + _P2, _wall(0.1), 0, (0, 0, 0), 0.0),
    ("cavity33x17_f16s", (33, 17, 1), (WALL,) * 4 + _P2, _wall(0.1), 3, (0, 0, 0), 0.0),
    ("cavity33x17_bf16s", (33, 17, 1), (WALL,) * 4 + _P2, _wall(0.1), 4, (0, 0, 0), 0.0),
]


def _run(torch, lbm, case, multi, chunk):
    name, n, bc, wall_u, storage, force, smag = case
    desc = lbm.make_desc(9, n, bc, 0.62, storage=storage, wall_u=wall_u, force=force, smagorinsky=smag,
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
    assert blk.scheme()["multistep"] == 5
    blk.set_multistep(multi)
    blk.use_graphs(chunk)
    u0 = lbm_inputs.velocity_perturbation(n, 0.02, seed=11, dims=2)
    blk.set_equilibrium(u=u0)
    res = []
    for steps, every in ((23, 7), (12, 0), (41, 10), (3, 0), (9, 9), (98, 0)):
        blk.step_n(steps, every)
        res.append(blk.step)
        if every:
            bm, fl = blk.sensor_flags()[:2]
            res += [bm, fl]
    res.append(blk.populations())
    blk.close()
    return res


@pytest.mark.parametrize("chunk", [0, 6], ids=["eager", "graph6"])
@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_multistep_matches_one_launch_per_step(lbm, case, chunk):
    import torch
    print(f"\n[case] multistep {case[0]} chunk={chunk}", flush=True)
    ref = _run(torch, lbm, case, 0, chunk)
    for multi in (5, 2, 3):
        out = _run(torch, lbm, case, multi, chunk)
        for a, b in zip(ref, out):
            assert np.array_equal(np.asarray(a), np.asarray(b)), f"multistep {multi} differs"
    assert np.isfinite(ref[-1]).all()


def test_multistep_setting(lbm, monkeypatch):
    """Where the path applies by default, and the errors of lbm_set_multistep."""
    import torch
    print("\n[case] multistep setting", flush=True)
    monkeypatch.delenv("LBM_STREAMING", raising=False)
    s = torch.cuda.Stream()
    cav = lbm_inputs.cavity2d()
    d = lbm.make_desc(9, cav.n, cav.bc, 0.6, storage=lbm.LBM_F64)
    blk = lbm.Blocks(d, stream=s)
    sc = blk.scheme()
    assert not sc["inplace"] and sc["multistep"] == 5      # automatic streaming picks ping-pong here
    for bad in (1, 6, -1):
        with pytest.raises(lbm.LbmError):
            blk.set_multistep(bad)
    blk.set_multistep(0)
    assert blk.scheme()["multistep"] == 0
    blk.close()
    monkeypatch.setenv("LBM_STREAMING", "inplace")
    blk = lbm.Blocks(d, stream=s)
    sc = blk.scheme()
    assert sc["inplace"] and sc["multistep"] == 0
    with pytest.raises(lbm.LbmError):
        blk.set_multistep(5)
    blk.close()
    monkeypatch.delenv("LBM_STREAMING")
    for q, n, storage in ((9, (300, 300, 1), lbm.LBM_F32), (9, (32, 32, 1), lbm.LBM_F16_SHIFTED_SR),
                          (19, (16, 16, 16), lbm.LBM_F32)):
        bc = (WALL,) * 6 if q == 19 else (WALL,) * 4 + _P2
        blk = lbm.Blocks(lbm.make_desc(q, n, bc, 0.6, storage=storage), stream=s)
        assert blk.scheme()["multistep"] == 0
        with pytest.raises(lbm.LbmError):
            blk.set_multistep(3)
        blk.close()
