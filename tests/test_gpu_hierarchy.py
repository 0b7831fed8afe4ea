"""The two-level patch hierarchy on the GPU against its FP64 oracle
(oracle/hier.py): coarse and fine populations, fine sensor block maxima and
flags after several coarse steps, for D3Q19 and D3Q27, float64 and shifted
float32; graph replay against launch-by-launch stepping; the autotuners
leave results unchanged.

Tolerances: float64 populations 1e-13 absolute (values ~0.01-0.3), block
maxima 1e-11 relative; shifted float32 populations 2e-7 absolute, fields as
in the single-grid parity tests (1e-5 relative), block maxima 2e-5 relative
to max(M, 1e-3).  Plain float32 (the storage of the refined benchmark)
rounds every stored f_i ~ w_i rho0 <= 1/3 to 2^-24 relative (up to 2e-8)
at each of 12 coarse and 24 fine steps, mixed by the interpolation and the
restriction: populations 1e-6 absolute, block maxima 2e-4 relative (its
sensor floor, as in the single-grid tests).  Both sensor kinds (Sec. 3.2,
Eqs. sensor and kkn)."""
import numpy as np
import pytest

import lbm_inputs
from lbm_inputs import WALL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1507_06767_amd as lbm
    return torch, lbm


def _lid(u):
    w = [[0.0] * 3 for _ in range(6)]
    w[3][0] = u
    return w


# three patches: two abutting along x, one apart (coarse boxes [lo, hi))
_BOXES = [((4, 4, 4), (8, 8, 12)), ((8, 4, 4), (12, 8, 12)), ((14, 10, 6), (22, 18, 10))]
_N = (24, 20, 16)


def _make(torch, lbm, q, storage, use_graph, tau=0.6, boxes=_BOXES, kind=0):
    desc = lbm.make_desc(q, _N, (WALL,) * 6, tau, storage=storage, wall_u=_lid(0.06),
                         streaming=lbm.LBM_STREAMING_PINGPONG, sensor_kind=kind)
    blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
    H = lbm.Hierarchy(blk, boxes, use_graph=use_graph)
    return blk, H


# (q, storage, sensor kind): storage 0 float64, 1 float32, 2 shifted float32
_CASES = [(19, 0, 0), (19, 2, 0), (27, 0, 0), (27, 2, 0), (19, 1, 0), (19, 0, 1), (19, 2, 1), (27, 0, 1)]
_TOL = {0: (1e-13, 1e-11), 1: (1e-6, 2e-4), 2: (2e-7, 2e-5)}   # populations (absolute), block maxima


@pytest.mark.parametrize("case", _CASES, ids=[f"q{q}_{('f64', 'f32', 'f32s')[s]}_{('l2', 'kkn')[k]}"
                                              for q, s, k in _CASES])
def test_hierarchy_matches_oracle(env, orc, case):
    torch, lbm = env
    from oracle.hier import Hierarchy as OH
    q, storage, kind = case
    print(f"\n[case] hierarchy q={q} storage={storage} sensor kind={kind}", flush=True)
    blk, H = _make(torch, lbm, q, storage, use_graph=True, kind=kind)
    G = orc.Grid(q=q, n=_N, bc=(WALL,) * 6, wall_u=_lid(0.06), tau=0.6, sensor_kind=kind)
    O = OH(G, _BOXES)
    S = G.equilibrium_state()
    O.init_from(S)
    steps = 12
    H.step_n(steps, steps)
    bmax_ref = None
    for k in range(steps):
        S, bm = O.step(S, k, sensor=(k == steps - 1))
        if bm is not None:
            bmax_ref = np.concatenate([b.ravel() for b in bm])
    bm_gpu, fl_gpu, kk = H.sensor()
    assert kk == steps
    tol_f, tol_b = _TOL[storage]
    ec = np.abs(blk.populations() - S).max()
    ef = max(np.abs(H.patch_fields(p)[2] - O.patch_fields(p)[2]).max() for p in range(len(_BOXES)))
    eb = float((np.abs(bm_gpu - bmax_ref) / np.maximum(bmax_ref, 1e-3)).max())
    print(f"hierarchy q={q} storage={storage} kind={kind}: coarse pop err {ec:.2e}, fine pop err {ef:.2e}, "
          f"fine block max rel err {eb:.2e}, max M {bmax_ref.max():.3e}")
    assert ec < tol_f and ef < tol_f and eb < tol_b
    ref_flags = np.where(bmax_ref > 1e-3, 1, np.where(bmax_ref < 5e-4, -1, 0))
    near = (np.abs(bmax_ref - 1e-3) <= tol_b * 1e-3) | (np.abs(bmax_ref - 5e-4) <= tol_b * 5e-4)
    assert not ((fl_gpu != ref_flags) & ~near).any()
    info = H.info()
    assert info["fine_cells"] == sum(8 * np.prod([hi[a] - lo[a] for a in range(3)]) for lo, hi in _BOXES)
    assert info["n_eff"] == 0.5 * np.prod(_N) + info["fine_cells"]
    H.close()
    blk.close()


# 16-bit shifted storages on both levels (float32 arithmetic): bounds about
# 2.5x the errors measured on MI355X after 12 coarse steps (24 fine):
# (populations absolute, block maxima relative to max(M, 1e-3));
# measured coarse / fine populations, block maxima: f16s 5.5e-6 / 1.8e-6,
# 5.9e-4; bf16s 6.1e-5 / 1.6e-5, 3.4e-3; f16sr 8.9e-6 / 2.6e-6, 4.6e-4;
# bf16sr 7.6e-5 / 2.2e-5, 1.9e-3.  One half-precision spacing of the
# deviations d ~ 0.01 is 7.6e-6 (bfloat16: 6.1e-5).
_LOWPREC = {3: ("f16s", 1.5e-5, 1.5e-3), 4: ("bf16s", 1.5e-4, 1e-2), 5: ("f16sr", 2.5e-5, 1.5e-3),
            6: ("bf16sr", 2e-4, 5e-3)}


@pytest.mark.parametrize("storage", sorted(_LOWPREC), ids=[_LOWPREC[k][0] for k in sorted(_LOWPREC)])
def test_hierarchy_lowprec_matches_oracle(env, orc, storage):
    """Shifted half and bfloat16 storage, rounding to nearest or
    stochastically, on the coarse grid and the patches (ghost fill,
    restriction and the fine step store 16 bits), against the FP64 hierarchy
    oracle; stochastic rounding runs launch by launch (its keys follow the
    step index), rounding to nearest from the captured graph."""
    torch, lbm = env
    from oracle.hier import Hierarchy as OH
    name, tol_f, tol_b = _LOWPREC[storage]
    sr = storage in (5, 6)
    print(f"\n[case] hierarchy {name}", flush=True)
    blk, H = _make(torch, lbm, 19, storage, use_graph=not sr)
    G = orc.Grid(q=19, n=_N, bc=(WALL,) * 6, wall_u=_lid(0.06), tau=0.6)
    O = OH(G, _BOXES)
    S = G.equilibrium_state()
    O.init_from(S)
    steps = 12
    H.step_n(steps, steps)
    bmax_ref = None
    for k in range(steps):
        S, bm = O.step(S, k, sensor=(k == steps - 1))
        if bm is not None:
            bmax_ref = np.concatenate([b.ravel() for b in bm])
    bm_gpu, fl_gpu, kk = H.sensor()
    assert kk == steps
    ec = np.abs(blk.populations() - S).max()
    ef = max(np.abs(H.patch_fields(p)[2] - O.patch_fields(p)[2]).max() for p in range(len(_BOXES)))
    eb = float((np.abs(bm_gpu - bmax_ref) / np.maximum(bmax_ref, 1e-3)).max())
    moved = max(np.abs(O.patch_fields(p)[2] - G.equilibrium_state()[:, :1, :1, :1].reshape(19, 1, 1, 1)).max()
                for p in range(len(_BOXES)))
    ref_flags = np.where(bmax_ref > 1e-3, 1, np.where(bmax_ref < 5e-4, -1, 0))
    differ = int((fl_gpu != ref_flags).sum())
    print(f"hierarchy {name}: coarse pop err {ec:.2e}, fine pop err {ef:.2e} (fine populations moved "
          f"{moved:.2e} from rest), fine block max rel err {eb:.2e}, flags differing {differ} of {fl_gpu.size}")
    assert ec < tol_f and ef < tol_f and eb < tol_b
    near = (np.abs(bmax_ref - 1e-3) <= tol_b * 1e-3) | (np.abs(bmax_ref - 5e-4) <= tol_b * 5e-4)
    assert not ((fl_gpu != ref_flags) & ~near).any()
    H.close()
    blk.close()


def test_hierarchy_sr_refuses_graphs(env):
    torch, lbm = env
    desc = lbm.make_desc(19, _N, (WALL,) * 6, 0.6, storage=lbm.LBM_F16_SHIFTED_SR, wall_u=_lid(0.06),
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
    with pytest.raises(lbm.LbmError) as e:
        lbm.Hierarchy(blk, _BOXES, use_graph=True)
    assert e.value.status == lbm.LBM_ENOTSUP
    blk.close()


@pytest.mark.parametrize("storage", [2, 3], ids=["f32s", "f16s"])
def test_graph_replay_matches_launches(env, storage):
    """Steps replayed from the captured graph (in several calls, with host
    reads in between) give the same bits as launch-by-launch stepping."""
    torch, lbm = env
    print(f"\n[case] hierarchy graph vs eager storage={storage}", flush=True)
    out = {}
    for use_graph in (True, False):
        blk, H = _make(torch, lbm, 19, storage, use_graph)
        for n in (4, 3, 5, 2):
            H.step_n(n, 0)
            _ = H.patch_fields(0)          # eager work and a synchronisation between replays
        out[use_graph] = (blk.populations(), [H.patch_fields(p)[2] for p in range(len(_BOXES))])
        H.close()
        blk.close()
    assert np.array_equal(out[True][0], out[False][0])
    for a, b in zip(out[True][1], out[False][1]):
        assert np.array_equal(a, b)


def test_hierarchy_autotune_keeps_results(env):
    torch, lbm = env
    print("\n[case] hierarchy autotune", flush=True)
    res = []
    for tune in (False, True):
        blk, H = _make(torch, lbm, 19, 2, use_graph=True)
        H.step_n(3, 0)
        if tune:
            tx, wg, us = H.autotune(3)
            print(f"autotune picked tiles up to {tx}x8x8, {wg} workgroups ({us:.1f} us per fine step)")
            assert tx in (8, 16, 32, 48) and wg >= 1     # 48: bands (patch_band_step)
        H.step_n(5, 0)
        res.append((blk.populations(), H.patch_fields(2)[2]))
        H.close()
        blk.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("streaming", ["pingpong", "inplace"])
def test_single_grid_autotune_keeps_results(env, streaming):
    """lbm_autotune times the tile widths without changing the state, and
    every width gives the same bits."""
    torch, lbm = env
    print(f"\n[case] autotune 64^3 {streaming}", flush=True)
    mode = lbm.LBM_STREAMING_PINGPONG if streaming == "pingpong" else lbm.LBM_STREAMING_INPLACE
    res = []
    for tune in (False, True):
        desc = lbm.make_desc(19, (64, 64, 64), (WALL,) * 6, 0.55, storage=lbm.LBM_F32_SHIFTED, wall_u=_lid(0.05),
                             streaming=mode)
        blk = lbm.Blocks(desc)
        blk.step_n(7, 7)
        if tune:
            before = blk.populations()
            tx = blk.autotune(3)
            print(f"autotune picked tile width {tx}")
            # row tiles (256 cells of one row) are a candidate for 3D ping-pong only
            assert tx in ((32, 64, 128, 256) if streaming == "pingpong" else (32, 64, 128))
            assert blk.scheme()["tile_x"] == tx
            assert np.array_equal(before, blk.populations())
        blk.step_n(9, 8)
        res.append((blk.populations(), blk.sensor_flags()[0]))
        blk.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_hierarchy_rejects_bad_boxes(env):
    torch, lbm = env
    print("\n[case] hierarchy argument checks", flush=True)
    desc = lbm.make_desc(19, _N, (WALL,) * 6, 0.6, storage=lbm.LBM_F32_SHIFTED, wall_u=_lid(0.06),
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    blk = lbm.Blocks(desc)
    bad = [
        [((0, 4, 4), (4, 8, 8))],                              # touches the domain face
        [((4, 4, 4), (7, 8, 8))],                              # extent not a multiple of 4
        [((4, 4, 4), (8, 8, 8)), ((6, 4, 4), (10, 8, 8))],     # overlap
    ]
    for boxes in bad:
        st, _ = lbm.lbm_hierarchy_required_bytes(blk.h, boxes)
        assert st == lbm.LBM_EINVAL, boxes
    blk.close()
    desc = lbm.make_desc(19, _N, (WALL,) * 6, 0.6, storage=lbm.LBM_F32_SHIFTED, wall_u=_lid(0.06),
                         streaming=lbm.LBM_STREAMING_INPLACE)
    blk = lbm.Blocks(desc)
    st, _ = lbm.lbm_hierarchy_required_bytes(blk.h, _BOXES)
    assert st == lbm.LBM_ENOTSUP                               # the coarse grid must stream ping-pong
    blk.close()


@pytest.mark.parametrize("q", [19, 27])
def test_lds_ghost_fill_matches_list_fill(env, monkeypatch, q):
    """The ghost fill staged in LDS per face tile and the plain list-driven
    one perform the same arithmetic in the same order: identical bits."""
    torch, lbm = env
    print(f"\n[case] hierarchy ghost fill LDS vs plain q={q}", flush=True)
    out = {}
    for mode in ("lds", "plain"):
        monkeypatch.setenv("LBM_HIER_GHOSTS", mode)
        blk, H = _make(torch, lbm, q, 2, use_graph=True)
        H.step_n(7, 7)
        out[mode] = (blk.populations(), [H.patch_fields(p)[2] for p in range(len(_BOXES))], H.sensor()[0])
        H.close()
        blk.close()
    assert np.array_equal(out["lds"][0], out["plain"][0]) and np.array_equal(out["lds"][2], out["plain"][2])
    for a, b in zip(out["lds"][1], out["plain"][1]):
        assert np.array_equal(a, b)


def test_profile_times_kernels_and_steps_like_eager(env):
    """lbm_hierarchy_profile advances the state exactly as eager stepping
    does (identical bits) and returns positive per-launch durations."""
    torch, lbm = env
    print("\n[case] hierarchy profile", flush=True)
    out = []
    for prof in (True, False):
        blk, H = _make(torch, lbm, 19, 2, use_graph=False)
        H.step_n(2, 0)
        if prof:
            us = H.profile(3)
            print("profile us per launch:", {k: round(v, 1) for k, v in us.items()})
            assert set(us) == {"coarse", "ghosts", "fine", "fine_restrict"}
            assert all(v > 0.0 for v in us.values())
        else:
            H.step_n(3, 0)
        out.append((blk.populations(), [H.patch_fields(p)[2] for p in range(len(_BOXES))]))
        H.close()
        blk.close()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
    blk, H = _make(torch, lbm, 19, 2, use_graph=False)
    st, _ = lbm.lbm_hierarchy_profile(H.h, 0)
    assert st == lbm.LBM_EINVAL
    H.close()
    blk.close()


@pytest.mark.parametrize("storage", [0, 2], ids=["f64", "f32s"])
@pytest.mark.parametrize("tiles", ["bands", "32"])
def test_fused_restriction_matches_separate_kernel(env, monkeypatch, storage, tiles):
    """The restriction inside the second fine step, in bands (the default)
    and in W x 8 x 8 tiles (LBM_HIER_TILES=32), against the separate
    list-driven kernel: all three sum a coarse cell's 8 fine deviations in
    64-bit fixed point, exactly and in any order, so after 8 coarse steps
    the coarse and fine populations and the sensor maxima are the same
    bits."""
    torch, lbm = env
    print(f"\n[case] fused vs separate restriction storage={storage} tiles={tiles}", flush=True)
    if tiles == "bands":
        monkeypatch.delenv("LBM_HIER_TILES", raising=False)
    else:
        monkeypatch.setenv("LBM_HIER_TILES", tiles)
    out = {}
    for mode in ("fused", "separate"):
        if mode == "separate":
            monkeypatch.setenv("LBM_HIER_RESTRICT", "separate")
        else:
            monkeypatch.delenv("LBM_HIER_RESTRICT", raising=False)
        blk, H = _make(torch, lbm, 19, storage, use_graph=True)
        assert H.info()["tile_x"] == (48 if tiles == "bands" else 32)
        H.step_n(8, 8)
        out[mode] = (blk.populations(), [H.patch_fields(p)[2] for p in range(len(_BOXES))], H.sensor()[0])
        H.close()
        blk.close()
    ec = np.abs(out["fused"][0] - out["separate"][0]).max()
    ef = max(np.abs(a - b).max() for a, b in zip(out["fused"][1], out["separate"][1]))
    print(f"fused vs separate: coarse {ec:.2e}, fine {ef:.2e}")
    assert np.array_equal(out["fused"][0], out["separate"][0])
    for a, b in zip(out["fused"][1], out["separate"][1]):
        assert np.array_equal(a, b)
    assert np.array_equal(out["fused"][2], out["separate"][2])


@pytest.mark.parametrize("case", [(19, 2, 0), (19, 0, 1), (27, 1, 0)], ids=["q19_f32s_l2", "q19_f64_kkn", "q27_f32_l2"])
def test_bands_match_tiles(env, monkeypatch, case):
    """The band form of the fine step (the default) against W x 8 x 8 tiles:
    the same arithmetic per cell and the same fixed-point restriction, so
    after 1 and after 6 coarse steps the coarse and fine populations and the
    sensor maxima are the same bits."""
    torch, lbm = env
    q, storage, kind = case
    print(f"\n[case] bands vs tiles q={q} storage={storage} kind={kind}", flush=True)
    # boxes whose rows are 16, 24, 32, 48 and 64 fine cells wide (the last in
    # two bands, 48 + 16), two pairs touching
    boxes = [((4, 4, 4), (12, 8, 12)), ((12, 4, 4), (24, 8, 8)), ((4, 10, 4), (20, 14, 8)),
             ((4, 10, 8), (28, 14, 12)), ((2, 16, 12), (34, 20, 16))]
    n = (40, 24, 24)
    out = {}
    for tiles in ("bands", "16"):
        if tiles == "bands":
            monkeypatch.delenv("LBM_HIER_TILES", raising=False)
        else:
            monkeypatch.setenv("LBM_HIER_TILES", tiles)
        desc = lbm.make_desc(q, n, (WALL,) * 6, 0.6, storage=storage, wall_u=_lid(0.06),
                             streaming=lbm.LBM_STREAMING_PINGPONG, sensor_kind=kind)
        blk = lbm.Blocks(desc, stream=torch.cuda.Stream())
        blk.set_equilibrium(u=lbm_inputs.velocity_perturbation(n, 0.02, 4))
        H = lbm.Hierarchy(blk, boxes, use_graph=False)
        # one coarse step: fine steps 1 and 2 start from the same interpolated state
        H.step_n(1, 1)
        first = ([H.patch_fields(p)[2] for p in range(len(boxes))], H.sensor()[0])
        H.step_n(5, 5)
        out[tiles] = (first, blk.populations(), [H.patch_fields(p)[2] for p in range(len(boxes))], H.sensor()[0])
        H.close()
        blk.close()
    a, b = out["bands"], out["16"]
    for fa, fb in zip(a[0][0], b[0][0]):
        assert np.array_equal(fa, fb)
    assert np.array_equal(a[0][1], b[0][1])
    ec = np.abs(a[1] - b[1]).max()
    ef = max(np.abs(x - y).max() for x, y in zip(a[2], b[2]))
    print(f"bands vs tiles after 6 coarse steps: coarse {ec:.2e}, fine {ef:.2e}")
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[3], b[3])
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
