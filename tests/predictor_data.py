"""Solver-generated data of the learned flag predictor, shared by its GPU
test and the schedule selection script: seeded 128^3 lid-driven cavities
(D3Q19, shifted float32, Smagorinsky C = 0.14, Re in [1000, 5000], lid speed
in [0.03, 0.08]), 25 snapshots each, 64 steps apart.  Three disjoint seed
streams: training, validation (picks the training schedule) and the held-out
test cavities (scored only by the test)."""
import numpy as np

import lbm_inputs

HORIZON = 64
THETA = np.log10(1e-3)          # refine flag: M_b > 1e-3
TRAIN_SEED, VALID_SEED, TEST_SEED = 101, 303, 202
SNAPSHOTS = 25


def snapshots(lbm, P, seed, count):
    """(raw features [S, 16, 16, 16, 6], log10 M_b at t + 64 [S, 16, 16, 16],
    (Re, lid) per cavity) of `count` cavities drawn from stream `seed`.  The
    raw features are (rho - rho0, u, log10 M_b at t - 64, log10 M_b at t)."""
    raws, tgts, kept = [], [], []
    for w in lbm_inputs.predictor_cavities(count, seed):
        st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
        assert st == 0
        desc = lbm.make_desc(19, w.n, w.bc, tau, storage=lbm.LBM_F32_SHIFTED, wall_u=w.wall_u, smagorinsky=0.14)
        r = P.snapshot_run(lbm.Blocks, desc, SNAPSHOTS, HORIZON, warm=2 * HORIZON)
        assert r is not None, f"Re {w.reynolds:.0f} lid {w.lid_speed:.3f} went non-finite"
        raws.append(r[0])
        tgts.append(r[1])
        kept.append((round(w.reynolds), round(w.lid_speed, 3)))
    return np.concatenate(raws), np.concatenate(tgts), kept


# The two networks: the configured one reads the block means of (rho - rho0,
# u) only and predicts log10 M_b directly; the extension also reads the
# sensor now and one horizon earlier and predicts the change.
NETS = {"rho_u": dict(channels=(4, 16, 16, 16, 1), residual=False),
        "sensor": dict(channels=(6, 16, 16, 16, 1), residual=True)}


def inputs(raw, kind):
    return raw[..., :4] if kind == "rho_u" else raw


def make_net(P, kind, seed=0):
    return P.FlagPredictor(seed=seed, **NETS[kind])


def f1(p, r):
    return 2 * p * r / max(p + r, 1e-30)


def climatology(target_train):
    """A forecast that sees neither the sensor nor the flow: the mean over
    the training snapshots of log10 M_b at each block (the average sensor
    field of the training cavities)."""
    return np.asarray(target_train, dtype=np.float64).mean(axis=0)


def scores(P, pred_log, raw, target_log, clim):
    """Refine-flag precision, recall and F1 of predicted log10 M_b against
    the exact sensor at the horizon, the squared error of log10 M_b (blocks
    above 1e-8 now and then), and the same for two baselines: reusing the
    flags of t (the exact sensor alone) and the training climatology."""
    true = target_log > THETA
    reuse = raw[..., -1] > THETA
    mine = pred_log > THETA
    clim_pred = np.broadcast_to(clim, target_log.shape)
    p1, r1 = P.flag_scores(mine, true)
    p0, r0 = P.flag_scores(reuse, true)
    pc, rc = P.flag_scores(clim_pred > THETA, true)
    live = (target_log > -8) & (raw[..., -1] > -8)
    changed = true != reuse
    return {"precision": p1, "recall": r1, "f1": f1(p1, r1),
            "mse": float(np.mean((pred_log - target_log)[live] ** 2)),
            "reuse_precision": p0, "reuse_recall": r0, "reuse_f1": f1(p0, r0),
            "reuse_mse": float(np.mean((raw[..., -1] - target_log)[live] ** 2)),
            "clim_precision": pc, "clim_recall": rc, "clim_f1": f1(pc, rc),
            "clim_mse": float(np.mean((clim_pred - target_log)[live] ** 2)),
            "var": float(np.var(target_log[live])),
            "changed": int(changed.sum()), "fixed": int((changed & (mine == true)).sum()),
            "broken": int((~changed & (mine != true)).sum())}
