"""Picks the training schedule of each flag predictor on the validation
cavities, without touching the held-out test cavities.  Run on a GPU from
the repository root:

    python tests/select_predictor_schedule.py [--frozen]

Trains each network (predictor_data.NETS) on the training cavities for every
candidate (Adam iterations, initial cosine learning rate), scores refine
flags 64 steps ahead on the validation cavities, and prints one line per
candidate and the choice: the highest F1, then the lowest squared error of
log10 M_b.  The choice is frozen in tests/test_gpu_predictor.py (SCHEDULES).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import predictor_data as D  # noqa: E402

CANDIDATES = [(iters, lr) for iters in (3000, 6000, 10000) for lr in (1e-3, 2e-3, 4e-3)]
if "--frozen" in sys.argv:     # only the schedules frozen in the test, to restate their validation scores
    CANDIDATES = [(10000, 2e-3)]


def main():
    import paper_1507_06767_amd as lbm
    from paper_1507_06767_amd import predictor as P
    t0 = time.time()
    Xtr, Ytr, runs_tr = D.snapshots(lbm, P, D.TRAIN_SEED, 8)
    Xva, Yva, runs_va = D.snapshots(lbm, P, D.VALID_SEED, 4)
    print(f"training cavities (Re, lid) {runs_tr}\nvalidation cavities {runs_va}\n"
          f"data in {time.time() - t0:.0f} s", flush=True)
    for kind in D.NETS:
        best = None
        for iters, lr in CANDIDATES:
            net = D.make_net(P, kind)
            net.fit(D.inputs(Xtr, kind), Ytr, iters=iters, batch=8, lr=lr)
            s = D.scores(P, net.predict_log(D.inputs(Xva, kind)), Xva, Yva, D.climatology(Ytr))
            print(f"{kind:6s} iters {iters:5d} lr {lr:.0e}: precision {s['precision']:.4f} recall {s['recall']:.4f} "
                  f"F1 {s['f1']:.4f} mse {s['mse']:.3e} (reuse P {s['reuse_precision']:.4f} R "
                  f"{s['reuse_recall']:.4f} F1 {s['reuse_f1']:.4f} mse {s['reuse_mse']:.3e}; climatology P "
                  f"{s['clim_precision']:.4f} R {s['clim_recall']:.4f} F1 {s['clim_f1']:.4f} mse {s['clim_mse']:.3e}; "
                  f"variance {s['var']:.3e}; fixed {s['fixed']} broken {s['broken']} of {s['changed']} changed)",
                  flush=True)
            key = (s["f1"], -s["mse"])
            if best is None or key > best[0]:
                best = (key, iters, lr)
        print(f"chosen for {kind}: iters {best[1]}, lr {best[2]:.0e} (validation F1 {best[0][0]:.4f})", flush=True)


if __name__ == "__main__":
    main()
