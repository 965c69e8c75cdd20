"""Train and evaluate the learned corrector of a g5 run toward a g7 run.

    python -m paper_1607_05535_amd.train_corrector [--seeds 10] [--pairs 200]
        [--spinup 576] [--steps 4000] [--out results.json]

Pairs come from trajectories of the fine gas-giant run (one noise seed per
trajectory, seeds 1000, 1001, ...), each spun up for `spinup` fine steps of
150 s and then cut into `pairs` consecutive 600 s intervals; the last seed is
held out for evaluation.  Prints one JSON report.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(fine=7, coarse=5, seeds=10, pairs=200, spinup=576, steps=4000, batch=4096, lr=1e-3, base_seed=1000,
        log=None):
    """Generate pairs, train, evaluate on the held-out (last) seed and time
    600 s of simulated time both ways; returns the report as a dict."""
    import torch

    import workloads
    from paper_1607_05535_amd import learned

    fw, cw = workloads.corrector_pair(fine, coarse)
    P = learned.Pipeline(fw, cw, ratio=4)
    seed_list = list(range(base_seed, base_seed + seeds))
    train_seeds, test_seeds = seed_list[:-1], seed_list[-1:]
    t0 = time.perf_counter()
    C, F = P.make_pairs(train_seeds, spinup, pairs, log=log)
    t_data = time.perf_counter() - t0
    norm = P.norm(C, F)
    t0 = time.perf_counter()
    net, corr, losses = P.train(C, F, norm, steps, batch=batch, lr=lr, seed=0, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del C, F
    res = P.evaluate(corr, test_seeds, spinup, pairs)

    # wall time of 600 s of simulated time: corrected coarse vs plain fine
    fine_st = P._fine(test_seeds[0])
    fine_st.step(2, fw.n_acoustic)
    P.work.step(2, cw.n_acoustic)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        fine_st.step(4, fw.n_acoustic)
    torch.cuda.synchronize()
    t_fine = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        P.work.step(1, cw.n_acoustic)
        corr.apply(count=False)
    torch.cuda.synchronize()
    t_corr = (time.perf_counter() - t0) / reps
    return {
        "fine": f"g{fine}L{fw.n_lev} dt {fw.dt:.0f} s", "coarse": f"g{coarse}L{cw.n_lev} dt {cw.dt:.0f} s",
        "train_pairs": len(train_seeds) * pairs, "held_out_pairs": len(test_seeds) * pairs,
        "seeds": seed_list, "spinup_fine_steps": spinup, "train_steps": steps, "batch": batch,
        "loss_first_last": [losses[0][1], losses[-1][1]],
        "held_out": res,
        "seconds": {"data": t_data, "train": t_train},
        "ms_per_600s": {"fine_4_steps": t_fine * 1e3, "coarse_step_plus_corrector": t_corr * 1e3},
        "speedup_vs_fine": t_fine / t_corr,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fine", type=int, default=7)
    ap.add_argument("--coarse", type=int, default=5)
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--pairs", type=int, default=200)
    ap.add_argument("--spinup", type=int, default=576)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = run(args.fine, args.coarse, args.seeds, args.pairs, args.spinup, args.steps, args.batch, args.lr,
              log=lambda msg: print(msg, flush=True))
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
