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

    import torch

    import workloads
    from paper_1607_05535_amd import learned, thor

    def log(msg):
        print(msg, flush=True)

    fw, cw = workloads.corrector_pair(args.fine, args.coarse)
    P = learned.Pipeline(fw, cw, ratio=4)
    seeds = list(range(1000, 1000 + args.seeds))
    train_seeds, test_seeds = seeds[:-1], seeds[-1:]
    t0 = time.perf_counter()
    C, F = P.make_pairs(train_seeds, args.spinup, args.pairs, log=log)
    t_data = time.perf_counter() - t0
    norm = P.norm(C, F)
    t0 = time.perf_counter()
    net, corr, losses = P.train(C, F, norm, args.steps, batch=args.batch, lr=args.lr, seed=0, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = P.evaluate(corr, test_seeds, args.spinup, args.pairs)

    # wall time of 600 s of simulated time: corrected coarse vs plain fine
    fine = P._fine(test_seeds[0])
    fine.step(2, fw.n_acoustic)
    P.work.step(2, cw.n_acoustic)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        fine.step(4, fw.n_acoustic)
    torch.cuda.synchronize()
    t_fine = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        P.work.step(1, cw.n_acoustic)
        corr.apply(count=False)
    torch.cuda.synchronize()
    t_corr = (time.perf_counter() - t0) / reps
    out = {
        "fine": f"g{args.fine}L{fw.n_lev} dt {fw.dt:.0f} s", "coarse": f"g{args.coarse}L{cw.n_lev} dt {cw.dt:.0f} s",
        "train_pairs": int(C.shape[0]), "held_out_pairs": len(test_seeds) * args.pairs,
        "seeds": seeds, "spinup_fine_steps": args.spinup, "train_steps": args.steps, "batch": args.batch,
        "loss_first_last": [losses[0][1], losses[-1][1]],
        "held_out": res,
        "seconds": {"data": t_data, "train": t_train},
        "ms_per_600s": {"fine_4_steps": t_fine * 1e3, "coarse_step_plus_corrector": t_corr * 1e3},
        "speedup_vs_fine": t_fine / t_corr,
    }
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
