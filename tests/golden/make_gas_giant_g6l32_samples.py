"""Write the oracle's fields after one large step of the g6 L32 gas-giant
benchmark workload at seeded sample cells.

    python tests/golden/make_gas_giant_g6l32_samples.py

Calls only `oracle/` (FP64 CPU, a few minutes): the stored values are the
oracle's, never the library's.  Output: gas_giant_g6l32_one_step.txt, one
line per sample "col lev T u v w p rho", then a line "mass0 mass1".
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SAMPLES = 600
SAMPLE_SEED = 20161  # fixes which cells are sampled


def main():
    import workloads
    from oracle import dynamics as odyn
    from oracle import grid as ogrid

    w = workloads.gas_giant_c2()
    G = ogrid.Grid(w.glevel, k=100.0)
    model, st = odyn.model_from_workload(w, G)
    m0 = odyn.mass(model, st)
    st = odyn.run(model, st, 1, w.n_acoustic)
    f = odyn.fields(model, st)
    m1 = odyn.mass(model, st)
    rs = np.random.default_rng(SAMPLE_SEED)
    cols = rs.integers(0, w.n_col, N_SAMPLES)
    levs = rs.integers(0, w.n_lev, N_SAMPLES)
    # always include the poles, a ring pentagon and the bottom and top levels
    pent = int(np.flatnonzero(np.asarray(G.deg) == 5)[0])
    cols[:4] = [w.n_col - 2, w.n_col - 1, pent, pent]
    levs[:4] = [0, w.n_lev - 1, 0, w.n_lev - 1]
    path = os.path.join(HERE, "gas_giant_g6l32_one_step.txt")
    with open(path, "w") as fh:
        fh.write("# oracle fields after 1 large step of the g6 L32 gas giant (dt 300 s, n = 8),\n")
        fh.write("# written by make_gas_giant_g6l32_samples.py; col lev T u v w p rho\n")
        for c, k in zip(cols, levs):
            vals = [f[name][c, k] for name in ("T", "u", "v", "w", "p", "rho")]
            fh.write(f"{c} {k} " + " ".join(repr(float(v)) for v in vals) + "\n")
        fh.write(f"mass {m0!r} {m1!r}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
