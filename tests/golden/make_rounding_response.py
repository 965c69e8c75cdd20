"""Measure how much one large step of the oracle moves when its initial
state is perturbed by one unit in the last place: the rounding sensitivity
of the problem itself, which bounds how closely any two correct FP64
implementations of the step can agree.

    python tests/golden/make_rounding_response.py g6l32_hydrostatic
    python tests/golden/make_rounding_response.py g6l32

The oracle runs one large step from the workload's initial state and from
the same state with every rho and rho theta multiplied by 1 +/- 2^-52
(signs from a seeded generator).  Writes rounding_response_<case>.txt: per
field the largest difference over the sampled cells of
make_full_size_samples.py and over all cells, relative for T, p, rho, over
the RMS speed for u, v, w.  Calls only `oracle/`.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import make_full_size_samples as samples  # noqa: E402

PERTURB_SEED = 7


def main(case):
    from oracle import dynamics as odyn
    from oracle import grid as ogrid

    w = samples._workload(case)
    G = ogrid.Grid(w.glevel, k=100.0, scalar_atan2=True)
    model, st = odyn.model_from_workload(w, G)
    rs = np.random.default_rng(PERTURB_SEED)
    st2 = st.copy()
    st2.rho = st.rho * (1.0 + np.spacing(1.0) * rs.choice([-1.0, 1.0], st.rho.shape))
    st2.rth = st.rth * (1.0 + np.spacing(1.0) * rs.choice([-1.0, 1.0], st.rth.shape))
    a = odyn.fields(model, odyn.run(model, st, 1, w.n_acoustic))
    b = odyn.fields(model, odyn.run(model, st2, 1, w.n_acoustic))
    rs = np.random.default_rng(samples.SAMPLE_SEED)
    cols = rs.integers(0, w.n_col, samples.N_SAMPLES)
    levs = rs.integers(0, w.n_lev, samples.N_SAMPLES)
    pent = int(np.flatnonzero(np.asarray(G.deg) == 5)[0])
    cols[:4] = [w.n_col - 2, w.n_col - 1, pent, pent]
    levs[:4] = [0, w.n_lev - 1, 0, w.n_lev - 1]
    sp_s = np.sqrt(np.mean(a["u"][cols, levs] ** 2 + a["v"][cols, levs] ** 2 + a["w"][cols, levs] ** 2))
    sp_a = np.sqrt(np.mean(a["u"] ** 2 + a["v"] ** 2 + a["w"] ** 2))
    path = os.path.join(HERE, f"rounding_response_{case}.txt")
    with open(path, "w") as fh:
        fh.write(f"# one large step of {w.name} from its initial state and from that state with rho and\n"
                 f"# rho theta perturbed by one ulp (seed {PERTURB_SEED}); written by make_rounding_response.py\n"
                 f"# {case}; field, largest difference over the samples, over all cells (relative for\n"
                 f"# T p rho, over the RMS speed for u v w)\n")
        for k in ("T", "u", "v", "w", "p", "rho"):
            if k in ("u", "v", "w"):
                s_ = np.abs(a[k][cols, levs] - b[k][cols, levs]).max() / sp_s
                all_ = np.abs(a[k] - b[k]).max() / sp_a
            else:
                s_ = np.abs(a[k][cols, levs] / b[k][cols, levs] - 1).max()
                all_ = np.abs(a[k] / b[k] - 1).max()
            fh.write(f"{k} {float(s_)!r} {float(all_)!r}\n")
    print("wrote", path)


if __name__ == "__main__":
    if len(sys.argv) != 2 or sys.argv[1] not in samples.CASES:
        sys.exit("usage: make_rounding_response.py " + "|".join(samples.CASES))
    main(sys.argv[1])
