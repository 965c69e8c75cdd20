"""Write the oracle's fields after one large step (two for the hot Jupiter)
of a full-size workload at seeded sample cells.

    python tests/golden/make_full_size_samples.py g6l32   # 40962 columns x 32 levels
    python tests/golden/make_full_size_samples.py g7l48   # 163842 columns x 48 levels
    python tests/golden/make_full_size_samples.py hs_g5l37   # Held-Suarez, 10242 x 37
    python tests/golden/make_full_size_samples.py hj_g5l37   # hot Jupiter, 10242 x 37
    python tests/golden/make_full_size_samples.py g6l32_fixer   # also _hydrostatic, _shallow,
                                                                # _cubic, _anelastic: g6 L32
                                                                # with a switch on
    python tests/golden/make_full_size_samples.py ensemble_member0_g6l48   # first planet of the
                                                                           # 64-planet ensemble

Calls only `oracle/` (FP64 CPU; minutes for g6, about 15 for g7): the stored
values are the oracle's, never the library's.  Output (named by out_name):
one line per sample "col lev T u v w p rho", then a line "mass mass0 mass1".
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SAMPLES = 600
SAMPLE_SEED = 20161  # fixes which cells are sampled


def _workload(case):
    import workloads
    return {"g6l32": workloads.gas_giant_c2, "g7l48": workloads.gas_giant_c3,
            "hs_g5l37": lambda: workloads.held_suarez(glevel=5, n_lev=37),
            "hj_g5l37": lambda: workloads.hot_jupiter(glevel=5, n_lev=37),
            "g6l32_fixer": lambda: _switched("energy_fixer", True),
            "g6l32_hydrostatic": lambda: _switched("hydrostatic", True),
            "g6l32_shallow": lambda: _switched("shallow", True),
            "g6l32_cubic": lambda: _switched("lagrange_order", 3),
            "g6l32_anelastic": lambda: _switched("anelastic", True),
            "ensemble_member0_g6l48": lambda: workloads.ensemble()[0]}[case]()


def _switched(attr, value):
    """The g6 L32 gas giant with one of its switches set."""
    import workloads
    w = workloads.gas_giant_c2()
    setattr(w, attr, value)
    return w


CASES = ("g6l32", "g7l48", "hs_g5l37", "hj_g5l37",
         "g6l32_fixer", "g6l32_hydrostatic", "g6l32_shallow", "g6l32_cubic", "g6l32_anelastic",
         "ensemble_member0_g6l48")
# the hot Jupiter starts at rest with no noise: its winds appear in the
# second step, once the first step's relaxation has set up the day/night
# contrast
N_STEPS = {"hj_g5l37": 2}


def out_name(case):
    if case.startswith(("g6l32", "g7l48")):
        return f"gas_giant_{case}_one_step.txt"
    return f"{case}_two_steps.txt" if N_STEPS.get(case, 1) == 2 else f"{case}_one_step.txt"


def main(case):
    from oracle import dynamics as odyn
    from oracle import grid as ogrid

    w = _workload(case)
    # the C library's atan2 makes the oracle's grid bit-identical to the
    # host builder's (NumPy's vectorised atan2 differs in the last bit, which
    # the spring relaxation would amplify into the winds)
    G = ogrid.Grid(w.glevel, k=100.0, scalar_atan2=True)
    model, st = odyn.model_from_workload(w, G)
    m0 = odyn.mass(model, st)
    n_steps = N_STEPS.get(case, 1)
    st = odyn.run(model, st, n_steps, w.n_acoustic)
    f = odyn.fields(model, st)
    m1 = odyn.mass(model, st)
    rs = np.random.default_rng(SAMPLE_SEED)
    cols = rs.integers(0, w.n_col, N_SAMPLES)
    levs = rs.integers(0, w.n_lev, N_SAMPLES)
    # always include the poles, a ring pentagon and the bottom and top levels
    pent = int(np.flatnonzero(np.asarray(G.deg) == 5)[0])
    cols[:4] = [w.n_col - 2, w.n_col - 1, pent, pent]
    levs[:4] = [0, w.n_lev - 1, 0, w.n_lev - 1]
    path = os.path.join(HERE, out_name(case))
    with open(path, "w") as fh:
        fh.write(f"# oracle fields after {n_steps} large step(s) of {w.name} "
                 f"(dt {w.dt:g} s, n = {w.n_acoustic}),\n")
        fh.write(f"# written by make_full_size_samples.py {case}; col lev T u v w p rho\n")
        for c, k in zip(cols, levs):
            vals = [f[name][c, k] for name in ("T", "u", "v", "w", "p", "rho")]
            fh.write(f"{c} {k} " + " ".join(repr(float(v)) for v in vals) + "\n")
        fh.write(f"mass {m0!r} {m1!r}\n")
    print("wrote", path)


if __name__ == "__main__":
    if len(sys.argv) != 2 or sys.argv[1] not in CASES:
        sys.exit("usage: make_full_size_samples.py " + "|".join(CASES))
    main(sys.argv[1])
