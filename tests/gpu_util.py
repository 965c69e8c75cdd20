"""Helpers shared by the GPU tests: run the library and the oracle on the
same seeded workload and compare fields."""
import sys

import numpy as np

import workloads
from oracle import dynamics as odyn
from tests.conftest import oracle_grid

_ORACLE = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_fields(w, n_large=None):
    """Oracle fields after n_large steps (cached per workload recipe)."""
    n_large = w.n_large if n_large is None else n_large
    key = (repr(w), n_large)
    if key not in _ORACLE:
        # built with the C library's atan2, as the host grid builder is: the
        # two grids are then bit-identical
        G = oracle_grid(w.glevel, scalar_atan2=True)
        model, st = odyn.model_from_workload(w, G)
        m0 = odyn.mass(model, st)
        st = odyn.run(model, st, n_large, w.n_acoustic)
        out = odyn.fields(model, st)
        out["_mass0"] = m0
        out["_mass"] = odyn.mass(model, st)
        _ORACLE[key] = out
    return _ORACLE[key]


def lib_state(w, precision=0, device="cuda:0"):
    from paper_1607_05535_amd import thor
    g = thor.Grid(w.glevel)
    return thor.State(g, *thor.structs_from_workload(w, precision), device=device)


def lib_fields(st, names=("T", "u", "v", "w", "p", "rho", "rhotheta")):
    out = {}
    for n in names:
        f, rc = st.field(n)
        assert rc == 0, (n, rc)
        out[n] = f
    return out


WINDS = ("u", "v", "w")


def cell_errors(got, ref):
    """Cell-by-cell errors per field: the largest |got - ref| / |ref| over
    every cell for T, p, rho and rho theta (positive everywhere), and for the
    winds the largest |got - ref| over the RMS speed of the reference (a
    wind component passes through zero, so it has no relative error of its
    own)."""
    speed = np.sqrt(np.mean(ref["u"] ** 2 + ref["v"] ** 2 + ref["w"] ** 2))
    out = {}
    for k in got:
        d = np.abs(got[k] - ref[k])
        out[k] = float(d.max() / speed) if k in WINDS else float((d / np.abs(ref[k])).max())
    return out


def small_earth(glevel=3, n_lev=20, n_large=3, noise=0.1, seed=1):
    w = workloads.earth_c1()
    w.glevel, w.n_lev, w.n_large, w.noise_amp, w.seed = glevel, n_lev, n_large, noise, seed
    w.z_top = 36.0e3 * n_lev / 20
    return w


def read_samples(fname):
    """Stored oracle samples (tests/golden/<fname>, written by
    make_full_size_samples.py): cols, levs, {field: values}, (mass0, mass1)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", fname)
    rows, mass = [], None
    for line in open(path):
        if line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "mass":
            mass = (float(parts[1]), float(parts[2]))
        else:
            rows.append([float(x) for x in parts])
    S = np.array(rows)
    ref = dict(zip(("T", "u", "v", "w", "p", "rho"), S[:, 2:].T))
    return S[:, 0].astype(int), S[:, 1].astype(int), ref, mass


def sample_errors(st, cols, levs, ref):
    """Largest relative error of T, p, rho and largest wind error over the
    samples' RMS speed, from a state's (or ensemble member's) fields."""
    got = {}
    for name in ("T", "u", "v", "w", "p", "rho"):
        f, rc = st.field(name)
        assert rc == 0, name
        got[name] = f[cols, levs]
    return cell_errors(got, ref)


def rounding_response(case):
    """The oracle's own response to a one-ulp perturbation of its initial
    state after one large step (tests/golden/rounding_response_<case>.txt,
    written by make_rounding_response.py from the oracle alone): {field:
    (over the sampled cells, over all cells)}."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"rounding_response_{case}.txt")
    out = {}
    for line in open(path):
        if line.startswith("#"):
            continue
        k, a, b = line.split()
        out[k] = (float(a), float(b))
    return out
