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
        G = oracle_grid(w.glevel)
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


def rel_errors(got, ref):
    """Per-field relative L2 errors; winds are measured against the speed."""
    speed = np.sqrt(ref["u"] ** 2 + ref["v"] ** 2 + ref["w"] ** 2)
    out = {}
    for k in got:
        den = np.linalg.norm(speed) if k in ("u", "v", "w") else np.linalg.norm(ref[k])
        out[k] = float(np.linalg.norm(got[k] - ref[k]) / den)
    return out


def small_earth(glevel=3, n_lev=20, n_large=3, noise=0.1, seed=1):
    w = workloads.earth_c1()
    w.glevel, w.n_lev, w.n_large, w.noise_amp, w.seed = glevel, n_lev, n_large, noise, seed
    w.z_top = 36.0e3 * n_lev / 20
    return w
