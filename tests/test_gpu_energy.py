"""Total energy and the energy fixer through the C ABI against the oracle
(the globally uniform internal-energy adjustment the paper implements,
Sec. 3; Williamson 2009)."""
import numpy as np
import pytest

import workloads
from oracle import dynamics as odyn
from tests.conftest import oracle_grid
from tests.gpu_util import lib_fields, lib_state, oracle_fields, cell_errors, say, small_earth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def test_total_energy_matches_the_oracle():
    w = small_earth(glevel=3, n_lev=20, n_large=2, noise=1.0)
    model, ost = odyn.model_from_workload(w, oracle_grid(w.glevel))
    st = lib_state(w)
    for k in range(2):
        e, rc = st.energy()
        ref = odyn.total_energy(model, ost)
        say(f"[energy] {w.name} after {k} steps: rel {abs(e / ref - 1):.2e}")
        assert rc == 0 and abs(e / ref - 1) < 1e-12
        st.step(1, w.n_acoustic)
        ost = odyn.run(model, ost, 1, w.n_acoustic)


def _fixer_parity(w, precision=0):
    say(f"[fixer] {w.name} g{w.glevel} L{w.n_lev} forcing={w.forcing_kind} n_large={w.n_large}")
    st = lib_state(w, precision)
    st.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(st), oracle_fields(w))
    say(f"        errors {err}")
    for k, e in err.items():
        assert e < TOL, (k, e)
    return st


def test_fixer_without_forcing_conserves_energy():
    w = small_earth(glevel=3, n_lev=12, n_large=3, noise=2.0)
    w.diff_D *= 4.0            # more dissipation for the fixer to return
    w.energy_fixer = True
    st = lib_state(w)
    e0, _ = st.energy()
    st.step(1, w.n_acoustic)
    e1, _ = st.energy()
    st.step(2, w.n_acoustic)
    e3, _ = st.energy()
    say(f"[fixer] energy drift {e1 / e0 - 1:.2e}, {e3 / e0 - 1:.2e}")
    assert abs(e1 / e0 - 1) < 1e-13 and abs(e3 / e0 - 1) < 1e-13
    w2 = small_earth(glevel=3, n_lev=12, n_large=3, noise=2.0)
    w2.diff_D *= 4.0
    st2 = lib_state(w2)
    st2.step(3, w2.n_acoustic)
    e3b, _ = st2.energy()
    assert abs(e3b / e0 - 1) > 1e-10              # without the fixer it drifts
    _fixer_parity(w)


def test_fixer_with_newtonian_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.energy_fixer = True
    _fixer_parity(w)


def test_fixer_with_held_suarez_forcing():
    """The fixer runs before the physics, so sigma of the friction and of the
    relaxation is that of the adjusted state."""
    w = workloads.held_suarez(glevel=3, n_lev=37, n_large=3, dt=3000.0, noise_amp=1.0)
    w.energy_fixer = True
    _fixer_parity(w)


def test_fixer_in_mixed_precision_stays_close():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.energy_fixer = True
    st = lib_state(w, precision=1)
    st.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(st, ("T", "p", "rho")), oracle_fields(w))
    say(f"[fixer] mixed errors {err}")
    assert all(e < 1e-5 for e in err.values()), err


def test_ensembles_reject_the_fixer():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=8, n_large=1)
    w.energy_fixer = True
    g = thor.Grid(w.glevel)
    with pytest.raises(thor.ThorError, match="energy fixer"):
        thor.Batch([g], [thor.structs_from_workload(w)])


@pytest.mark.parametrize("shallow", [False, True])
def test_axial_angular_momentum_matches_the_oracle(shallow):
    """The absolute axial angular momentum through the C ABI, at rest and
    after two large steps of the day/night forcing have set up winds (deep
    and shallow forms)."""
    w = workloads.small_gas_giant(glevel=3, n_lev=13, n_large=2)
    w.shallow = shallow
    model, ost = odyn.model_from_workload(w, oracle_grid(w.glevel))
    st = lib_state(w)
    for k in range(2):
        a, rc = st.angular_momentum()
        ref = odyn.axial_angular_momentum(model, ost)
        say(f"[angmom] shallow={shallow} after {2 * k} steps: rel {abs(a / ref - 1):.2e}")
        assert rc == 0 and abs(a / ref - 1) < 1e-12
        st.step(2, w.n_acoustic)
        ost = odyn.run(model, ost, 2, w.n_acoustic)
