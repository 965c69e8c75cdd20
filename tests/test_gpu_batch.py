"""Ensemble form: many planets with different grid levels, layer counts and
constants advanced by one launch per phase.  Each member must equal the same
planet advanced alone, bitwise (FP64)."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import read_samples, sample_errors, say

pytestmark = pytest.mark.gpu


def _small_ensemble():
    ws = workloads.ensemble(n=6, seed=11, glevels=(2, 3), levels=(7, 20, 33, 48))
    ws[0].forcing_kind, ws[0].tau, ws[0].T_mean, ws[0].dT_daynight = 1, 1e5, ws[0].T0, 40.0
    ws[1].forcing_kind = 3   # Held-Suarez: relaxation and the separate friction launch
    return ws


def _grids(ws):
    from paper_1607_05535_amd import thor
    cache = {}
    return [cache.setdefault(w.glevel, thor.Grid(w.glevel)) for w in ws]


@pytest.mark.parametrize("precision", [0, 1])
def test_members_equal_single_runs_bitwise(precision):
    from paper_1607_05535_amd import thor
    ws = _small_ensemble()
    say(f"[batch] {[w.name for w in ws]} precision={precision}")
    grids = _grids(ws)
    members = []
    for i, w in enumerate(ws):
        pl, v, num, fo, ini = thor.structs_from_workload(w, precision)
        ini.planet_index = i
        members.append((pl, v, num, fo, ini))
    b = thor.Batch(grids, members)
    b.step(3, 8)
    for i, (w, m) in enumerate(zip(ws, members)):
        st = thor.State(grids[i], *m)
        st.step(3, 8)
        ref, rc0 = st.export()
        got, rc1 = b.members[i].export()
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(got, ref), w.name


def test_member_cannot_be_stepped_alone():
    from paper_1607_05535_amd import thor
    ws = _small_ensemble()[:2]
    grids = _grids(ws)
    b = thor.Batch(grids, [thor.structs_from_workload(w) for w in ws])
    with pytest.raises(thor.ThorError) as e:
        thor.thor_step(b.members[0].handle, 1, 8)
    assert e.value.code == thor.THOR_EINVAL


def test_batch_autotune_leaves_state_unchanged():
    from paper_1607_05535_amd import thor
    ws = _small_ensemble()
    grids = _grids(ws)
    b = thor.Batch(grids, [thor.structs_from_workload(w) for w in ws])
    b.step(1, 8)
    before = [m.export()[0] for m in b.members]
    wpb = b.autotune(8)
    assert set(wpb.values()) <= {1, 2, 4, 8}
    after = [m.export()[0] for m in b.members]
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    b.step(2, 8)
    a = thor.Batch(grids, [thor.structs_from_workload(w) for w in ws])
    a.step(3, 8)
    for m1, m2 in zip(a.members, b.members):
        assert np.array_equal(m1.export()[0], m2.export()[0])


def test_sixty_four_planet_ensemble():
    """The ensemble workload: 64 planets, g in {4,5,6}, L in {20,32,48}."""
    from paper_1607_05535_amd import thor
    ws = workloads.ensemble()
    grids = _grids(ws)
    members = []
    for i, w in enumerate(ws):
        pl, v, num, fo, ini = thor.structs_from_workload(w)
        ini.planet_index = i
        members.append((pl, v, num, fo, ini))
    b = thor.Batch(grids, members)
    m0 = [m.mass()[0] for m in b.members]
    b.step(2, 8)
    for i, m in enumerate(b.members):
        mass, rc = m.mass()
        assert rc == 0, ws[i].name
        assert abs(mass / m0[i] - 1) < 1e-13, ws[i].name


def test_ensemble_member_at_full_size_matches_stored_oracle_samples():
    """The 64-planet ensemble in the benchmark's launch configuration
    (autotuned, one graph-replayed large step for all planets): its first
    planet (g6, 40962 columns x 48 levels) against the oracle's stored
    samples (tests/golden/ensemble_member0_g6l48_one_step.txt), every field
    to 1e-10."""
    from paper_1607_05535_amd import thor
    ws = workloads.ensemble()
    cols, levs, ref, mass = read_samples("ensemble_member0_g6l48_one_step.txt")
    grids = _grids(ws)
    members = []
    for i, w in enumerate(ws):
        pl, v, num, fo, ini = thor.structs_from_workload(w)
        ini.planet_index = i
        members.append((pl, v, num, fo, ini))
    b = thor.Batch(grids, members)
    tuned = b.autotune(8)
    say(f"[batch] 64 planets, tuned {tuned}; member 0 {ws[0].name}")
    m0, rc = b.members[0].mass()
    assert rc == 0 and abs(m0 / mass[0] - 1) < 1e-13
    b.step(1, 8)
    errs = sample_errors(b.members[0], cols, levs, ref)
    say(f"        max errors {errs}")
    for k, e in errs.items():
        assert e < 1e-10, (k, e)
    m1, rc = b.members[0].mass()
    assert rc == 0 and abs(m1 / mass[1] - 1) < 1e-12
