"""FP64 parity of the HIP path with the oracle, through the C ABI."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import (cell_errors, lib_fields, lib_state, oracle_fields, read_samples, rounding_response,
                             sample_errors, say, small_earth)

pytestmark = pytest.mark.gpu

# FP64 path: largest cell error after the run (relative for T, p, rho and
# rho theta; over the RMS speed for the winds); the oracle's grid is
# bit-identical to the host grid, so every field keeps this bar
TOL = 1e-10


def _compare(w, tol=TOL, precision=0):
    say(f"[parity] {w.name} g{w.glevel} L{w.n_lev} n_large={w.n_large} n={w.n_acoustic}")
    st = lib_state(w, precision)
    st.step(w.n_large, w.n_acoustic)
    got = lib_fields(st)
    ref = oracle_fields(w)
    err = cell_errors(got, ref)
    say(f"         errors {err}")
    for k, e in err.items():
        assert e < tol, (k, e)
    mass, rc = st.mass()
    assert rc == 0
    assert abs(mass / ref["_mass0"] - 1) < 1e-13
    return st, got, ref


def test_c1_earth_g4_l20_ten_steps():
    """The CPU-sized workload: g4 (2562 columns) x 20 levels, 10 steps of
    600 s with 6 substeps, +/-0.1 K noise."""
    _compare(workloads.earth_c1())


def test_gas_giant_with_newtonian_forcing():
    _compare(workloads.small_gas_giant(glevel=3, n_lev=32, n_large=3))


@pytest.mark.parametrize("n_lev", [1, 2, 7, 20, 33, 48, 64])
def test_ragged_level_counts(n_lev):
    """Columns per wavefront 64, 32, 9, 3, 1, 1, 1: padding lanes, odd L and
    a full wavefront per column."""
    _compare(small_earth(glevel=2, n_lev=n_lev, n_large=2))


def test_no_divergence_damping_and_no_diffusion():
    w = small_earth(glevel=3, n_lev=12, n_large=2)
    w.div_damp = False
    w.diff_D = 0.0
    _compare(w)


def test_rest_state_stays_at_rest_on_gpu():
    w = small_earth(glevel=3, n_lev=20, n_large=5, noise=0.0)
    st = lib_state(w)
    st.step(w.n_large, w.n_acoustic)
    f = lib_fields(st, ("u", "v", "w"))
    for k, v in f.items():
        assert np.abs(v).max() < 1e-8, k


def _full_size_samples(fname, w, precision, tol_thermo, tol_wind, n_steps=1, tol_w=None):
    """Full-size workload in the benchmark's launch configuration
    (autotuned workgroup sizes, graph replay of thor_step): after n_steps
    large steps the sampled cells are compared with the oracle's stored
    values (tests/golden/<fname>, written by make_full_size_samples.py
    beside it from the oracle alone)."""
    from paper_1607_05535_amd import thor
    cols, levs, ref, mass = read_samples(fname)
    say(f"[parity] full size {w.name} precision={precision}: autotune, {n_steps} graph-replayed large step(s), "
        f"{len(cols)} samples")
    st = lib_state(w, precision)
    tuned = thor.thor_autotune(st.handle, w.n_acoustic)
    say(f"         tuned {tuned}")
    m0, rc = st.mass()
    assert rc == 0 and abs(m0 / mass[0] - 1) < 1e-13
    st.step(n_steps, w.n_acoustic)
    errs = sample_errors(st, cols, levs, ref)
    say(f"         max errors {errs}")
    for k in ("T", "p", "rho"):
        assert errs[k] < tol_thermo, (k, errs[k])
    for k in ("u", "v", "w"):
        bar = tol_w if (k == "w" and tol_w is not None) else tol_wind
        assert errs[k] < bar, (k, errs[k], bar)
    m1, rc = st.mass()
    assert rc == 0 and abs(m1 / mass[1] - 1) < 1e-12


# the mixed form's bars against the oracle after one or two steps at full
# size: about 20 times the largest errors measured over these workloads
# (thermodynamic 4.5e-10, winds 3.5e-7 of the RMS speed)
MIXED_THERMO, MIXED_WIND = 1e-8, 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_gas_giant_g6_l32_full_size_samples_after_one_step(precision):
    """The benchmark workload at full size (40962 columns x 32 levels), FP64
    and mixed."""
    tol = (TOL, TOL) if precision == 0 else (MIXED_THERMO, MIXED_WIND)
    _full_size_samples("gas_giant_g6l32_one_step.txt", workloads.gas_giant_c2(), precision, *tol)


@pytest.mark.parametrize("precision", [0, 1])
def test_gas_giant_g7_l48_full_size_samples_after_one_step(precision):
    """The largest single-planet workload (163842 columns x 48 levels) in
    FP64 and in the mixed form it is run in, whose FP32 horizontal stencils
    leave relative errors of order 1e-7 in T, p and rho after a step
    (bounded as in the mixed-form tests)."""
    if precision == 0:
        _full_size_samples("gas_giant_g7l48_one_step.txt", workloads.gas_giant_c3(), 0, TOL, TOL)
    else:
        _full_size_samples("gas_giant_g7l48_one_step.txt", workloads.gas_giant_c3(), 1, MIXED_THERMO, MIXED_WIND)


@pytest.mark.parametrize("attr,value", [("energy_fixer", True), ("hydrostatic", True), ("shallow", True),
                                        ("lagrange_order", 3), ("anelastic", True)])
def test_gas_giant_g6_l32_switches_full_size_samples_after_one_step(attr, value):
    """The benchmark workload with each of the switches the benchmark times
    (energy fixer, hydrostatic, shallow, cubic vertical interpolation,
    anelastic)."""
    w = workloads.gas_giant_c2()
    setattr(w, attr, value)
    name = {"energy_fixer": "fixer", "hydrostatic": "hydrostatic", "shallow": "shallow",
            "lagrange_order": "cubic", "anelastic": "anelastic"}[attr]
    tol_w = None
    if attr == "hydrostatic":
        # the hydrostatic form diagnoses W from a nearly cancelling balance:
        # one large step of the oracle itself moves w by 4.7e-10 of the RMS
        # speed when its initial state is perturbed by one ulp (stored
        # measurement), so two correct FP64 implementations, whose roundings
        # differ by a few such perturbations, cannot agree to 1e-10 there;
        # the w bar is four times that response
        tol_w = max(TOL, 4.0 * rounding_response("g6l32_hydrostatic")["w"][1])
    _full_size_samples(f"gas_giant_g6l32_{name}_one_step.txt", w, 0, TOL, TOL, tol_w=tol_w)


@pytest.mark.parametrize("precision", [0, 1])
def test_held_suarez_g5_l37_full_size_samples_after_one_step(precision):
    """The paper's Earth benchmark setup at its own size (10242 columns x 37
    levels), autotuned (phase V may take the two-levels-per-lane mapping),
    FP64 and mixed."""
    tol = (TOL, TOL) if precision == 0 else (MIXED_THERMO, MIXED_WIND)
    _full_size_samples("hs_g5l37_one_step.txt", workloads.held_suarez(glevel=5, n_lev=37), precision, *tol)


@pytest.mark.parametrize("precision", [0, 1])
def test_hot_jupiter_g5_l37_full_size_samples_after_two_steps(precision):
    """The paper's hot-Jupiter setup at its own size, FP64 and mixed; it
    starts at rest, so the winds compared are those of the second step."""
    tol = (TOL, TOL) if precision == 0 else (MIXED_THERMO, MIXED_WIND)
    _full_size_samples("hj_g5l37_two_steps.txt", workloads.hot_jupiter(glevel=5, n_lev=37), precision, *tol,
                       n_steps=2)


def test_hot_jupiter_benchmark_forcing():
    """The hot-Jupiter benchmark physics (Eqs. teq-hj, btrop, tvert; 37 layers
    to 4875 km, a level count that is not a multiple of 4) on g3 with a step
    scaled to the coarser grid."""
    w = workloads.hot_jupiter(glevel=3, n_lev=37, n_large=3, dt=2400.0, noise_amp=0.1)
    _compare(w)


def test_held_suarez_forcing():
    """The Earth benchmark physics (Held-Suarez relaxation and boundary-layer
    friction, 37 layers to 32 km) on g3 with a step scaled to the coarser grid."""
    w = workloads.held_suarez(glevel=3, n_lev=37, n_large=4, dt=3000.0, noise_amp=1.0)
    _compare(w)


@pytest.mark.parametrize("nl", [1, 2, 4])
@pytest.mark.parametrize("case", ["held_suarez_37", "earth_48", "earth_33_hydrostatic"])
def test_phase_v_mappings_above_32_levels(nl, case):
    """One, two and four levels per lane in phase V (the autotuner chooses
    among them for 33-64 levels): each matches the oracle, with forcing in
    the last substep and with the hydrostatic rows."""
    from paper_1607_05535_amd import thor
    if case == "held_suarez_37":
        w = workloads.held_suarez(glevel=3, n_lev=37, n_large=3, dt=3000.0, noise_amp=1.0)
    elif case == "earth_48":
        w = small_earth(glevel=3, n_lev=48, n_large=2)
    else:
        w = small_earth(glevel=3, n_lev=33, n_large=2)
        w.hydrostatic = True
    say(f"[parity] {w.name} phase V with {nl} level(s) per lane")
    st = lib_state(w)
    thor.thor_set_vert_levels_per_lane(st.handle, nl)
    st.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(st), oracle_fields(w))
    say(f"         errors {err}")
    for k, e in err.items():
        assert e < TOL, (k, e)


@pytest.mark.parametrize("n_lev", [1, 2, 3, 4, 5, 7, 13, 20, 32, 64])
def test_phase_v_four_levels_per_lane(n_lev):
    """Four levels per lane in phase V at every kind of level count: one lane
    per column with identity rows above the top (1-4), a partly filled top
    lane (5, 7, 13), 5 lanes x 12 columns (20), 8 x 8 (32), 16 x 4 (64)."""
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=n_lev, n_large=2)
    say(f"[parity] {w.name} L{n_lev} phase V with 4 levels per lane")
    st = lib_state(w)
    thor.thor_set_vert_levels_per_lane(st.handle, 4)
    st.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(st), oracle_fields(w))
    say(f"         errors {err}")
    for k, e in err.items():
        assert e < TOL, (k, e)


@pytest.mark.parametrize("case", ["gas_giant_32", "hot_jupiter_37", "hydrostatic_20", "no_damping_12"])
def test_phase_v_four_levels_per_lane_with_forcing_and_switches(case):
    """The four-levels mapping with Newtonian and hot-Jupiter relaxation in
    the last substep, the hydrostatic rows, and without damping/diffusion."""
    from paper_1607_05535_amd import thor
    if case == "gas_giant_32":
        w = workloads.small_gas_giant(glevel=3, n_lev=32, n_large=3)
    elif case == "hot_jupiter_37":
        w = workloads.hot_jupiter(glevel=3, n_lev=37, n_large=3, dt=2400.0, noise_amp=0.1)
    elif case == "hydrostatic_20":
        w = small_earth(glevel=3, n_lev=20, n_large=2, noise=1.0)
        w.hydrostatic = True
    else:
        w = small_earth(glevel=3, n_lev=12, n_large=2)
        w.div_damp = False
        w.diff_D = 0.0
    say(f"[parity] {w.name} ({case}) phase V with 4 levels per lane")
    st = lib_state(w)
    thor.thor_set_vert_levels_per_lane(st.handle, 4)
    st.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(st), oracle_fields(w))
    say(f"         errors {err}")
    for k, e in err.items():
        assert e < TOL, (k, e)


def test_vert_mapping_argument_errors():
    from paper_1607_05535_amd import thor
    st = lib_state(small_earth(glevel=2, n_lev=20, n_large=1))
    for nl in (0, 2, 3, 8):
        with pytest.raises(thor.ThorError, match="levels_per_lane"):
            thor.thor_set_vert_levels_per_lane(st.handle, nl)
    w3 = small_earth(glevel=2, n_lev=20, n_large=1)
    w3.lagrange_order = 3
    st3 = lib_state(w3)
    with pytest.raises(thor.ThorError, match="levels_per_lane"):
        thor.thor_set_vert_levels_per_lane(st3.handle, 4)
    thor.thor_set_vert_levels_per_lane(st.handle, 4)
    thor.thor_set_vert_levels_per_lane(st.handle, 1)


@pytest.mark.parametrize("glevel", [0, 1])
def test_smallest_grids(glevel):
    """The icosahedron itself (12 pentagon columns, whose two-rings cover
    the whole sphere) and its first bisection (42 columns)."""
    w = small_earth(glevel=glevel, n_lev=9, n_large=2, noise=1.0)
    w.dt = 600.0 * 2 ** (4 - glevel)
    _compare(w)


def test_zero_large_steps_leave_the_state_unchanged():
    w = small_earth(glevel=2, n_lev=8, n_large=0)
    st = lib_state(w)
    before = st.export()[0]
    st.step(0, w.n_acoustic)
    assert np.array_equal(st.export()[0], before)
