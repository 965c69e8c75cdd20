"""The switchable approximations of Sec. 3 through the C ABI against the
oracle (FP64 parity, same bar as the default equations)."""
import pytest

import workloads
from tests.gpu_util import lib_fields, lib_state, oracle_fields, cell_errors, say, small_earth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _parity(w, precision=0, tol=TOL, names=("T", "u", "v", "w", "p", "rho", "rhotheta")):
    say(f"[variant] {w.name} g{w.glevel} L{w.n_lev} hydrostatic={w.hydrostatic} shallow={w.shallow} order={w.lagrange_order} "
        f"anelastic={w.anelastic} n_large={w.n_large} precision={precision}")
    st = lib_state(w, precision)
    st.step(w.n_large, w.n_acoustic)
    got = lib_fields(st, names)
    ref = oracle_fields(w)
    err = cell_errors(got, ref)
    say(f"          errors {err}")
    for k, e in err.items():
        assert e < tol, (k, e)


@pytest.mark.parametrize("n_lev", [1, 12, 33])
def test_hydrostatic_earth(n_lev):
    w = small_earth(glevel=3, n_lev=n_lev, n_large=3, noise=1.0)
    w.hydrostatic = True
    _parity(w)


def test_hydrostatic_gas_giant_with_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.hydrostatic = True
    _parity(w)


def test_hydrostatic_mixed_precision_stays_close():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.hydrostatic = True
    _parity(w, precision=1, tol=1e-5, names=("T", "p", "rho"))


@pytest.mark.parametrize("n_lev", [1, 12, 33])
def test_shallow_earth(n_lev):
    """Level counts with and without the 4-level vector path of the slow
    kernel, and one level."""
    w = small_earth(glevel=3, n_lev=n_lev, n_large=3, noise=1.0)
    w.shallow = True
    _parity(w)


def test_shallow_gas_giant_with_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.shallow = True
    _parity(w)


def test_shallow_and_hydrostatic_together():
    w = small_earth(glevel=3, n_lev=16, n_large=3, noise=1.0)
    w.shallow = True
    w.hydrostatic = True
    _parity(w)


def test_shallow_mixed_precision_stays_close():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.shallow = True
    _parity(w, precision=1, tol=1e-5, names=("T", "p", "rho"))


def test_ensembles_reject_the_shallow_form():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=8, n_large=1)
    w.shallow = True
    g = thor.Grid(w.glevel)
    with pytest.raises(thor.ThorError, match="shallow"):
        thor.Batch([g], [thor.structs_from_workload(w)])


@pytest.mark.parametrize("n_lev", [4, 12, 33])
def test_cubic_vertical_interpolation_earth(n_lev):
    """Order-3 Lagrange interpolation: the fewest levels it allows, the
    4-level vector path, and ragged lanes."""
    w = small_earth(glevel=3, n_lev=n_lev, n_large=3, noise=1.0)
    w.lagrange_order = 3
    _parity(w)


def test_cubic_vertical_interpolation_gas_giant_with_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.lagrange_order = 3
    _parity(w)


def test_cubic_shallow_hydrostatic_together():
    w = small_earth(glevel=3, n_lev=16, n_large=3, noise=1.0)
    w.lagrange_order = 3
    w.shallow = True
    w.hydrostatic = True
    _parity(w)


def test_cubic_mixed_precision_stays_close():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.lagrange_order = 3
    _parity(w, precision=1, tol=1e-5, names=("T", "p", "rho"))


def test_order_zero_is_order_one_and_bad_orders_are_rejected():
    import numpy as np
    from paper_1607_05535_amd import thor
    outs = []
    for order in (0, 1):
        w = small_earth(glevel=2, n_lev=8, n_large=2, noise=1.0)
        w.lagrange_order = order
        st = lib_state(w)
        st.step(w.n_large, w.n_acoustic)
        outs.append(lib_fields(st, ("T", "u")))
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k])
    for order, n_lev in ((2, 8), (3, 3), (4, 8)):
        w = small_earth(glevel=2, n_lev=n_lev, n_large=1)
        w.lagrange_order = order
        with pytest.raises(thor.ThorError, match="lagrange_order"):
            lib_state(w)


@pytest.mark.parametrize("n_lev", [1, 13, 32])
def test_anelastic_earth(n_lev):
    """The reference-density mass flux of Sec. 3: one level (horizontal
    flux only), a ragged top lane, and whole lanes."""
    w = small_earth(glevel=3, n_lev=n_lev, n_large=3, noise=1.0)
    w.anelastic = True
    _parity(w)


@pytest.mark.parametrize("glevel,n_lev", [(0, 2), (1, 7), (2, 64)])
def test_anelastic_edge_sizes(glevel, n_lev):
    """The 12 pentagons alone (g0) with two levels (one interior
    interface), g1 with an odd level count, and the largest level count."""
    w = small_earth(glevel=glevel, n_lev=n_lev, n_large=2, noise=1.0)
    w.anelastic = True
    _parity(w)


def test_anelastic_gas_giant_with_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=19, n_large=3)
    w.anelastic = True
    _parity(w)


def test_anelastic_hydrostatic_shallow_together():
    w = small_earth(glevel=3, n_lev=16, n_large=3, noise=1.0)
    w.anelastic = True
    w.hydrostatic = True
    w.shallow = True
    _parity(w)


def test_anelastic_held_suarez_with_energy_fixer():
    w = workloads.held_suarez(glevel=3, n_lev=37, n_large=3, dt=3000.0, noise_amp=1.0)
    w.anelastic = True
    w.energy_fixer = True
    _parity(w)


def test_anelastic_mixed_precision_stays_close():
    w = workloads.small_gas_giant(glevel=3, n_lev=20, n_large=3)
    w.anelastic = True
    _parity(w, precision=1, tol=1e-5, names=("T", "p", "rho"))


def test_anelastic_conserves_mass_and_changes_the_flow():
    """The reference-density flux is still a flux divergence, so the total
    mass keeps to rounding; and the switch is live: the winds differ from
    the compressible run's by far more than the parity bar."""
    import numpy as np
    w = small_earth(glevel=4, n_lev=24, n_large=4, noise=2.0)
    w.anelastic = True
    a = lib_state(w)
    m0, _ = a.mass()
    a.step(w.n_large, w.n_acoustic)
    m1, _ = a.mass()
    say(f"[variant] anelastic mass {m0!r} -> {m1!r}")
    assert abs(m1 - m0) < 1e-13 * m0
    w.anelastic = False
    b = lib_state(w)
    b.step(w.n_large, w.n_acoustic)
    fa, fb = lib_fields(a, ("u", "w")), lib_fields(b, ("u", "w"))
    speed = np.sqrt(np.mean(fb["u"] ** 2))
    assert np.abs(fa["u"] - fb["u"]).max() > 1e-6 * speed
    assert np.abs(fa["w"] - fb["w"]).max() > 0


def test_anelastic_keeps_the_four_level_mapping():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=36, n_large=1)
    w.anelastic = True
    st = lib_state(w)
    for nl in (1, 2):
        with pytest.raises(thor.ThorError, match="anelastic"):
            thor.thor_set_vert_levels_per_lane(st.handle, nl)
    thor.thor_set_vert_levels_per_lane(st.handle, 4)
    w.lagrange_order = 3
    with pytest.raises(thor.ThorError, match="anelastic"):
        lib_state(w)


@pytest.mark.parametrize("switches", [
    dict(energy_fixer=True, hydrostatic=True),
    dict(shallow=True, lagrange_order=3),
    dict(anelastic=True, hydrostatic=True),
    dict(energy_fixer=True, shallow=True, lagrange_order=3, forcing_kind=1)])
def test_switches_under_graphs_checkpoints_and_autotune(switches):
    """With the switches on: graph replays equal eager launches bitwise,
    a checkpoint restart equals a straight run bitwise, and autotuning
    leaves the state as it found it."""
    import numpy as np
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=3, n_lev=16, n_large=4, noise=1.0)
    for k, v in switches.items():
        setattr(w, k, v)
    say(f"[variant] runtime checks {switches}")
    a = lib_state(w)
    a.step(4, 6)
    ref = a.export()[0]
    b = lib_state(w)
    thor.thor_set_timing(b.handle, 1)      # eager launches
    b.step(4, 6)
    thor.thor_set_timing(b.handle, 0)
    assert np.array_equal(b.export()[0], ref)
    c = lib_state(w)
    c.step(2, 6)
    blob = c.export()[0]
    d = lib_state(w)
    d.load(blob)
    thor.thor_autotune(d.handle, 6)
    assert np.array_equal(d.export()[0], blob)
    # the tuner may have chosen another phase-V mapping (equal to rounding);
    # back on the default one the restart equals the straight run bitwise
    # (workgroup sizes do not change the arithmetic)
    thor.thor_set_vert_levels_per_lane(d.handle, 4 if w.lagrange_order == 1 else 1)
    d.step(2, 6)
    assert np.array_equal(d.export()[0], ref)
