"""Runtime behaviour of libthor on the GPU through the C ABI: error paths,
checkpoints, determinism, graph replay vs eager launches, non-finite
detection, and the C2-sized workload's invariants."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import lib_fields, lib_state, say, small_earth

pytestmark = pytest.mark.gpu


def test_step_argument_errors_enqueue_nothing():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=8)
    st = lib_state(w)
    before = st.export()[0]
    for n_large, n in ((1, 0), (1, 3), (1, 7), (-1, 6), (2, 1)):
        with pytest.raises(thor.ThorError) as e:
            st.step(n_large, n)
        assert e.value.code == thor.THOR_EINVAL
    after = st.export()[0]
    assert np.array_equal(before, after)


def test_checkpoint_restart_is_bitwise():
    """Export after 3 steps, import into a fresh state, 2 more steps equal 5
    straight steps bitwise."""
    w = small_earth(glevel=3, n_lev=16)
    a = lib_state(w)
    a.step(5, 6)
    ref = a.export()[0]
    b = lib_state(w)
    b.step(3, 6)
    blob = b.export()[0]
    c = lib_state(w)
    c.load(blob)
    c.step(2, 6)
    assert np.array_equal(c.export()[0], ref)


def test_runs_are_deterministic_and_graph_equals_eager():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=3, n_lev=20)
    a = lib_state(w)
    a.step(4, 6)
    b = lib_state(w)
    b.step(4, 6)
    c = lib_state(w)
    thor.thor_set_timing(c.handle, 1)     # eager launches with events
    c.step(4, 6)
    ms, cnt = thor.thor_kernel_time(c.handle, "vert")
    assert cnt == 4 * 10 and ms > 0
    thor.thor_set_timing(c.handle, 0)
    ea, eb, ec = a.export()[0], b.export()[0], c.export()[0]
    assert np.array_equal(ea, eb) and np.array_equal(ea, ec)


def test_non_finite_state_is_reported():
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=2, n_lev=8)
    st = lib_state(w)
    blob = st.export()[0]
    blob[4 + 123] = np.nan           # one density value
    st.load(blob)
    m, rc = st.mass()
    assert rc == thor.THOR_ENONFINITE
    assert "non-finite" in thor.lib().thor_last_error().decode()


def test_gas_giant_g6_l32_invariants():
    """The benchmark workload at full size: mass conserved to round-off,
    finite fields, bounded winds after 10 large steps."""
    w = workloads.gas_giant_c2()
    say(f"[c2] g{w.glevel} L{w.n_lev}")
    st = lib_state(w)
    m0, rc = st.mass()
    st.step(10, w.n_acoustic)
    m1, rc = st.mass()
    assert rc == 0
    assert abs(m1 / m0 - 1) < 1e-13
    sc, rc = st.scalars()
    assert rc == 0 and 0 < sc["max_speed"] < 50.0
    assert 700 < sc["min_T"] and sc["max_T"] < 1700


def test_maximum_size_rest_state():
    """The largest supported configuration, g8 (655362 columns) x 64 levels
    (41.9 M cells, ~14 GB of FP64 state), autotuned and graph-replayed: a
    resting isothermal atmosphere in discrete hydrostatic balance stays at
    rest and keeps its mass."""
    import torch
    from paper_1607_05535_amd import thor
    w = small_earth(glevel=8, n_lev=64, n_large=1, noise=0.0)
    w.dt = 100.0
    say(f"[max size] g8 L64: {w.cells} cells")
    st = lib_state(w)
    m0, rc = st.mass()
    assert rc == 0
    thor.thor_autotune(st.handle, w.n_acoustic)
    st.step(w.n_large, w.n_acoustic)
    sc, rc = st.scalars()
    assert rc == 0
    m1, _ = st.mass()
    say(f"          max speed {sc['max_speed']:.3e} m/s, max |w| {sc['max_w']:.3e}, mass drift {m1 / m0 - 1:.2e}")
    assert sc["max_speed"] < 1e-8 and sc["max_w"] < 1e-8
    assert abs(m1 / m0 - 1) < 1e-13
    del st
    torch.cuda.empty_cache()
