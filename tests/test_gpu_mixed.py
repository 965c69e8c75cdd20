"""Mixed-precision form (FP32 horizontal stencils and advection; FP64
vertical solve, reference state, density, rho theta, W and mass sums)
against the FP64 path on the same GPU.  The per-field error is a reported
property of the form, bounded here so that a broken FP32 path fails."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import lib_fields, lib_state, cell_errors, say, small_earth

pytestmark = pytest.mark.gpu


def _pair(w, n_large):
    a = lib_state(w, 0)
    b = lib_state(w, 1)
    a.step(n_large, w.n_acoustic)
    b.step(n_large, w.n_acoustic)
    return a, b


@pytest.mark.parametrize("maker", [lambda: small_earth(glevel=4, n_lev=20, n_large=10),
                                   lambda: workloads.small_gas_giant(glevel=4, n_lev=32, n_large=10)])
def test_mixed_tracks_fp64(maker):
    w = maker()
    say(f"[mixed] {w.name} g{w.glevel} L{w.n_lev}")
    a, b = _pair(w, w.n_large)
    fa, fb = lib_fields(a), lib_fields(b)
    err = cell_errors(fb, fa)
    say(f"        errors {err}")
    # bars about 30 and 50 times the largest errors measured (thermodynamic
    # 3.7e-9, winds 1.9e-6 of the RMS speed after 10 steps)
    for k in ("T", "p", "rho", "rhotheta"):
        assert err[k] < 1e-7, (k, err[k])
    for k in ("u", "v", "w"):
        assert err[k] < 1e-4, (k, err[k])
    ma, _ = a.mass()
    mb, rc = b.mass()
    assert rc == 0
    # the FP32 flux divergences cancel between cells only to FP32 rounding of
    # small density increments: mass is kept to ~1e-13, bounded at 1e-12
    m0 = lib_state(w, 1).mass()[0]
    assert abs(mb / m0 - 1) < 1e-12


def test_mixed_rest_state():
    w = small_earth(glevel=3, n_lev=20, n_large=5, noise=0.0)
    st = lib_state(w, 1)
    st.step(w.n_large, w.n_acoustic)
    for k, v in lib_fields(st, ("u", "v", "w")).items():
        assert np.abs(v).max() < 1e-4, k


def test_mixed_four_levels_per_lane_matches_one_level():
    """The mixed form's phase V on the four-levels mapping (FP32 horizontal
    fields in 16-byte float4 rows) agrees with the one-level mapping to the
    form's rounding."""
    from paper_1607_05535_amd import thor
    w = workloads.small_gas_giant(glevel=3, n_lev=32, n_large=3)
    a = lib_state(w, 1)
    b = lib_state(w, 1)
    thor.thor_set_vert_levels_per_lane(a.handle, 1)
    thor.thor_set_vert_levels_per_lane(b.handle, 4)
    a.step(w.n_large, w.n_acoustic)
    b.step(w.n_large, w.n_acoustic)
    err = cell_errors(lib_fields(b), lib_fields(a))
    say(f"[mixed] four vs one level per lane {err}")
    # measured: thermodynamic 4.4e-9, winds 4.0e-7
    for k in ("T", "p", "rho", "rhotheta"):
        assert err[k] < 1e-7, (k, err[k])
    for k in ("u", "v", "w"):
        assert err[k] < 1e-5, (k, err[k])
