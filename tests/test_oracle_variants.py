"""Pins of the oracle's switchable approximations (Sec. 3 lists them: the
model implements them although the paper's runs leave them off)."""
import numpy as np

from oracle import dynamics as dy
from tests.conftest import oracle_grid
from tests.gpu_util import small_earth


def _model(w):
    return dy.model_from_workload(w, oracle_grid(w.glevel))


def _one_substep(model, st, dtau):
    """Large-step terms, first-stage slow forcing and one substep of dtau."""
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    return large, f, dy.acoustic_substep(model, st, f, dtau, large)


def _imbalance(model, st, large):
    """I + deviation pressure gradient + buoyancy at the interior interfaces:
    the vertical-momentum tendency without its slow terms."""
    g, dz = model.planet.gravity, model.dz
    ps = model.eos(st.rth) - large["p_t"]
    rs = st.rho - large["rho_t"]
    return (large["I"][:, 1:-1] - (ps[:, 1:] - ps[:, :-1]) / dz
            - 0.5 * g * (rs[:, :-1] + rs[:, 1:]))


def test_hydrostatic_substep_balances_the_column():
    """T noise at fixed p leaves the initial columns out of hydrostatic
    balance (buoyancy).  One short hydrostatic substep (2 s, a vertical
    acoustic Courant number of about 0.4) removes the imbalance up to the
    linearisation of the equation of state, second order in the 0.1 K
    noise; a non-hydrostatic one only starts to accelerate W."""
    res = {}
    for hyd in (False, True):
        w = small_earth(glevel=2, n_lev=12, noise=0.1)
        w.hydrostatic = hyd
        model, st = _model(w)
        large, f, out = _one_substep(model, st, 2.0)
        # the imbalance measured against the state's own [t] terms
        r0 = np.abs(_imbalance(model, st, large)).max()
        r1 = np.abs(_imbalance(model, out, large)).max()
        res[hyd] = r1 / r0
    assert res[True] < 1e-3
    assert res[False] > 0.5


def test_hydrostatic_substep_forgets_the_vertical_momentum():
    """Without vertical acceleration the new W does not depend on the old W
    nor on the slow forcing of W (divergence damping off: its 3D divergence
    reads W)."""
    w = small_earth(glevel=2, n_lev=10, noise=1.0)
    w.hydrostatic = True
    w.div_damp = False
    model, st = _model(w)
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    a = dy.acoustic_substep(model, st, f, 100.0, large)
    rs = np.random.default_rng(5)
    W2 = st.W.copy()
    W2[:, 1:-1] += rs.normal(size=W2[:, 1:-1].shape)
    f2 = dict(f)
    f2["S_W"] = f["S_W"] + rs.normal(size=f["S_W"].shape)
    b = dy.acoustic_substep(model, dy.State(st.rho, st.M, st.rth, W2), f2, 100.0, large)
    for x, y in ((a.W, b.W), (a.rho, b.rho), (a.rth, b.rth), (a.M, b.M)):
        assert np.array_equal(x, y)


def test_hydrostatic_rest_state_stays_at_rest():
    w = small_earth(glevel=2, n_lev=12, n_large=3, noise=0.0)
    w.hydrostatic = True
    model, st = _model(w)
    out = dy.run(model, st, w.n_large, w.n_acoustic)
    f = dy.fields(model, out)
    for k in ("u", "v", "w"):
        assert np.abs(f[k]).max() < 1e-8, k


def test_hydrostatic_and_nonhydrostatic_agree_at_hydrostatic_scales():
    """Cells ~1000 km wide and 1.8 km deep: the horizontal winds of the two
    forms differ little after three steps, while the vertical velocity (a
    diagnosed balance in one, a prognostic in the other) may differ more."""
    out = {}
    for hyd in (False, True):
        w = small_earth(glevel=3, n_lev=20, n_large=3, noise=1.0)
        w.hydrostatic = hyd
        model, st = _model(w)
        out[hyd] = dy.fields(model, dy.run(model, st, w.n_large, w.n_acoustic))
    speed = np.sqrt(out[False]["u"] ** 2 + out[False]["v"] ** 2).max()
    du = max(np.abs(out[True][k] - out[False][k]).max() for k in ("u", "v"))
    dT = np.abs(out[True]["T"] - out[False]["T"]).max()
    assert 1e-6 * speed < du < 0.01 * speed      # a real change, and a small one
    assert dT < 0.005


def _zonal_flow_state(model, st, U):
    """The state's density and rho theta with u = U cos(lat) at every level,
    no vertical motion."""
    lam, phi = dy.lon_lat(model.rhat)
    east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], axis=-1)
    u = U * np.cos(phi)
    M = st.rho[..., None] * (u[:, None, None] * east[:, None, :])
    return dy.State(st.rho, M, st.rth, np.zeros_like(st.W)), u, phi


def test_vertical_momentum_forcing_of_a_zonal_flow():
    """u = U cos(lat), w = 0.  Deep form: the radial equation receives the
    curvature and Coriolis accelerations rho (u^2 / r + 2 Omega u cos(lat))
    (up to the discretisation); shallow form with the traditional
    approximation: neither, so S_W is the [t] imbalance plus hyperdiffusion
    alone."""
    U = 60.0
    for shallow in (False, True):
        w = small_earth(glevel=4, n_lev=6, noise=0.0)
        w.shallow = shallow
        model, st = _model(w)
        st, u, phi = _zonal_flow_state(model, st, U)
        large = dy.large_step_terms(model, st)
        f = dy.slow_forcing(model, st, large)
        extra = f["S_W"][:, 1:-1] - (large["I"][:, 1:-1] + large["H_W"][:, 1:-1])
        if shallow:
            assert np.abs(extra).max() <= 1e-12 * np.abs(large["I"][:, 1:-1]).max()
        else:
            Om, rI = model.planet.omega, model.rI[1:-1]
            rhoI = 0.5 * (st.rho[:, :-1] + st.rho[:, 1:])
            acc = (u * u)[:, None] / rI[None, :] + (2 * Om * u * np.cos(phi))[:, None]
            ref = rhoI * acc
            err = np.abs(extra - ref).max() / np.abs(ref).max()
            assert err < 2e-3, err


def test_shallow_rest_state_stays_at_rest():
    w = small_earth(glevel=2, n_lev=12, n_large=3, noise=0.0)
    w.shallow = True
    model, st = _model(w)
    f = dy.fields(model, dy.run(model, st, w.n_large, w.n_acoustic))
    for k in ("u", "v", "w"):
        assert np.abs(f[k]).max() < 1e-8, k


def test_shallow_and_deep_agree_for_a_thin_atmosphere():
    """A 36 km atmosphere on a 6371 km planet: the two forms differ at the
    order of H / A in their geometry and by the dropped small terms."""
    out = {}
    for shallow in (False, True):
        w = small_earth(glevel=3, n_lev=20, n_large=3, noise=1.0)
        w.shallow = shallow
        model, st = _model(w)
        st, _, _ = _zonal_flow_state(model, st, 30.0)
        out[shallow] = dy.fields(model, dy.run(model, st, w.n_large, w.n_acoustic))
    speed = np.sqrt(out[False]["u"] ** 2 + out[False]["v"] ** 2).max()
    du = max(np.abs(out[True][k] - out[False][k]).max() for k in ("u", "v"))
    assert 1e-6 * speed < du < 0.01 * speed


# ---------------------------------------------------------------------------
# Vertical Lagrange interpolation of order k (Sec. 2.1)
# ---------------------------------------------------------------------------
def test_lagrange_weights_reproduce_polynomials_up_to_their_degree():
    rs = np.random.default_rng(2)
    for k in (1, 2, 3, 5):
        nodes = np.sort(rs.uniform(-3, 3, k + 1))
        t = rs.uniform(-2, 2)
        w = dy.lagrange_weights(nodes, t)
        for deg in range(k + 1):
            assert abs(np.dot(w, nodes ** deg) - t ** deg) < 1e-9 * max(1, abs(t) ** deg)
        # one degree more is not reproduced in general
        assert abs(np.dot(w, nodes ** (k + 1)) - t ** (k + 1)) > 1e-9


def test_order_one_matrices_are_the_two_point_means():
    L = 7
    rs = np.random.default_rng(3)
    x = rs.normal(size=(5, L))
    W = rs.normal(size=(5, L + 1))
    assert np.allclose(x @ dy.centre_to_interface_matrix(L, 1).T, dy.to_interfaces(x), rtol=0, atol=1e-15)
    assert np.allclose(W @ dy.interface_to_centre_matrix(L, 1).T, dy.to_centres(W), rtol=0, atol=1e-15)


def test_cubic_interpolation_is_exact_for_cubics_in_height():
    """Order 3: interior rows are (-1, 9, 9, -1) / 16 (midpoint of four
    equally spaced nodes); every row, the shifted ones at the ground and the
    lid included, reproduces a cubic in z exactly."""
    L = 9
    Aci = dy.centre_to_interface_matrix(L, 3)
    Aic = dy.interface_to_centre_matrix(L, 3)
    mid = np.array([-1.0, 9.0, 9.0, -1.0]) / 16
    assert np.allclose(Aci[3, 2:6], mid, rtol=0, atol=1e-15)      # interface 4 from centres 2..5
    assert np.allclose(Aic[4, 3:7], mid, rtol=0, atol=1e-15)      # centre 4 from interfaces 3..6
    assert np.allclose(Aci.sum(axis=1), 1) and np.allclose(Aic.sum(axis=1), 1)
    f = lambda z: 2.0 - 0.3 * z + 0.05 * z ** 2 - 0.01 * z ** 3
    zc, zi = np.arange(L) + 0.5, np.arange(L + 1.0)
    assert np.abs(Aci @ f(zc) - f(zi[1:L])).max() < 1e-12
    assert np.abs(Aic @ f(zi) - f(zc)).max() < 1e-12
    assert np.abs(dy.centre_to_interface_matrix(L, 1) @ f(zc) - f(zi[1:L])).max() > 1e-3


def test_order_three_rest_state_and_closeness_to_order_one():
    w = small_earth(glevel=2, n_lev=12, n_large=3, noise=0.0)
    w.lagrange_order = 3
    model, st = _model(w)
    f = dy.fields(model, dy.run(model, st, w.n_large, w.n_acoustic))
    for k in ("u", "v", "w"):
        assert np.abs(f[k]).max() < 1e-8, k
    out = {}
    for order in (1, 3):
        w = small_earth(glevel=3, n_lev=20, n_large=3, noise=1.0)
        w.lagrange_order = order
        model, st = _model(w)
        st, _, _ = _zonal_flow_state(model, st, 30.0)
        out[order] = dy.fields(model, dy.run(model, st, w.n_large, w.n_acoustic))
    speed = np.sqrt(out[1]["u"] ** 2 + out[1]["v"] ** 2).max()
    du = max(np.abs(out[3][k] - out[1][k]).max() for k in ("u", "v", "w"))
    assert 1e-9 * speed < du < 0.01 * speed


def test_order_three_needs_four_levels():
    import pytest
    w = small_earth(glevel=2, n_lev=3)
    w.lagrange_order = 3
    with pytest.raises(ValueError):
        _model(w)


def test_order_one_allows_a_single_level():
    w = small_earth(glevel=2, n_lev=1)
    _model(w)
