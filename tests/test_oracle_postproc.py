"""Pins of the post-processing oracle (pressure levels, zonal and time
means, eddy fluxes, mass streamfunction)."""
import numpy as np

import workloads
from oracle import dynamics as dy
from oracle import postproc as pp
from tests.conftest import oracle_grid


def test_interpolation_is_exact_for_fields_linear_in_pressure():
    rs = np.random.default_rng(0)
    N, L = 20, 9
    p = np.sort(rs.uniform(1e3, 1e5, size=(N, L)), axis=1)[:, ::-1]   # decreasing upward
    q = 3.0 - 2e-5 * p
    plev = np.array([5e2, 2e3, 1e4, 5e4, 9e4, 2e5])
    out, valid = pp.interpolate(p, q, plev)
    inside = (plev[None, :] >= p[:, -1:]) & (plev[None, :] <= p[:, :1])
    assert np.array_equal(valid, inside)
    assert np.abs(out[valid] - (3.0 - 2e-5 * np.broadcast_to(plev, out.shape)[valid])).max() < 1e-12
    assert not valid[:, 0].any() and not valid[:, -1].any()


def _state_with_winds(w, U, V):
    """The isothermal rest state of workload w with u = U cos(lon),
    v = V cos(lon) at every level."""
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    lam, phi = dy.lon_lat(model.rhat)
    east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], axis=-1)
    north = np.stack([-np.sin(phi) * np.cos(lam), -np.sin(phi) * np.sin(lam), np.cos(phi)], axis=-1)
    vel = (U * np.cos(lam))[:, None] * east + (V * np.cos(lam))[:, None] * north
    M = st.rho[..., None] * vel[:, None, :]
    return model, dy.State(st.rho, M, st.rth, st.W), lam, phi


def test_zonal_means_and_eddy_flux_of_a_wavenumber_one_wind():
    """u = U cos(lon), v = V cos(lon): band means U<cos>, V<cos> and eddy flux
    U V (<cos^2> - <cos>^2) with <.> the area-weighted band mean, computed here
    from the grid alone; an isothermal state has T = T0 and no heat flux."""
    w = workloads.small_gas_giant(glevel=3, n_lev=12)
    w.noise_amp = 0.0
    U, V = 7.0, -3.0
    model, st, lam, phi = _state_with_winds(w, U, V)
    f = dy.fields(model, st)
    plev = np.linspace(f["p"][0, -1] * 1.01, f["p"][0, 0] * 0.99, 6)
    nb = 8
    out, present = pp.snapshot(model, st, plev, nb)
    assert present.all()
    A = model.G.Ac
    band = pp.band_of(phi, nb)
    for b in range(nb):
        wgt = A[band == b] / A[band == b].sum()
        c = np.cos(lam[band == b])
        mc, mc2 = np.sum(wgt * c), np.sum(wgt * c * c)
        assert np.allclose(out["u"][b], U * mc, rtol=0, atol=1e-12)
        assert np.allclose(out["v"][b], V * mc, rtol=0, atol=1e-12)
        assert np.allclose(out["upvp"][b], U * V * (mc2 - mc * mc), rtol=1e-12, atol=1e-12)
    assert np.abs(out["T"] - w.T0).max() < 1e-9
    assert np.abs(out["vpTp"]).max() < 1e-9
    assert np.all(out["weight"] == 1.0)


def test_streamfunction_of_a_constant_meridional_wind():
    """[v] = c at every level: Psi = 2 pi A cos(lat) c p / g exactly."""
    nb, plev = 6, np.array([1e3, 5e3, 2e4, 8e4])
    vbar = np.full((nb, len(plev)), 2.5)
    psi = pp.streamfunction(vbar, plev, 1e8, 8.0)
    lat = pp.band_latitudes(nb)
    ref = 2 * np.pi * 1e8 * np.cos(lat)[:, None] * 2.5 * plev[None, :] / 8.0
    assert np.abs(psi / ref - 1).max() < 1e-14


def test_time_mean_counts_only_present_snapshots():
    a = {k: np.array([[1.0, 2.0]]) for k in pp.QUANTITIES}
    b = {k: np.array([[3.0, 9.0]]) for k in pp.QUANTITIES}
    mean, cnt = pp.time_mean([(a, np.array([[True, True]])), (b, np.array([[True, False]]))])
    assert np.array_equal(cnt, [[2, 1]])
    assert np.allclose(mean["u"], [[2.0, 2.0]])


def test_bands_cover_the_sphere_once():
    lat = np.array([-np.pi / 2, -0.1, 0.0, 0.3, np.pi / 2])
    b = pp.band_of(lat, 4)
    assert list(b) == [0, 1, 2, 2, 3]


def _state_with_first_layer_w(w, target):
    """The rest state of workload w with first-layer vertical velocity
    `target` [n_col]: the momentum at the first interior interface set to
    2 rho target (the ground interface carries none)."""
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    W = np.zeros_like(st.W)
    W[:, 1] = 2.0 * st.rho[:, 0] * target
    return model, dy.State(st.rho, st.M, st.rth, W)


def test_first_layer_w_is_the_centre_value_of_the_diagnostic_field():
    w = workloads.small_gas_giant(glevel=2, n_lev=6)
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    rs = np.random.default_rng(3)
    W = rs.normal(size=st.W.shape)
    W[:, 0] = W[:, -1] = 0.0
    st = dy.State(st.rho, st.M, st.rth, W)
    assert np.abs(pp.first_layer_w(model, st) - dy.fields(model, st)["w"][:, 0]).max() < 1e-15


def test_imprint_of_a_zonally_varying_w():
    """w = a(band) + b cos(lon): w* = b (cos(lon) - <cos(lon)>_band), with the
    band mean weighted by the control-volume areas; the band constants
    vanish, w* averages to zero over every band, and a resting state has
    none."""
    w = workloads.small_gas_giant(glevel=3, n_lev=8)
    w.noise_amp = 0.0
    nb = 7
    G = oracle_grid(w.glevel)
    lam, lat = dy.lon_lat(G.P)
    band = pp.band_of(lat, nb)
    a = 0.05 * (band - 3.0) ** 2
    b = 0.02
    model, st = _state_with_first_layer_w(w, a + b * np.cos(lam))
    ws = pp.imprint_snapshot(model, st, nb)
    A = G.Ac
    for k in range(nb):
        m = band == k
        mc = np.sum(A[m] * np.cos(lam[m])) / A[m].sum()
        assert np.abs(ws[m] - b * (np.cos(lam[m]) - mc)).max() < 1e-14
        assert abs(np.sum(A[m] * ws[m])) < 1e-14 * A[m].sum()
    model, rest = dy.model_from_workload(w, G)
    assert np.all(pp.imprint_snapshot(model, rest, nb) == 0.0)


def test_imprint_map_is_the_time_mean():
    m1, m2 = np.array([1.0, -2.0, 0.5]), np.array([3.0, 0.0, -0.5])
    assert np.array_equal(pp.imprint_map([m1, m2]), [2.0, -1.0, 0.0])
