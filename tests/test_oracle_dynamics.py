"""Pins of the oracle time step (Sec. 3-5) against closed forms, invariants
and textbook routines."""
import os

import numpy as np
import pytest

import workloads
from oracle import dynamics as dy
from oracle import grid
from oracle import operators as op
from oracle import rng
from tests.conftest import oracle_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def earth_model(g=3, L=20, noise=0.1, diff_D=workloads.D_EARTH, seed=1, p_ref=1.0e5,
                div_damp=True, omega=7.292e-5):
    G = oracle_grid(g)
    planet = dy.Planet(6.371e6, omega, 9.8, 287.0, 1005.0, p_ref)
    model = dy.Model(G, planet, dy.Vertical(L, 36.0e3), dy.Numerics(600.0, diff_D, div_damp))
    st = dy.init_state(model, dy.Init(300.0, 1.0e5, noise, seed))
    return model, st


def test_splitmix64_reference_sequence():
    """First outputs of SplitMix64 started from state 0 (published sequence)."""
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    state = 0
    for v in vals:
        assert int(rng.mix64(state)) == v
        state = (state + 0x9E3779B97F4A7C15) % 2 ** 64


def test_noise_bounds_and_seed_dependence():
    e = rng.column_noise(5, 2562, 20, 0.1)
    assert e.shape == (2562, 20)
    assert np.abs(e).max() < 0.1 and abs(e.mean()) < 2e-3
    assert abs(e.std() - 0.1 / np.sqrt(3)) < 2e-3
    assert not np.array_equal(e, rng.column_noise(6, 2562, 20, 0.1))
    assert not np.array_equal(e, rng.column_noise(5, 2562, 20, 0.1, planet=1))


@pytest.mark.parametrize("lam", [-0.7, 0.3, 1.5j, -0.2 + 0.9j])
def test_split_explicit_reduces_to_ws_rk3(lam):
    """With only slow terms, one large step multiplies by 1 + z + z^2/2 + z^3/6."""
    dt = 0.8
    for n in (2, 6, 8):
        out = dy.split_explicit(1.0 + 0j, lambda phi: lam * phi,
                                lambda phi, f, dtau: phi + dtau * f, dt, n)
        z = lam * dt
        assert abs(out - (1 + z + z ** 2 / 2 + z ** 3 / 6)) < 1e-14


def test_substep_schedule():
    """Stage 1: one substep of dt/3; stage 2: n/2 of dt/n; stage 3: n of dt/n."""
    for n in (2, 4, 6, 8, 12):
        sched = dy.stage_schedule(600.0, n)
        assert sum(ns for ns, _ in sched) == 1 + 3 * n // 2
        assert np.allclose([ns * d for ns, d in sched], [200.0, 300.0, 600.0])
    for bad in (0, 1, 3, 7):
        with pytest.raises(ValueError):
            dy.stage_schedule(600.0, bad)


@pytest.mark.parametrize("m", range(1, 9))
def test_thomas_matches_dense_lu(m):
    rs = np.random.default_rng(m)
    n = 50
    a, c = rs.normal(size=(n, m)), rs.normal(size=(n, m))
    b = np.abs(a) + np.abs(c) + rs.uniform(0.5, 2.0, size=(n, m))
    d = rs.normal(size=(n, m))
    x = dy.thomas(a, b, c, d)
    for i in range(n):
        A = np.diag(b[i]) + np.diag(a[i, 1:], -1) + np.diag(c[i, :-1], 1)
        ref = np.linalg.solve(A, d[i])
        assert np.allclose(x[i], ref, rtol=1e-13, atol=1e-13)


def test_initial_state_is_in_discrete_hydrostatic_balance():
    model, st = earth_model(noise=0.0)
    large = dy.large_step_terms(model, st)
    scale = model.planet.gravity * st.rho.max()
    assert np.abs(large["I"]).max() < 1e-12 * scale
    f = dy.fields(model, st)
    assert np.allclose(f["T"], 300.0, rtol=1e-13, atol=0)
    # surface pressure recovered by the continuous hydrostatic half-layer
    p0 = f["p"][0, 0] * np.exp(model.planet.gravity * model.dz / 2 / (287.0 * 300.0))
    assert abs(p0 - 1.0e5) < 1e-8


def test_rest_state_stays_at_rest():
    model, st = earth_model(noise=0.0)
    st0 = st.copy()
    st = dy.run(model, st, 10, 6)
    f = dy.fields(model, st)
    for k in ("u", "v", "w"):
        assert np.abs(f[k]).max() < 1e-8
    assert np.abs(st.rho / st0.rho - 1).max() < 1e-13
    assert np.abs(st.rth / st0.rth - 1).max() < 1e-13


def test_mass_and_rho_theta_are_conserved():
    """Flux form (Eqs. mass, entropy) with a rigid lid: total mass is
    conserved to round-off; without diffusion or forcing total rho theta is
    too."""
    model, st = earth_model(noise=0.1)
    m0 = dy.mass(model, st)
    st1 = dy.run(model, st, 10, 6)
    assert abs(dy.mass(model, st1) / m0 - 1) < 1e-13
    model, st = earth_model(noise=0.1, diff_D=0.0)
    vol = model.G.Ac[:, None] * model.rC[None, :] ** 2

    def total(x):
        return float(np.sum(x * vol))
    s0 = total(st.rth)
    st1 = dy.run(model, st, 5, 6)
    assert abs(total(st1.rth) / s0 - 1) < 1e-13
    assert abs(total(st1.rho) / total(st.rho) - 1) < 1e-13
    assert np.abs(dy.fields(model, st1)["u"]).max() > 1e-3   # the flow moved


def test_mass_conserved_with_newtonian_forcing():
    w = workloads.small_gas_giant(glevel=3, n_lev=12)
    model, st = dy.model_from_workload(w, oracle_grid(3))
    m0 = dy.mass(model, st)
    st1 = dy.run(model, st, 3, 8)
    assert abs(dy.mass(model, st1) / m0 - 1) < 1e-13
    f = dy.fields(model, st1)
    assert np.all(np.isfinite(f["T"])) and np.abs(f["u"]).max() > 1e-3


def test_results_do_not_depend_on_reference_pressure():
    """Eq. pressure: p_ref is arbitrary; the discrete dynamics is invariant."""
    outs = []
    for p_ref in (1.0e5, 2.2e7):
        model, st = earth_model(noise=0.1, p_ref=p_ref)
        st = dy.run(model, st, 2, 6)
        outs.append(dy.fields(model, st))
    for k in ("T", "p", "rho"):
        assert np.abs(outs[0][k] / outs[1][k] - 1).max() < 1e-12
    for k in ("u", "v", "w"):
        scale = np.abs(outs[0][k]).max()
        assert np.abs(outs[0][k] - outs[1][k]).max() < 1e-9 * scale


def test_hevi_solution_satisfies_discrete_vertical_momentum_equation():
    """After a substep the new W, with rho from Eq. dens2 and p from the
    nonlinear EOS of the new rho theta, satisfies the discrete Eq. momr2 up to
    the linearisation error of the pressure (second order in the step)."""
    model, st = earth_model(noise=0.1)
    st = dy.run(model, st, 1, 6)       # develop some vertical motion
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    dtau = 100.0
    out = dy.acoustic_substep(model, st, f, dtau, large)
    g, dz = model.planet.gravity, model.dz
    ps = model.eos(out.rth) - large["p_t"]
    rs = out.rho - large["rho_t"]
    pgf = -(ps[:, 1:] - ps[:, :-1]) / dz - 0.5 * g * (rs[:, :-1] + rs[:, 1:])
    resid = out.W[:, 1:-1] - st.W[:, 1:-1] - dtau * (f["S_W"][:, 1:-1] + pgf)
    scale = np.abs(dtau * pgf).max()
    assert scale > 0 and np.abs(out.W).max() > 0
    assert np.abs(resid).max() < 1e-4 * scale
    # the explicit step alone (old W in the updates) would not satisfy it
    assert np.abs(out.W - st.W).max() > 1e-2 * np.abs(resid).max()


def test_warm_anomaly_rises():
    """Buoyancy sign (Eq. momr2): a cell made lighter at fixed pressure is
    accelerated upward through both of its interfaces in the first substep."""
    model, st = earth_model(noise=0.0)
    i, k = 100, 8
    p = model.eos(st.rth)
    T = p / (st.rho * model.planet.Rd)
    T[i, k] += 1.0
    st.rho[i, k] = p[i, k] / (model.planet.Rd * T[i, k])   # warmer at fixed p
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    out = dy.acoustic_substep(model, st, f, 20.0, large)
    assert out.W[i, k + 1] > 0 and out.W[i, k] > 0
    others = np.delete(np.abs(out.W[i]), [k, k + 1])
    assert min(out.W[i, k], out.W[i, k + 1]) > others.max()


def test_high_pressure_anomaly_diverges():
    """Pressure-gradient sign (Eq. mom2): flow leaves a high-pressure cell."""
    model, st = earth_model(noise=0.0)
    i, k = 200, 3
    p = model.eos(st.rth)
    p[i, k] *= 1.001
    st.rth[i, k] = model.rth_from_p(p[i, k])
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    out = dy.acoustic_substep(model, st, f, 50.0, large)
    D = op.div(model.G, out.M, model.rC)
    assert D[i, k] > 0
    for j in model.G.nbr[i, :model.G.deg[i]]:
        assert np.dot(out.M[j, k], model.G.P[j] - model.G.P[i]) > 0


def test_solid_body_rotation_slow_forcing():
    """Advection and Coriolis of a rigid rotation v = w zhat x r at uniform
    density: A + C = -rho (w^2 + 2 Omega w) s shat (s distance to the axis);
    S_M is its negative horizontal projection, S_W gets the radial part."""
    G = oracle_grid(5)
    Om, wr = 7.292e-5, 2.0e-5
    planet = dy.Planet(6.371e6, Om, 9.8, 287.0, 1005.0)
    model = dy.Model(G, planet, dy.Vertical(4, 8.0e3), dy.Numerics(600.0, 0.0, False))
    L = 4
    rho = np.full((G.n, L), 1.2)
    zhat = np.array([0.0, 0.0, 1.0])
    rpos = model.rC[None, :, None] * G.P[:, None, :]
    v = wr * np.cross(zhat, rpos)
    M = rho[..., None] * v
    st = dy.State(rho, M, np.full((G.n, L), 300.0), np.zeros((G.n, L + 1)))
    large = dict(G_t=np.zeros_like(M), H_M=np.zeros_like(M),
                 H_W=np.zeros((G.n, L + 1)), I=np.zeros((G.n, L + 1)),
                 H_rho=0.0, H_rth=0.0)
    f = dy.slow_forcing(model, st, large)
    s_vec = rpos.copy()
    s_vec[..., 2] = 0.0
    AC = -rho[..., None] * (wr ** 2 + 2 * Om * wr) * s_vec
    ref_M = op.proj_h(-AC, G.P)
    err = np.linalg.norm(f["S_M"] - ref_M, axis=-1).max()
    assert err < 1e-2 * np.linalg.norm(ref_M, axis=-1).max()
    ACr = op.proj_r(AC, G.P)
    ref_W = -0.5 * (ACr[:, :-1] + ACr[:, 1:])
    assert np.abs(f["S_W"][:, 1:L] - ref_W).max() < 1e-2 * np.abs(ref_W).max()


def test_hyperdiffusion_damps_a_harmonic():
    """Eq. diff_rho: F = -Kd lap lap rho = -Kd (l(l+1))^2 / r^4 rho' for a
    degree-l harmonic.  The composite Laplacian is only first order pointwise
    (O(1) local error at the pentagons), so the check is on the projection of
    F onto the harmonic, which converges at second order; Eq. diff_p must
    damp temperature anomalies."""
    dev = {}
    for g in (4, 5):
        G = oracle_grid(g)
        model, _ = earth_model(g=g, L=3, noise=0.0)
        Y = 3 * G.P[:, 2] ** 2 - 1                      # l = 2
        rho = 1.0 + 1e-3 * Y[:, None] * np.ones((1, 3))
        st = dy.State(rho, np.zeros((G.n, 3, 3)), model.rth_from_p(rho * 287.0 * 300.0),
                      np.zeros((G.n, 4)))
        p = model.eos(st.rth)
        H_rho, H_M, H_W, H_rth = dy.hyperdiffusion(model, st, p)
        ref = -model.Kd * 36.0 / model.rC[None, :] ** 4 * 1e-3 * Y[:, None]
        w = G.Ac[:, None]
        dev[g] = abs(np.sum(w * H_rho * Y[:, None]) / np.sum(w * ref * Y[:, None]) - 1)
        # temperature anomaly at fixed pressure is damped: H_rth anti-correlates with T'
        T = p / (rho * 287.0)
        assert np.sum(w * H_rth * (T - np.mean(T))) < 0
        assert np.abs(H_M).max() == 0 and np.abs(H_W).max() == 0
    assert dev[5] < 3e-3 and dev[5] < 0.5 * dev[4]


def test_divergence_damping_is_dissipative():
    model, st = earth_model(g=4, L=3, noise=0.0)
    G = model.G
    Y = G.P[:, 0] * G.P[:, 1]
    st.M = 0.5 * op.proj_h(op.grad(G, np.repeat(Y[:, None], 3, 1), model.rC), G.P) * model.rC[None, :, None]
    D = dy.momentum_divergence(model, st.M, st.W)
    GD = op.grad(G, D, model.rC)
    DD = np.stack([-model.Kd * op.lap(G, GD[..., q], model.rC) for q in range(3)], -1)
    rate = np.sum(G.Ac[:, None] * np.sum(DD * st.M, -1))
    assert rate < 0


def test_newtonian_relaxation_is_backward_euler():
    """Eq. im_eq_t: (T_new - T) / dt = K_T (T_eq - T_new), at fixed density."""
    w = workloads.small_gas_giant(glevel=2, n_lev=12)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    T0 = dy.fields(model, st)["T"]
    out = dy.newtonian(model, st)
    T1 = dy.fields(model, out)["T"]
    lhs = (T1 - T0) / model.num.dt
    rhs = (model.Teq - T1) / model.forcing.tau
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()
    assert np.array_equal(out.rho, st.rho)


def test_kd_matches_table1_damping_times():
    """Eqs. kd and tau_d with Table 1: tau_d = dbar^4 / (32 Kd)."""
    for D, tau, dt, A in ((workloads.D_EARTH, 6460.0, 1000.0, 6.371e6),
                          (workloads.D_HOT_JUPITER, 941.2, 600.0, 1.0e8)):
        G = oracle_grid(2)
        model = dy.Model(G, dy.Planet(A, 0.0, 9.8, 287.0, 1005.0), dy.Vertical(2, 1e4),
                         dy.Numerics(dt, D))
        dbar2 = grid.mean_spacing(2, A)
        assert abs(dbar2 ** 4 / (32 * model.Kd) / tau - 1) < 1e-12


# ---------------------------------------------------------------------------
# Hot-Jupiter benchmark forcing (Sec. 7.2, Eqs. teq-hj, btrop, tvert)
# ---------------------------------------------------------------------------

def test_hot_jupiter_vertical_profile_closed_forms():
    """Eq. tvert with the printed constants: continuous at z_stra, constant
    T_surf - Gamma z_stra + Delta T_stra above it (1210 K), and at the
    ground T_surf - Gamma z_stra / 2 + sqrt((Gamma z_stra / 2)^2 + Delta T^2)."""
    f = dy.Forcing(kind=2, tau=1.5e5, T_mean=1600.0, dT_daynight=300.0)
    zs = f.z_strat
    assert abs(dy.t_vert(f, np.array([zs]))[0] - 1210.0) < 1e-9
    assert np.all(dy.t_vert(f, np.array([zs + 1.0, 3e6, 4.875e6])) == 1210.0)
    assert abs(dy.t_vert(f, np.array([zs * (1 - 1e-12)]))[0] - 1210.0) < 1e-6
    assert abs(dy.t_vert(f, np.array([0.0]))[0] - (1400.0 + np.sqrt(200.0 ** 2 + 100.0))) < 1e-9
    # monotone cooling through the troposphere
    z = np.linspace(0.0, zs, 200)
    assert np.all(np.diff(dy.t_vert(f, z)) < 0)


def test_surface_pressure_of_the_hydrostatic_initial_state():
    """Sec. 5 extrapolation at constant temperature recovers the surface
    pressure the discrete hydrostatic isothermal state was built from."""
    w = workloads.hot_jupiter(glevel=2, n_lev=37)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    f = dy.fields(model, st)
    ps = dy.surface_pressure(model, f["p"], f["T"])
    assert np.abs(ps / w.p_surf - 1).max() < 1e-13


def test_hot_jupiter_teq_special_cases():
    """Eq. btrop: beta = sin(pi (sigma - sigma_stra) / (2 (1 - sigma_stra)))
    in the lowest cell (sigma from the extrapolated surface pressure), 0 at
    sigma = sigma_stra and above z_stra; Eq. teq-hj then gives T_vert +
    beta Delta T_E-P cos(lon) cos(lat), T_vert, and the stratosphere's T_vert."""
    w = workloads.hot_jupiter(glevel=2, n_lev=37)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    fc = model.forcing
    N, L = model.G.n, w.n_lev
    T = np.full((N, L), 1500.0)
    ps = 2.0e7
    z = model.zC
    # pressures chosen so that sigma = 1 in level 0 and sigma = sigma_stra in level 1
    p = np.empty((N, L))
    p0 = ps * np.exp(-w.gravity * z[0] / (w.Rd * 1500.0))
    p[:, 0] = p0
    p[:, 1] = fc.sigma_strat * ps
    p[:, 2:] = 1.0e5
    Teq = dy.hot_jupiter_teq(model, p, T)
    lam, phi = dy.lon_lat(model.rhat)
    h = np.cos(lam) * np.cos(phi)
    tv = dy.t_vert(fc, z)
    sig0 = p0 / ps
    beta0 = np.sin(np.pi * (sig0 - fc.sigma_strat) / (2 * (1 - fc.sigma_strat)))
    assert np.abs(Teq[:, 0] - (tv[0] + beta0 * 300.0 * h)).max() < 1e-9
    assert 0.0 < beta0 <= 1.0   # sigma < 1 at the lowest cell centre
    assert np.abs(Teq[:, 1] - tv[1]).max() < 1e-9
    above = z > fc.z_strat
    assert above.any() and np.all(Teq[:, above] == 1210.0)


def test_hot_jupiter_relaxation_is_backward_euler():
    """Eq. im_eq_t with the benchmark's T_eq of the dynamics output."""
    w = workloads.hot_jupiter(glevel=2, n_lev=37, noise_amp=0.5)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    f0 = dy.fields(model, st)
    Teq = dy.hot_jupiter_teq(model, f0["p"], f0["T"])
    out = dy.newtonian(model, st)
    T1 = dy.fields(model, out)["T"]
    lhs = (T1 - f0["T"]) / model.num.dt
    rhs = (Teq - T1) / model.forcing.tau
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()
    assert np.array_equal(out.rho, st.rho)


# ---------------------------------------------------------------------------
# Held-Suarez forcing (Sec. 7.1 Earth benchmark, Eqs. im_eq_v, im_eq_fv)
# ---------------------------------------------------------------------------

def _hs_pressures(w, model, sig, T=250.0):
    """Pressures whose sigma (with the extrapolated surface pressure) is sig
    per level, for levels 1..; level 0 sits at its hydrostatic sigma."""
    N, L = model.G.n, w.n_lev
    ps = 9.0e4
    p = np.empty((N, L))
    p[:, 0] = ps * np.exp(-w.gravity * model.zC[0] / (w.Rd * T))
    for k in range(1, L):
        p[:, k] = sig[k] * ps
    return p, np.full((N, L), T)


def test_held_suarez_rates_closed_forms():
    """K_v = 0 for sigma <= sigma_b and k_f (sigma - sigma_b) / (1 - sigma_b)
    above; K_T = k_a at sigma <= sigma_b; T_eq = max(200, 315 - 60 sin^2 lat) at
    p = p*; T_eq floors at 200 K at low pressure."""
    w = workloads.held_suarez(glevel=2, n_lev=6)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    f = model.forcing
    sig = np.array([0.0, 0.5, f.sigma_b, 0.85, f.p_star / 9.0e4, 1e-4])
    p, T = _hs_pressures(w, model, sig)
    Kv, KT, Teq = dy.held_suarez_rates(model, p, T)
    _, phi = dy.lon_lat(model.rhat)
    assert np.all(Kv[:, 1:3] == 0.0) and np.all(KT[:, 1:3] == f.k_a)
    assert np.allclose(Kv[:, 3], f.k_f * (0.85 - 0.7) / 0.3, rtol=1e-12)
    ramp = (0.85 - 0.7) / 0.3
    assert np.allclose(KT[:, 3], f.k_a + (f.k_s - f.k_a) * ramp * np.cos(phi) ** 4, rtol=1e-12)
    assert np.allclose(Teq[:, 4], np.maximum(200.0, 315.0 - 60.0 * np.sin(phi) ** 2), rtol=0, atol=1e-9)
    assert np.all(Teq[:, 5] == 200.0)


def test_held_suarez_physics_is_backward_euler():
    """Eqs. im_eq_v and im_eq_t: (M_new - M) / dt = -K_v M_new and
    (T_new - T) / dt = K_T (T_eq - T_new) with the rates of the dynamics
    output, at fixed density."""
    w = workloads.held_suarez(glevel=2, n_lev=12, noise_amp=0.5)
    model, st = dy.model_from_workload(w, oracle_grid(2))
    rs = np.random.default_rng(3)
    st = dy.State(st.rho, rs.normal(size=st.M.shape) * st.rho[..., None], st.rth, st.W)
    f0 = dy.fields(model, st)
    Kv, KT, Teq = dy.held_suarez_rates(model, f0["p"], f0["T"])
    assert Kv.max() > 0 and Kv.min() == 0.0
    out = dy.newtonian(model, st)
    dt = model.num.dt
    lhs = (out.M - st.M) / dt
    assert np.abs(lhs + Kv[..., None] * out.M).max() < 1e-12 * np.abs(lhs).max()
    T1 = dy.fields(model, out)["T"]
    assert np.abs((T1 - f0["T"]) / dt - KT * (Teq - T1)).max() < 1e-9 * np.abs(KT * (Teq - T1)).max()
    assert np.array_equal(out.rho, st.rho)


@pytest.mark.parametrize("forcing", ["none", "held_suarez"])
def test_large_steps_commute_with_the_grid_rotation(forcing):
    """The grid is invariant under a 72 degree rotation about the axis, and
    so are rotation (Coriolis about z), gravity and a forcing that depends
    on latitude alone.  Two large steps from a rotated state therefore give
    the rotated result of two steps from the original: every column's
    neighbour bookkeeping, every vector's handling and the physics must treat
    all columns alike.  A random horizontal wind makes advection and
    Coriolis act."""
    from scipy.spatial import cKDTree
    from oracle import operators as op
    from tests.gpu_util import small_earth
    if forcing == "none":
        w = small_earth(glevel=3, n_lev=8, n_large=2, noise=1.0)
    else:
        w = workloads.held_suarez(glevel=3, n_lev=10, n_large=2, dt=3000.0, noise_amp=1.0)
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    c, s = np.cos(2 * np.pi / 5), np.sin(2 * np.pi / 5)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    d, perm = cKDTree(model.G.P).query(model.G.P @ R.T)
    assert d.max() < 1e-12 and len(set(perm)) == model.G.n
    rs = np.random.default_rng(1)
    M = op.proj_h(rs.normal(size=st.M.shape) * 3.0, model.rhat) * st.rho[..., None]
    st = dy.State(st.rho, M, st.rth, st.W)

    def rot(x):
        y = np.empty_like(x)
        y[perm] = x
        return y

    st_r = dy.State(rot(st.rho), rot(st.M @ R.T), rot(st.rth), rot(st.W))
    out = dy.run(model, st, w.n_large, w.n_acoustic)
    out_r = dy.run(model, st_r, w.n_large, w.n_acoustic)
    for a, b in ((out_r.rho[perm], out.rho), (out_r.rth[perm], out.rth), (out_r.M[perm], out.M @ R.T)):
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12
    assert np.linalg.norm(out_r.W[perm] - out.W) / np.linalg.norm(out.W) < 1e-10
    # the rotated run is not trivially the same state
    assert np.linalg.norm(out_r.rho - out.rho) > 1e-6 * np.linalg.norm(out.rho)
