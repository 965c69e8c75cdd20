"""Pins of the oracle's total energy and of the energy fixer (a globally
uniform internal-energy adjustment in the manner of Williamson 2009, Sec. 3
discussion of the thermodynamic equation)."""
import math

import numpy as np
import pytest

import workloads
from oracle import dynamics as dy
from tests.conftest import oracle_grid


def _uniform_state(model, rho0, p0):
    n, L = model.G.n, model.vert.n_lev
    rho = np.full((n, L), rho0)
    rth = model.rth_from_p(np.full((n, L), p0))
    return dy.State(rho, np.zeros((n, L, 3)), rth, np.zeros((n, L + 1)))


def _model(glevel=4, n_lev=12):
    w = workloads.small_gas_giant(glevel=glevel, n_lev=n_lev)
    model, _ = dy.model_from_workload(w, oracle_grid(glevel))
    return model


def test_internal_and_potential_energy_of_a_uniform_shell():
    """Uniform rho0, p0, at rest: E = Cv p0 / Rd * V + rho0 g int z dV over the
    shell A <= r <= A + H.  The cells use the midpoint rule in r: for
    int z (A + z)^2 dz its relative error is about H / (3 A L^2), for the
    volume about dz^2 / (12 A^2)."""
    model = _model()
    pl = model.planet
    A, H = pl.radius, model.vert.z_top
    rho0, p0 = 0.3, 2.0e4
    E = dy.total_energy(model, _uniform_state(model, rho0, p0))
    V = 4 * math.pi * ((A + H) ** 3 - A ** 3) / 3
    Zint = 4 * math.pi * (A * A * H * H / 2 + 2 * A * H ** 3 / 3 + H ** 4 / 4)
    ref = model.Cv / pl.Rd * p0 * V + rho0 * pl.gravity * Zint
    L = model.vert.n_lev
    tol = H / (A * L * L)
    assert abs(E / ref - 1) < tol
    # each part alone: zero gravity leaves the internal energy
    model.planet.gravity, g = 0.0, model.planet.gravity
    try:
        E0 = dy.total_energy(model, _uniform_state(model, rho0, p0))
    finally:
        model.planet.gravity = g
    dz = model.dz
    assert abs(E0 / (model.Cv / pl.Rd * p0 * V) - 1) < dz * dz / (6 * A * A)
    assert abs((E - E0) / (rho0 * g * Zint) - 1) < tol


def test_kinetic_energy_of_solid_body_rotation():
    """u = U cos(lat) east, uniform rho0: the kinetic energy is
    rho0 U^2 / 2 * (8 pi / 3) int r^2 dr; the sum over the cells converges
    to it with the grid's area quadrature."""
    U, rho0, p0 = 40.0, 0.3, 2.0e4
    errs = []
    for g in (3, 4):
        model = _model(glevel=g)
        st = _uniform_state(model, rho0, p0)
        rest = dy.total_energy(model, st)
        lam, phi = dy.lon_lat(model.rhat)
        east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], axis=-1)
        M = (rho0 * U * np.cos(phi))[:, None, None] * east[:, None, :] * np.ones((1, model.vert.n_lev, 1))
        KE = dy.total_energy(model, dy.State(st.rho, M, st.rth, st.W)) - rest
        A, H = model.planet.radius, model.vert.z_top
        ref = 0.5 * rho0 * U * U * (8 * math.pi / 3) * ((A + H) ** 3 - A ** 3) / 3
        errs.append(abs(KE / ref - 1))
    assert errs[1] < 2e-3 and errs[1] < errs[0]


def test_vertical_kinetic_energy_uses_centre_momentum():
    """rho v_r = m at every interior interface (zero at the ground and the
    lid): the centre values are m in the interior layers and m / 2 in the
    first and last, so the vertical kinetic energy is
    m^2 / (2 rho0) * (sum of interior volumes + (first + last volumes) / 4)."""
    model = _model(glevel=3, n_lev=8)
    rho0, p0, m = 0.3, 2.0e4, 60.0   # large, so that E - E(rest) keeps its digits
    st = _uniform_state(model, rho0, p0)
    rest = dy.total_energy(model, st)
    W = np.zeros_like(st.W)
    W[:, 1:-1] = m
    KE = dy.total_energy(model, dy.State(st.rho, st.M, st.rth, W)) - rest
    vol = model.G.Ac.sum() * model.rC ** 2 * model.dz
    ref = m * m / (2 * rho0) * (vol[1:-1].sum() + (vol[0] + vol[-1]) / 4)
    assert abs(KE / ref - 1) < 1e-10


def test_fixer_restores_the_target_with_one_uniform_temperature_increment():
    w = workloads.small_gas_giant(glevel=3, n_lev=10)
    w.noise_amp = 1.0
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    pl = model.planet
    E = dy.total_energy(model, st)
    target = E * (1 + 3e-7)
    out = dy.fix_energy(model, st, target)
    assert abs(dy.total_energy(model, out) / target - 1) < 1e-14
    T0 = model.eos(st.rth) / (st.rho * pl.Rd)
    T1 = model.eos(out.rth) / (out.rho * pl.Rd)
    dT = T1 - T0
    assert dT.min() > 0 and dT.max() - dT.min() < 1e-12 * T0.max()   # round-off of T itself
    assert abs(dT.mean() / (3e-7 * E / (model.Cv * dy.mass(model, st))) - 1) < 1e-8
    assert out.rho is st.rho and out.M is st.M and out.W is st.W


@pytest.mark.parametrize("fixer", [False, True])
def test_a_large_step_with_the_fixer_conserves_total_energy(fixer):
    """With no forcing the fixer returns the total energy of the step's start
    (to round-off); without it the dynamics (hyperdiffusion, divergence
    damping, time truncation) changes it measurably."""
    w = workloads.small_gas_giant(glevel=3, n_lev=10)
    w.noise_amp = 2.0
    w.forcing_kind = 0
    w.energy_fixer = fixer
    model, st = dy.model_from_workload(w, oracle_grid(w.glevel))
    E0 = dy.total_energy(model, st)
    out = dy.run(model, st, 2, w.n_acoustic)
    rel = abs(dy.total_energy(model, out) / E0 - 1)
    if fixer:
        assert rel < 1e-13
    else:
        assert rel > 1e-10


def test_axial_angular_momentum_of_solid_body_rotation():
    """Uniform rho0, u = U cos(lat): the relative part is
    rho0 U (8 pi / 3) int r^3 dr and the planetary part
    rho0 Omega (8 pi / 3) int r^4 dr.  The cells integrate cos^2(lat) over
    the sphere exactly (the icosahedral symmetry); the midpoint rule in r
    leaves a relative error of about dz^2 / (2 A^2) for r^4 and
    dz^2 / (4 A^2) for r^3.  A purely meridional wind adds nothing."""
    rho0, p0, U = 0.3, 2.0e4, 40.0
    for g in (3, 4):
        model = _model(glevel=g)
        A, H, Om = model.planet.radius, model.vert.z_top, model.planet.omega
        dz = model.dz
        st = _uniform_state(model, rho0, p0)
        lam, phi = dy.lon_lat(model.rhat)
        east = np.stack([-np.sin(lam), np.cos(lam), np.zeros_like(lam)], axis=-1)
        north = np.stack([-np.sin(phi) * np.cos(lam), -np.sin(phi) * np.sin(lam), np.cos(phi)], axis=-1)
        L = model.vert.n_lev
        planetary = dy.axial_angular_momentum(model, st)
        ref_p = rho0 * Om * (8 * math.pi / 3) * ((A + H) ** 5 - A ** 5) / 5
        assert abs(planetary / ref_p - 1) < dz * dz / A ** 2
        M = (rho0 * U * np.cos(phi))[:, None, None] * east[:, None, :] * np.ones((1, L, 1))
        rel = dy.axial_angular_momentum(model, dy.State(st.rho, M, st.rth, st.W)) - planetary
        ref_r = rho0 * U * (8 * math.pi / 3) * ((A + H) ** 4 - A ** 4) / 4
        assert abs(rel / ref_r - 1) < dz * dz / (2 * A ** 2)
        Mn = (rho0 * 7.0 * np.cos(phi) ** 2)[:, None, None] * north[:, None, :] * np.ones((1, L, 1))
        mer = dy.axial_angular_momentum(model, dy.State(st.rho, Mn, st.rth, st.W)) - planetary
        assert abs(mer) < 1e-12 * abs(ref_r)
