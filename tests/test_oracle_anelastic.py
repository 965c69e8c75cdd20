"""Pins of the oracle's anelastic switch (Sec. 3 list of approximations:
the density in the divergence term of the mass continuity equation is
replaced by a reference density that depends on altitude only).  Reading:
the mass flux rho v becomes rho_r v, rho_r the isothermal reference column
of the initial state, v the momentum over the density of Phi[t]; the
momentum, rho theta and the equation of state keep the full density."""
import numpy as np

from oracle import dynamics as dy
from tests.conftest import oracle_grid
from tests.gpu_util import small_earth


def _model(w, anelastic):
    w.anelastic = anelastic
    return dy.model_from_workload(w, oracle_grid(w.glevel))


def _stirred(model, st, seed, amp=20.0):
    """The state with a tangent momentum field of magnitude ~amp x rho (and
    W left at zero), so that the mass flux has a horizontal divergence."""
    rs = np.random.default_rng(seed)
    v = rs.normal(size=st.M.shape)
    v = dy.op.proj_h(v, model.rhat)
    out = st.copy()
    out.M = amp * st.rho[..., None] * v
    return out


def test_anelastic_equals_compressible_when_rho_is_the_reference():
    """With rho[t] equal to the reference column in every cell (no
    temperature noise, reference set to the state's own column) the flux
    factors are exactly 1 and a whole large step is the compressible one,
    bit for bit."""
    outs = {}
    for ane in (False, True):
        w = small_earth(glevel=2, n_lev=8, noise=0.0)
        model, st = _model(w, ane)
        model.rho_ref = st.rho[0].copy()
        st = _stirred(model, st, seed=3)
        outs[ane] = dy.large_step(model, st, w.n_acoustic)
    for k in ("rho", "rth", "M", "W"):
        assert np.array_equal(getattr(outs[False], k), getattr(outs[True], k)), k


def test_single_level_density_tendency_scales_with_the_reference():
    """One level (no vertical flux): the density change of a substep beyond
    its slow forcing is -dtau div(rho_r / rho[t] M).  With rho[t]
    horizontally uniform and rho_r = lambda rho[t], it is lambda times the
    compressible one."""
    lam = 0.7
    dtau = 30.0
    res = {}
    for ane in (False, True):
        w = small_earth(glevel=2, n_lev=1, noise=0.0)
        model, st = _model(w, ane)
        model.rho_ref = lam * st.rho[0].copy()
        st = _stirred(model, st, seed=5)
        large = dy.large_step_terms(model, st)
        f = dy.slow_forcing(model, st, large)
        out = dy.acoustic_substep(model, st, f, dtau, large)
        res[ane] = out.rho - st.rho - dtau * f["S_rho"]
    ref = np.abs(res[False]).max()
    assert ref > 0
    assert np.abs(res[True] - lam * res[False]).max() < 1e-12 * ref


def test_anelastic_step_conserves_mass():
    """The mass flux stays in flux form (horizontal fluxes cancel between
    cells, the vertical flux vanishes at the ground and the top): total mass
    is kept to rounding over large steps of a noisy, stirred state whose
    density differs from the reference."""
    w = small_earth(glevel=2, n_lev=10, noise=2.0)
    model, st = _model(w, True)
    st = _stirred(model, st, seed=7, amp=5.0)
    m0 = dy.mass(model, st)
    out = dy.run(model, st, 2, w.n_acoustic)
    assert abs(dy.mass(model, out) / m0 - 1) < 1e-13
    # and the switch is engaged: the result differs from the compressible one
    w2 = small_earth(glevel=2, n_lev=10, noise=2.0)
    model2, st2 = _model(w2, False)
    st2 = _stirred(model2, st2, seed=7, amp=5.0)
    out2 = dy.run(model2, st2, 2, w2.n_acoustic)
    assert np.abs(out.rho - out2.rho).max() > 1e-6 * np.abs(out2.rho).max()


def test_anelastic_rest_state_stays_at_rest():
    """The isothermal column at rest, without noise, is its own reference to
    rounding: it stays at rest under the anelastic step."""
    w = small_earth(glevel=2, n_lev=12, noise=0.0)
    model, st = _model(w, True)
    out = dy.run(model, st, 2, w.n_acoustic)
    speed = np.sqrt(np.sum(out.M ** 2, axis=-1)) / out.rho
    assert speed.max() < 1e-9
    assert np.abs(out.W).max() < 1e-9 * out.rho.max()


def test_hydrostatic_anelastic_substep_balances_the_column():
    """The buoyancy of the W equation must see the same density change as
    the density update.  With the hydrostatic switch the new W is the one
    that leaves the column balanced at the end of the substep: the [t]
    imbalance, the deviation pressure gradient and the buoyancy of the
    output density sum to zero, with the pressure the scheme's linearised
    equation of state gives (p + Gamma (rho theta_out - rho theta)), to
    rounding.  The reference is 0.7 times the state's density, so the
    anelastic flux factor is far from 1."""
    w = small_earth(glevel=2, n_lev=12, noise=0.1)
    w.hydrostatic = True
    model, st = _model(w, True)
    model.rho_ref = 0.7 * st.rho.mean(axis=0)
    large = dy.large_step_terms(model, st)
    f = dy.slow_forcing(model, st, large)
    out = dy.acoustic_substep(model, st, f, 2.0, large)
    g, dz = model.planet.gravity, model.dz
    p_lin = model.eos(st.rth) + f["Gam"] * (out.rth - st.rth)
    ps = p_lin - large["p_t"]
    rs = out.rho - large["rho_t"]
    res = (large["I"][:, 1:-1] - (ps[:, 1:] - ps[:, :-1]) / dz - 0.5 * g * (rs[:, :-1] + rs[:, 1:]))
    scale = np.abs(large["I"][:, 1:-1]).max()
    assert np.abs(res).max() < 1e-9 * scale
