"""Pins of the oracle's Sec. 4 dissipation terms against closed forms on the
sphere: the momentum and vertical-momentum hyperdiffusion (Eqs. diff_vx,
diff_vy, diff_vz, diff_vr, reading F_q = -lap(rho Kd lap v_q) per Cartesian
component, projected) and the 3D divergence damping applied inside every
acoustic substep (Sec. 4, text after Eq. diff_vr; Eqs. kd, tau_d).

Closed forms used (unit sphere, Delta_S the surface Laplacian, Y a degree-l
spherical harmonic, lambda = l (l + 1)):
  * toroidal flow v = rhat x grad_S Y: every Cartesian component is a degree-l
    harmonic, so Delta_S Delta_S v = lambda^2 v (tangent);
  * poloidal flow v = grad_S Y: with F the harmonic polynomial extending Y,
    v_q = d_q F - l Y x_q, and Delta_S v = -lambda (v - 2 Y rhat); applying
    it twice, the tangent part of Delta_S Delta_S v is lambda (lambda + 4) v;
  * rigid rotation v = zhat x rhat (l = 1 toroidal) on a density
    rho0 (1 + eps z): Delta_S v = -2 v, and z v has degree-2 harmonic
    components, so -lap(rho lap v) = -rho0 (4 v + 12 eps z v); putting rho
    outside both Laplacians would give 4 for the second coefficient, inside
    both (on the momentum) 36.
On a sphere of radius r each Laplacian carries 1/r^2, each gradient or
divergence 1/r.  The discrete operators are only first order pointwise (the
pentagons), so every check projects the term onto the closed form's shape
with the control-volume areas; that projection converges at second order,
so the deviation must halve or better from g4 to g5.
"""
import numpy as np
import pytest

from oracle import dynamics as dy
from oracle import operators as op
from tests.conftest import oracle_grid

# a tall atmosphere on a small planet: the centre and interface radii differ
# by tens of percent, so a term taken at the wrong radius cannot pass
RADIUS, Z_TOP, L = 1.0e6, 1.2e6, 3
RHO_LEV = np.array([1.3, 0.7, 0.4])


def _model(g, div_damp=False):
    G = oracle_grid(g)
    planet = dy.Planet(RADIUS, 0.0, 9.8, 287.0, 1005.0)
    return dy.Model(G, planet, dy.Vertical(L, Z_TOP), dy.Numerics(600.0, 2.0e-2, div_damp))


def _coef(G, term, shape):
    """Area-weighted projection of term[n, L, (3)] onto shape[n, L, (3)], per
    level: sum A t . s / sum A s . s."""
    A = G.Ac[:, None]
    if term.ndim == 3:
        return np.sum(A * np.sum(term * shape, -1), 0) / np.sum(A * np.sum(shape * shape, -1), 0)
    return np.sum(A * term * shape, 0) / np.sum(A * shape * shape, 0)


def _harmonic_flows(P):
    """Unit-sphere degree-2 toroidal and poloidal flows of Y = 3 z^2 - 1 and
    the rigid rotation zhat x rhat."""
    z = P[:, 2]
    gradY = 6.0 * z[:, None] * (np.array([0.0, 0.0, 1.0]) - z[:, None] * P)
    tor = np.cross(P, gradY)
    rigid = np.cross(np.array([0.0, 0.0, 1.0]), P)
    return gradY, tor, rigid


def _state(model, M, rho):
    n = model.G.n
    return dy.State(rho, M, model.rth_from_p(rho * 287.0 * 250.0), np.zeros((n, L + 1)))


def _deviations(check):
    dev = {g: check(g) for g in (4, 5)}
    return dev


@pytest.mark.parametrize("kind,factor", [("toroidal", 36.0), ("poloidal", 60.0)])
def test_momentum_hyperdiffusion_of_degree2_flows(kind, factor):
    """Eqs. diff_vx-diff_vz at uniform density (per level): H_M equals
    -Kd rho (factor / r_C^4) v with factor lambda^2 = 36 (toroidal) or
    lambda (lambda + 4) = 60 (poloidal), and has no radial part."""
    def check(g):
        model = _model(g)
        G = model.G
        gradY, tor, _ = _harmonic_flows(G.P)
        v = (tor if kind == "toroidal" else gradY)[:, None, :] * np.array([3.0, -2.0, 5.0])[None, :, None]
        rho = np.broadcast_to(RHO_LEV, (G.n, L)).copy()
        st = _state(model, rho[..., None] * v, rho)
        _, H_M, _, _ = dy.hyperdiffusion(model, st, model.eos(st.rth))
        assert np.abs(op.proj_r(H_M, G.P)).max() < 1e-12 * np.abs(H_M).max()
        ref = -model.Kd * RHO_LEV * factor / model.rC ** 4
        return np.abs(_coef(G, H_M, v) / ref - 1).max()
    dev = _deviations(check)
    assert dev[5] < 1e-2 and dev[5] < 0.5 * dev[4], dev


def test_momentum_hyperdiffusion_density_between_the_laplacians():
    """Eq. diff_vx-diff_vz put rho between the two Laplacians: for a rigid
    rotation on rho0 (1 + eps z), H_M = -Kd rho0 / r_C^4 (4 v + 12 eps z v)."""
    eps = 0.3

    def check(g):
        model = _model(g)
        G = model.G
        _, _, rigid = _harmonic_flows(G.P)
        rho = RHO_LEV[None, :] * (1.0 + eps * G.P[:, 2:3])
        v = np.broadcast_to(rigid[:, None, :], (G.n, L, 3)) * 40.0
        st = _state(model, rho[..., None] * v, rho)
        _, H_M, _, _ = dy.hyperdiffusion(model, st, model.eos(st.rth))
        zv = G.P[:, 2, None, None] * v
        base = -model.Kd * RHO_LEV / model.rC ** 4
        d1 = np.abs(_coef(G, H_M, v) / (4.0 * base) - 1).max()
        d2 = np.abs(_coef(G, H_M, zv) / (12.0 * eps * base) - 1).max()
        return max(d1, d2)
    dev = _deviations(check)
    assert dev[5] < 1e-2 and dev[5] < 0.5 * dev[4], dev


def test_vertical_momentum_hyperdiffusion():
    """Eq. diff_vr at the interior interfaces: F = -lap(rho_I Kd lap w) with
    w = W / rho_I and r the interface radius.  Uniform rho_I and w a degree-2
    harmonic: -Kd rho_I 36 / r_I^4 w.  rho_I (1 + eps z) with w = x (degree
    1): -Kd rho_I / r_I^4 (4 x + 12 eps x z)."""
    eps = 0.25

    def check(g):
        model = _model(g)
        G = model.G
        x, z = G.P[:, 0], G.P[:, 2]
        rI = model.rI[1:L]
        rhoI_lev = 0.5 * (RHO_LEV[:-1] + RHO_LEV[1:])
        out = []
        for shape, rho_h, factors in (((3 * z ** 2 - 1), 0.0, (36.0, None)),
                                      (x, eps, (4.0, 12.0))):
            rho = RHO_LEV[None, :] * (1.0 + rho_h * z[:, None])
            rhoI = rhoI_lev[None, :] * (1.0 + rho_h * z[:, None])
            w = shape[:, None] * np.array([2.0, -1.5])[None, :]
            W = np.zeros((G.n, L + 1))
            W[:, 1:L] = rhoI * w
            st = dy.State(rho, np.zeros((G.n, L, 3)), model.rth_from_p(rho * 287.0 * 250.0), W)
            _, _, H_W, _ = dy.hyperdiffusion(model, st, model.eos(st.rth))
            assert np.all(H_W[:, 0] == 0) and np.all(H_W[:, L] == 0)
            base = -model.Kd * rhoI_lev / rI ** 4
            out.append(np.abs(_coef(G, H_W[:, 1:L], w) / (factors[0] * base) - 1).max())
            if factors[1] is not None:
                xz = (x * z)[:, None] * np.array([2.0, -1.5])[None, :]
                out.append(np.abs(_coef(G, H_W[:, 1:L], xz) / (factors[1] * rho_h * base) - 1).max())
        return max(out)
    dev = _deviations(check)
    assert dev[5] < 1e-2 and dev[5] < 0.5 * dev[4], dev


def _substep_pair(model_on, model_off, st):
    """The same acoustic substep with divergence damping on and off."""
    large = dy.large_step_terms(model_on, st)
    f = dy.slow_forcing(model_on, st, large)
    dtau = 75.0
    on = dy.acoustic_substep(model_on, st, f, dtau, large)
    off = dy.acoustic_substep(model_off, st, f, dtau, large)
    return on, off, dtau


def test_divergence_damping_inside_the_substep_horizontal():
    """Sec. 4: the substep adds dtau * proj_h(-Kd lap(grad D)) to M.  For the
    irrotational M = c_k grad_S Y (Y of degree 2, W = 0), D = -6 c_k Y / r,
    grad D = -6 M / r^2 and the tangent part of the damping is
    -Kd (6 / r_C^2)^2 M: the momentum difference between the substep with
    and without damping is that times dtau."""
    def check(g):
        m_on, m_off = _model(g, True), _model(g, False)
        G = m_on.G
        gradY, _, _ = _harmonic_flows(G.P)
        M = gradY[:, None, :] * np.array([0.8, -0.3, 0.5])[None, :, None]
        rho = np.broadcast_to(RHO_LEV, (G.n, L)).copy()
        on, off, dtau = _substep_pair(m_on, m_off, _state(m_on, M, rho))
        dM = on.M - off.M
        ref = -dtau * m_on.Kd * 36.0 / m_on.rC ** 4
        return np.abs(_coef(G, dM, M) / ref - 1).max()
    dev = _deviations(check)
    assert dev[5] < 1e-2 and dev[5] < 0.5 * dev[4], dev


def test_divergence_damping_inside_the_substep_vertical():
    """D is the 3D divergence: with M = 0 and W_j = c s_j Y at the interior
    interfaces, D_k = g_k Y with g_k = c (r_{k+1}^2 s_{k+1} - r_k^2 s_k) /
    (r_C,k^2 dz) (interface radii r), and the damping's tangent part is
    +6 Kd g_k / r_C^3 grad_S Y (momentum pushed toward the divergence
    maxima, which lowers them)."""
    def check(g):
        m_on, m_off = _model(g, True), _model(g, False)
        G = m_on.G
        gradY, _, _ = _harmonic_flows(G.P)
        Y = 3 * G.P[:, 2] ** 2 - 1
        s = np.array([0.0, 0.6, -0.9, 0.0]) * 2.0
        W = Y[:, None] * s[None, :]
        rho = np.broadcast_to(RHO_LEV, (G.n, L)).copy()
        st = dy.State(rho, np.zeros((G.n, L, 3)), m_on.rth_from_p(rho * 287.0 * 250.0), W)
        on, off, dtau = _substep_pair(m_on, m_off, st)
        dM = on.M - off.M
        rI2 = m_on.rI ** 2
        gk = (rI2[1:] * s[1:] - rI2[:-1] * s[:-1]) / (m_on.rC ** 2 * m_on.dz)
        ref = dtau * 6.0 * m_on.Kd * gk / m_on.rC ** 3
        shape = np.broadcast_to(gradY[:, None, :], (G.n, L, 3))
        return np.abs(_coef(G, dM, shape) / ref - 1).max()
    dev = _deviations(check)
    assert dev[5] < 1e-2 and dev[5] < 0.5 * dev[4], dev


def test_divergence_damping_lowers_the_divergence():
    """The damped substep leaves a smaller momentum divergence than the
    undamped one when the divergence comes from M alone."""
    m_on, m_off = _model(4, True), _model(4, False)
    G = m_on.G
    gradY, _, _ = _harmonic_flows(G.P)
    M = gradY[:, None, :] * np.array([0.8, -0.3, 0.5])[None, :, None]
    rho = np.broadcast_to(RHO_LEV, (G.n, L)).copy()
    on, off, _ = _substep_pair(m_on, m_off, _state(m_on, M, rho))
    A = G.Ac[:, None]
    d_on = np.sum(A * op.div(G, on.M, m_on.rC) ** 2)
    d_off = np.sum(A * op.div(G, off.M, m_on.rC) ** 2)
    assert d_on < d_off
