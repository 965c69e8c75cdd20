"""Pins of the oracle operators (Eqs. int_grid, flx_div, div_gauss, grad and
the triangle-gradient Laplacian of Sec. 4) against closed forms."""
import numpy as np
import pytest

from oracle import operators as op
from tests.conftest import oracle_grid


def lonlat(P):
    return np.arctan2(P[:, 1], P[:, 0]), np.arcsin(np.clip(P[:, 2], -1, 1))


def heikes_randall(P, m, n):
    """Test functions of Sec. 2.2: alpha = sin(lon), beta = cos(m lon) cos^4(n lat),
    v = alpha grad(beta).  Returns beta, grad beta, v, div v (unit sphere).
    The printed i-component carries sin(lat) where v = alpha grad beta gives
    sin(lon); the definition v = alpha grad beta is used."""
    lam, phi = lonlat(P)
    e = np.stack([-np.sin(lam), np.cos(lam), 0 * lam], -1)
    nn = np.stack([-np.sin(phi) * np.cos(lam), -np.sin(phi) * np.sin(lam), np.cos(phi)], -1)
    cn, sn = np.cos(n * phi), np.sin(n * phi)
    beta = np.cos(m * lam) * cn ** 4
    g_l = -m * np.sin(m * lam) * cn ** 4 / np.cos(phi)
    g_p = -4 * n * cn ** 3 * sn * np.cos(m * lam)
    gb = g_l[:, None] * e + g_p[:, None] * nn
    v = np.sin(lam)[:, None] * gb
    grad_a_dot_grad_b = -m * np.cos(lam) * np.sin(m * lam) * cn ** 4 / np.cos(phi) ** 2
    lap_b = (-m ** 2 * np.cos(m * lam) * cn ** 4 / np.cos(phi) ** 2
             - 4 * n * np.cos(m * lam) * (n * (cn ** 4 - 3 * cn ** 2 * sn ** 2)
                                          - np.tan(phi) * cn ** 3 * sn))
    return beta, gb, v, grad_a_dot_grad_b + np.sin(lam) * lap_b


def hr_errors(G, m, n):
    beta, gb, v, dv = heikes_randall(G.P, m, n)
    w = G.Ac / G.Ac.sum()
    ed = op.div(G, v) - dv
    eg = np.linalg.norm(op.proj_h(op.grad(G, beta), G.P) - gb, axis=1)
    return dict(div_l2=np.sqrt(np.sum(w * ed ** 2)), div_linf=np.abs(ed).max(),
                grad_l2=np.sqrt(np.sum(w * eg ** 2)), grad_linf=eg.max())


def harmonics(P):
    """Real spherical harmonics as harmonic polynomials: (l, Y)."""
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    return [(1, z), (1, x), (2, x * y), (2, 3 * z ** 2 - 1), (3, z * (5 * z ** 2 - 3)),
            (3, x * (x ** 2 - 3 * y ** 2)), (4, 35 * z ** 4 - 30 * z ** 2 + 3),
            (4, x * y * (x ** 2 - y ** 2))]


@pytest.mark.parametrize("smooth", [False, True])
def test_gradient_of_constant_vanishes(smooth):
    """The curvature term of Eq. grad makes grad(const) = 0."""
    G = oracle_grid(4, smooth=smooth)
    g = op.grad(G, np.full(G.n, 7.5))
    assert np.abs(g).max() < 1e-12
    # without the correction term it would not vanish
    sc = op.corner_values(G, np.full(G.n, 7.5))
    assert np.abs(sc - 7.5 * (G.deg[:, None] > np.arange(6))).max() < 1e-12
    assert np.abs(7.5 * G.Sc).max() > 1e-3


def test_discrete_gauss_theorem():
    """sum_i A_i div(F)_i = 0 and sum_i A_i lap(s)_i = 0: every edge flux
    appears twice with opposite normals."""
    G = oracle_grid(4)
    rs = np.random.default_rng(3)
    F = rs.normal(size=(G.n, 3))
    s = rs.normal(size=G.n)
    assert abs(np.sum(G.Ac * op.div(G, F))) < 1e-11
    assert abs(np.sum(G.Ac * op.lap(G, s))) < 1e-10


def test_heikes_randall_second_order_on_modified_grid():
    """Sec. 2.2 / Figs. MN, MN2: on the modified grid the l2 errors of div v
    and grad beta fall at second order; the standard grid is worse, and its
    max-norm divergence error only falls at first order."""
    errs_mod = {g: hr_errors(oracle_grid(g), 1, 1) for g in (3, 4, 5)}
    errs_std = {g: hr_errors(oracle_grid(g, smooth=False), 1, 1) for g in (3, 4, 5)}
    for key in ("div_l2", "grad_l2", "div_linf"):
        slope = np.log2(errs_mod[4][key] / errs_mod[5][key])
        assert slope > 1.85, (key, slope)
    for key in ("div_l2", "div_linf", "grad_l2", "grad_linf"):
        assert errs_mod[5][key] < errs_std[5][key]
    assert np.log2(errs_std[4]["div_linf"] / errs_std[5]["div_linf"]) < 1.3
    e33 = {g: hr_errors(oracle_grid(g), 3, 3) for g in (4, 5)}
    assert np.log2(e33[4]["div_l2"] / e33[5]["div_l2"]) > 1.85


def test_standard_grid_error_peaks_near_icosahedron_edges():
    """Fig. MAPMN: on the standard grid the largest div-error sits next to
    the geodesics of the original icosahedron."""
    from oracle import grid
    G = oracle_grid(5, smooth=False)
    beta, gb, v, dv = heikes_randall(G.P, 1, 1)
    err = np.abs(op.div(G, v) - dv)
    north, south, upper, lower = grid.icosahedron()
    ico = np.vstack([north, south, upper, lower])
    G0 = oracle_grid(0, smooth=False)
    edges = {tuple(sorted(e)) for t in G0.tri for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    normals = np.array([grid.nrm(np.cross(G0.P[a], G0.P[b])) for a, b in edges])
    worst = G.P[np.argsort(err)[-10:]]
    # distance (angle) from each point to the nearest great circle of an edge
    ang = np.min(np.abs(np.arcsin(worst @ normals.T)), axis=1)
    assert np.all(ang < 1.5 * grid.mean_angle(5))
    del ico


@pytest.mark.parametrize("smooth", [False, True])
def test_laplacian_of_spherical_harmonics(smooth):
    """lap Y_l = -l(l+1) Y_l on the unit sphere.  The composite operator of
    Sec. 4 (trapezoid-rule triangle gradients, then the control-volume
    divergence) converges at first order in the area-weighted l2 norm; at the
    12 pentagons its local error stays O(1) under refinement."""
    e = {}
    for g in (4, 5, 6):
        G = oracle_grid(g, smooth=smooth)
        w = G.Ac / G.Ac.sum()
        e[g] = []
        for l, Y in harmonics(G.P):
            err = op.lap(G, Y) + l * (l + 1) * Y
            e[g].append(np.sqrt(np.sum(w * err ** 2)) / (l * (l + 1) * np.sqrt(np.sum(w * Y ** 2))))
    assert max(e[6]) < 1e-2
    slopes = np.log2(np.array(e[5]) / np.array(e[6]))
    assert slopes.min() > 0.9, slopes
    G = oracle_grid(5, smooth=smooth)
    assert np.abs(op.lap(G, np.ones(G.n))).max() < 1e-12


def test_operators_scale_with_radius():
    G = oracle_grid(3)
    rs = np.random.default_rng(5)
    s = rs.normal(size=G.n)
    F = rs.normal(size=(G.n, 3))
    r = 6.0e6
    assert np.allclose(op.div(G, F, r), op.div(G, F) / r, rtol=1e-14, atol=0)
    assert np.allclose(op.grad(G, s, r), op.grad(G, s) / r, rtol=1e-14, atol=1e-30)
    assert np.allclose(op.lap(G, s, r), op.lap(G, s) / r ** 2, rtol=1e-14, atol=1e-40)


def test_level_broadcasting_matches_single_level():
    G = oracle_grid(3)
    rs = np.random.default_rng(6)
    s = rs.normal(size=(G.n, 4))
    F = rs.normal(size=(G.n, 4, 3))
    r = np.array([1.0, 2.0, 3.0, 4.0])
    for k in range(4):
        assert np.allclose(op.div(G, F, r)[:, k], op.div(G, F[:, k], r[k]), rtol=1e-15, atol=1e-15)
        assert np.allclose(op.grad(G, s, r)[:, k], op.grad(G, s[:, k], r[k]), rtol=1e-15, atol=1e-15)
        assert np.allclose(op.lap(G, s, r)[:, k], op.lap(G, s[:, k], r[k]), rtol=1e-15, atol=1e-15)
