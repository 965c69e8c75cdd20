"""Oracle: finite-volume horizontal operators on the icosahedral grid.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

  * corner values by Eq. int_grid (area weights A1, A2, A3);
  * divergence by Eqs. flx_div and div_gauss (Gauss theorem over the 5 or 6
    control-volume edges);
  * gradient by Eq. grad, including the curvature correction term that makes
    the gradient of a constant vanish;
  * Laplacian as in Sec. 4: gradient on the primal triangles (values at the
    cell points, result at the control-volume corners), then Eq. div_gauss on
    the control volume.

Fields are arrays of shape [n] or [n, L] (scalars) and [n, 3] or [n, L, 3]
(Cartesian 3-vectors).  ``r`` is the radius of the spherical surface the
operator acts on (scalar or [L] array); the unit-sphere geometry of ``Grid``
is scaled by it.
"""
import numpy as np


def _radius(r, field_ndim_extra):
    r = np.asarray(r, dtype=np.float64)
    if r.ndim == 0:
        return r
    # broadcast over [n, L] or [n, L, 3]
    return r.reshape((1, -1) + (1,) * field_ndim_extra)


def corner_values(G, f):
    """Eq. int_grid: f*_k at corner C_k of every cell; shape [n, 6, ...]."""
    nb = np.where(G.nbr >= 0, G.nbr, 0)
    nb1 = np.roll(nb, -1, axis=1)
    # pentagons: the cycle closes after 5 entries
    pent = G.deg == 5
    nb1[pent, 4] = nb[pent, 0]
    extra = (1,) * (f.ndim - 1)
    w0 = G.w[:, :, 0].reshape(G.n, 6, *extra)
    wk = G.w[:, :, 1].reshape(G.n, 6, *extra)
    wk1 = G.w[:, :, 2].reshape(G.n, 6, *extra)
    fc = w0 * f[:, None] + wk * f[nb] + wk1 * f[nb1]
    fc[pent, 5] = 0.0
    return fc


def _next_corner(G, fc):
    nxt = np.roll(fc, -1, axis=1)
    pent = G.deg == 5
    nxt[pent, 4] = fc[pent, 0]
    nxt[pent, 5] = 0.0
    return nxt


def div(G, F, r=1.0):
    """Horizontal divergence of a Cartesian vector field F[n, (L,) 3]."""
    fc = corner_values(G, F)
    avg = 0.5 * (fc + _next_corner(G, fc))
    extra = F.ndim - 2
    ln = (G.l[..., None] * G.nh).reshape((G.n, 6) + (1,) * extra + (3,))
    flux = np.sum(np.sum(avg * ln, axis=-1), axis=1)
    return flux / (G.Ac.reshape((G.n,) + (1,) * extra) * _radius(r, 0))


def grad(G, s, r=1.0):
    """Horizontal gradient of a scalar s[n, (L)], as Cartesian vectors."""
    sc = corner_values(G, s)
    avg = 0.5 * (sc + _next_corner(G, sc))
    extra = s.ndim - 1
    ln = (G.l[..., None] * G.nh).reshape((G.n, 6) + (1,) * extra + (3,))
    total = np.sum(avg[..., None] * ln, axis=1)
    Sc = G.Sc.reshape((G.n,) + (1,) * extra + (3,))
    total = total - s[..., None] * Sc
    return total / (G.Ac.reshape((G.n,) + (1,) * extra + (1,)) * _radius(r, 1))


def triangle_grad(G, s):
    """Eq. grad on the primal triangles (unit sphere); result at corners C_tau."""
    t = G.tri
    sv = s[t]                                   # [T, 3, ...]
    se = np.roll(sv, -1, axis=1)                # edge e: vertex e -> e+1
    extra = s.ndim - 1
    tl = G.tl.reshape(G.tl.shape + (1,) * extra + (1,))
    tn = G.tn.reshape((G.tn.shape[0], 3) + (1,) * extra + (3,))
    total = np.sum(tl * 0.5 * (sv + se)[..., None] * tn, axis=1)
    tw = G.tw.reshape((G.tw.shape[0], 3) + (1,) * extra)
    s_c = np.sum(tw * sv, axis=1)               # value at the centroid
    Sl = np.sum(tl * tn, axis=1)
    total = total - s_c[..., None] * Sl
    return total / G.tA.reshape((-1,) + (1,) * extra + (1,))


def lap(G, s, r=1.0):
    """Horizontal Laplacian (Sec. 4): control-volume divergence of the
    triangle gradients, which already sit at the control-volume corners."""
    Gt = triangle_grad(G, s)                    # [T, ..., 3]
    ct = np.where(G.corner_tri >= 0, G.corner_tri, 0)
    gc = Gt[ct]                                 # [n, 6, ..., 3]
    pent = G.deg == 5
    gc[pent, 5] = 0.0
    avg = 0.5 * (gc + _next_corner(G, gc))
    extra = s.ndim - 1
    ln = (G.l[..., None] * G.nh).reshape((G.n, 6) + (1,) * extra + (3,))
    flux = np.sum(np.sum(avg * ln, axis=-1), axis=1)
    rr = _radius(r, 0)
    return flux / (G.Ac.reshape((G.n,) + (1,) * extra) * rr * rr)


def proj_h(F, rhat):
    """Eq. proj_h: remove the radial component, F - (F . rhat) rhat."""
    rh = rhat.reshape((rhat.shape[0],) + (1,) * (F.ndim - 2) + (3,))
    return F - np.sum(F * rh, axis=-1, keepdims=True) * rh


def proj_r(F, rhat):
    """Eq. proj_r: radial component F . rhat."""
    rh = rhat.reshape((rhat.shape[0],) + (1,) * (F.ndim - 2) + (3,))
    return np.sum(F * rh, axis=-1)
