"""Oracle: post-processing of THOR output on pressure levels.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's results are shown on pressure levels: fields are interpolated
linearly in pressure from the model levels (Sec. 7, opening of the results),
averaged zonally and in time; eddies are deviations from the zonal average
(phi' = phi - [phi]) and the mass streamfunction is
Psi = 2 pi A cos(lat) / g * integral_0^p [v] dp.

Readings (the paper does not say how these are formed on an icosahedral
grid, nor what happens outside a column's pressure range):
  * a pressure level outside [p of the top cell, p of the bottom cell] of a
    column has no value there and is left out of that column's averages;
  * zonal averages are area-weighted means over latitude bands of equal
    width (band b covers [-90 + 180 b / n, -90 + 180 (b + 1) / n) degrees;
    the north pole belongs to the last band) of the columns with a value;
  * eddy fluxes are formed per snapshot, [u'v'] = [uv] - [u][v], and then
    averaged in time like every other quantity; a band/level without any
    value in a snapshot contributes nothing to that snapshot's average;
  * Psi integrates with the trapezoid rule over the pressure levels and
    takes [v] at p = 0 equal to its value at the first (smallest) level;
  * the grid-imprinting map [w*] (Sec. 7.1, Held-Suarez results) uses the
    deviation of w from its zonal (band) mean, w* = w - {w}, on the first
    model layer, and then averages it in time: with the bracket read as a
    time mean alone, w - [w] would average to zero identically.
"""
import numpy as np

from .dynamics import lon_lat

QUANTITIES = ("u", "v", "T", "theta", "upvp", "vpTp", "weight")


def interpolate(p, q, plev):
    """Linear interpolation in pressure of q [N, L] (levels upward, p
    decreasing) to the pressures plev [P].  Returns values [N, P] and a mask
    of the columns/levels inside the column's pressure range."""
    N, L = p.shape
    out = np.zeros((N, len(plev)))
    valid = np.zeros((N, len(plev)), dtype=bool)
    for i in range(N):
        for j, pj in enumerate(plev):
            for k in range(L - 1):
                lo, hi = p[i, k + 1], p[i, k]   # lo < hi
                if lo <= pj <= hi:
                    w = (pj - lo) / (hi - lo)
                    out[i, j] = q[i, k + 1] + w * (q[i, k] - q[i, k + 1])
                    valid[i, j] = True
                    break
    return out, valid


def band_of(lat, n_bands):
    b = np.floor((lat + np.pi / 2) / np.pi * n_bands).astype(int)
    return np.clip(b, 0, n_bands - 1)


def snapshot(model, st, plev, n_bands):
    """Band means [n_bands, P] of u, v, T, theta and the eddy fluxes of one
    state, plus the valid weight fraction of each band/level."""
    from .dynamics import fields
    f = fields(model, st)
    theta = st.rth / st.rho
    A = model.G.Ac
    lam, lat = lon_lat(model.rhat)
    band = band_of(lat, n_bands)
    vals = {}
    valid = None
    for name, q in (("u", f["u"]), ("v", f["v"]), ("T", f["T"]), ("theta", theta)):
        vals[name], valid = interpolate(f["p"], q, plev)
    out = {k: np.zeros((n_bands, len(plev))) for k in QUANTITIES}
    present = np.zeros((n_bands, len(plev)), dtype=bool)
    for b in range(n_bands):
        cols = np.flatnonzero(band == b)
        Ab = A[cols].sum()
        for j in range(len(plev)):
            m = valid[cols, j]
            if not m.any():
                continue
            c = cols[m]
            w = A[c] / A[c].sum()
            mean = {k: np.sum(w * vals[k][c, j]) for k in ("u", "v", "T", "theta")}
            for k in ("u", "v", "T", "theta"):
                out[k][b, j] = mean[k]
            out["upvp"][b, j] = np.sum(w * (vals["u"][c, j] - mean["u"]) * (vals["v"][c, j] - mean["v"]))
            out["vpTp"][b, j] = np.sum(w * (vals["v"][c, j] - mean["v"]) * (vals["T"][c, j] - mean["T"]))
            out["weight"][b, j] = A[c].sum() / Ab
            present[b, j] = True
    return out, present


def time_mean(snaps):
    """Average of snapshot results; each band/level over the snapshots in
    which it had a value."""
    keys = QUANTITIES
    num = {k: np.zeros_like(snaps[0][0][k]) for k in keys}
    cnt = np.zeros_like(snaps[0][0]["u"])
    for out, present in snaps:
        for k in keys:
            num[k] += np.where(present, out[k], 0.0)
        cnt += present
    return {k: np.where(cnt > 0, num[k] / np.maximum(cnt, 1), 0.0) for k in keys}, cnt


def band_latitudes(n_bands):
    return -np.pi / 2 + (np.arange(n_bands) + 0.5) * np.pi / n_bands


def streamfunction(vbar, plev, radius, gravity):
    """Psi [n_bands, P] = 2 pi A cos(lat) / g * int_0^p [v] dp (trapezoid
    over plev ascending; [v](0) = [v](plev[0]))."""
    lat = band_latitudes(vbar.shape[0])
    integ = np.zeros_like(vbar)
    integ[:, 0] = vbar[:, 0] * plev[0]
    for j in range(1, len(plev)):
        integ[:, j] = integ[:, j - 1] + 0.5 * (vbar[:, j] + vbar[:, j - 1]) * (plev[j] - plev[j - 1])
    return 2 * np.pi * radius * np.cos(lat)[:, None] / gravity * integ


def first_layer_w(model, st):
    """Vertical velocity at the centre of the lowest layer, per column: the
    mean of its two interface momenta (the ground one is zero) over rho."""
    return 0.5 * (st.W[:, 0] + st.W[:, 1]) / st.rho[:, 0]


def imprint_snapshot(model, st, n_bands):
    """w* of one state in the first layer: w minus the area-weighted mean of
    w over the column's latitude band (the grid-imprinting diagnostic of
    Sec. 7.1 before its time average)."""
    w = first_layer_w(model, st)
    _, lat = lon_lat(model.rhat)
    band = band_of(lat, n_bands)
    A = model.G.Ac
    out = np.zeros_like(w)
    for b in range(n_bands):
        c = np.flatnonzero(band == b)
        if len(c):
            out[c] = w[c] - np.sum(A[c] * w[c]) / A[c].sum()
    return out


def imprint_map(snaps):
    """[w*]: the time average of the per-snapshot w* maps."""
    return np.mean(np.stack(snaps), axis=0)
