"""Oracle: icosahedral grid, spring dynamics and control-volume geometry.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. 2.1 (standard icosahedral grid: icosahedron with vertices at
the poles, 10-rhombus decomposition, recursive edge bisection, Eq. grid_qts,
dual grid of pentagons and hexagons) and Sec. 2.2 (spring dynamics, Eqs.
spring_force / spr_vel / dbar, then centroid relocation with the centroid
equation).  Where the paper is silent (icosahedron longitude, point numbering,
neighbour order, integrator, spring constant) the readings listed in the
design notes are used:

  * icosahedron: upper ring at latitude atan(1/2), longitudes 2 pi k / 5;
    lower ring at -atan(1/2), longitudes 2 pi k / 5 + pi / 5;
  * rhombus r = k (north): corners (T, Lf, B, R) = (N, U_k, L_k, U_k+1),
    rhombus r = 5 + k (south): (U_k+1, L_k, S, L_k+1);
  * lattice (a, b) in [0, M]^2, M = 2^g, T = (0,0), Lf = (M,0), R = (0,M),
    B = (M,M); every level bisects the three edge directions;
  * canonical id: rhombus r owns a in [1, M], b in [0, M-1],
    id = r M^2 + (a-1) M + b; north pole 10 M^2, south pole 10 M^2 + 1;
  * neighbours of p: counter-clockwise cycle starting at the smallest id;
    pentagons pad slot 6 with -1;
  * spring dynamics: tangent unit vectors, symplectic Euler, synchronous
    update of the hexagon points, stop when every point moved < tol;
  * spring constant k = 100 (the paper gives none; with k = 1 the stopping
    rule holds after the first step and nothing is relaxed);
  * centroid of a spherical polygon: nrm(sum_i nhat_i * theta_i) with theta_i
    the arc angle of edge i (the paper's printed arctangent is the
    complementary angle; the 1/(2 pi) factor vanishes in the normalisation);
  * control-volume corners = centroids of the triangles; cell point moved
    once to the centroid of its control volume (modified grid only).
"""
import math

import numpy as np


def nrm(x):
    """Unit vector(s) along the last axis."""
    return x / np.sqrt(np.sum(x * x, axis=-1, keepdims=True))


# ---------------------------------------------------------------------------
# Eq. grid_qts
# ---------------------------------------------------------------------------
def n_vertices(g):
    """Number of grid points per layer, N = 2 + 10 * 2^(2 g) (Eq. grid_qts)."""
    return 2 + 10 * 2 ** (2 * g)


def mean_spacing(g, radius):
    """Average grid spacing dbar = sqrt(2 pi / 5) A / 2^g (Eq. grid_qts)."""
    return np.sqrt(2.0 * np.pi / 5.0) * radius / 2.0 ** g


def mean_angle(g):
    """Average angular resolution thetabar = sqrt(2 pi / 5) / 2^g (Eq. grid_qts)."""
    return np.sqrt(2.0 * np.pi / 5.0) / 2.0 ** g


# ---------------------------------------------------------------------------
# Sec. 2.1: icosahedron and its ten rhombi
# ---------------------------------------------------------------------------
def icosahedron():
    """Twelve vertices: N, S, upper ring U[0..4], lower ring L[0..4]."""
    lat = np.arctan(0.5)
    north = np.array([0.0, 0.0, 1.0])
    south = np.array([0.0, 0.0, -1.0])
    upper = np.array([[np.cos(lat) * np.cos(2 * np.pi * k / 5),
                       np.cos(lat) * np.sin(2 * np.pi * k / 5),
                       np.sin(lat)] for k in range(5)])
    lower = np.array([[np.cos(lat) * np.cos(2 * np.pi * k / 5 + np.pi / 5),
                       np.cos(lat) * np.sin(2 * np.pi * k / 5 + np.pi / 5),
                       -np.sin(lat)] for k in range(5)])
    return north, south, upper, lower


def rhombus_corners(r):
    """Corners (T, Lf, B, R) of rhombus r; triangles (T,Lf,R), (Lf,B,R) are CCW."""
    north, south, upper, lower = icosahedron()
    k = r % 5
    if r < 5:
        return north, upper[k], lower[k], upper[(k + 1) % 5]
    return upper[(k + 1) % 5], lower[k], south, lower[(k + 1) % 5]


def rhombus_lattice(r, g):
    """Point positions of rhombus r on its (M+1)^2 lattice by recursive bisection.

    Each level keeps the old points at even indices and puts the normalised
    mid-point of every lattice edge (directions (1,0), (0,1), (1,-1)) at the
    new odd indices, i.e. each triangle is split into four (Fig. icogrid).
    """
    T, Lf, B, R = rhombus_corners(r)
    pos = np.zeros((2, 2, 3))
    pos[0, 0], pos[1, 0], pos[0, 1], pos[1, 1] = T, Lf, R, B
    for _ in range(g):
        m = pos.shape[0] - 1
        new = np.zeros((2 * m + 1, 2 * m + 1, 3))
        new[0::2, 0::2] = pos
        new[1::2, 0::2] = nrm(pos[:-1, :] + pos[1:, :])
        new[0::2, 1::2] = nrm(pos[:, :-1] + pos[:, 1:])
        new[1::2, 1::2] = nrm(pos[1:, :-1] + pos[:-1, 1:])
        pos = new
    return pos


def canonical_id(r, a, b, M):
    """Canonical id of lattice point (a, b) of rhombus r (integer rules only)."""
    while True:
        north = r < 5
        k = r % 5
        if north and a == 0 and b == 0:
            return 10 * M * M
        if (not north) and a == M and b == M:
            return 10 * M * M + 1
        if a == 0:
            if north:
                r, a, b = (k + 1) % 5, b, 0
            else:
                r, a, b = (k + 1) % 5, M, b
            continue
        if b == M:
            if north:
                r, a, b = 5 + k, a, 0
            else:
                r, a, b = 5 + (k + 1) % 5, M, a
            continue
        return r * M * M + (a - 1) * M + b


def id_table(g):
    """ids[r, a, b] for every lattice point of every rhombus."""
    M = 2 ** g
    ids = np.zeros((10, M + 1, M + 1), dtype=np.int64)
    for r in range(10):
        for a in range(M + 1):
            for b in range(M + 1):
                ids[r, a, b] = canonical_id(r, a, b, M)
    return ids


def triangles(g, ids=None):
    """All 20 * 4^g triangles (p, q, s), counter-clockwise seen from outside."""
    M = 2 ** g
    if ids is None:
        ids = id_table(g)
    tri = np.zeros((10, M, M, 2, 3), dtype=np.int64)
    a = np.arange(M)[:, None]
    b = np.arange(M)[None, :]
    for r in range(10):
        tri[r, :, :, 0, 0] = ids[r, a, b]
        tri[r, :, :, 0, 1] = ids[r, a + 1, b]
        tri[r, :, :, 0, 2] = ids[r, a, b + 1]
        tri[r, :, :, 1, 0] = ids[r, a + 1, b]
        tri[r, :, :, 1, 1] = ids[r, a + 1, b + 1]
        tri[r, :, :, 1, 2] = ids[r, a, b + 1]
    return tri.reshape(-1, 3)


def neighbour_table(tri, n):
    """CCW neighbour cycles starting at the smallest neighbour id; pad -1.

    From each CCW triangle (p, q, s): succ_p(q) = s, succ_q(s) = p,
    succ_s(p) = q.
    """
    centre = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    frm = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    to = np.concatenate([tri[:, 2], tri[:, 0], tri[:, 1]])
    key = centre * n + frm
    order = np.argsort(key)
    key, to_sorted = key[order], to[order]
    deg = np.bincount(centre, minlength=n)
    start = np.full(n, np.iinfo(np.int64).max)
    np.minimum.at(start, centre, frm)
    nbr = np.full((n, 6), -1, dtype=np.int64)
    cur = start.copy()
    cells = np.arange(n)
    for k in range(6):
        nbr[:, k] = cur
        idx = np.searchsorted(key, cells * n + cur)
        cur = to_sorted[idx]
    nbr[deg == 5, 5] = -1
    return nbr, deg


def positions(g):
    """Unit-sphere positions of the canonical points (standard grid)."""
    M = 2 ** g
    n = n_vertices(g)
    pts = np.zeros((n, 3))
    for r in range(10):
        lat = rhombus_lattice(r, g)
        for a in range(1, M + 1):
            for b in range(M):
                pts[r * M * M + (a - 1) * M + b] = lat[a, b]
    north, south, _, _ = icosahedron()
    pts[10 * M * M] = north
    pts[10 * M * M + 1] = south
    return pts


# ---------------------------------------------------------------------------
# Sec. 2.2: spring dynamics (Eqs. spring_force, spr_vel, dbar)
# ---------------------------------------------------------------------------
_SCALAR_ATAN2 = np.frompyfunc(math.atan2, 2, 1)


def libm_atan2(y, x):
    """Elementwise atan2 of the C library (one scalar call per element).
    NumPy's vectorised atan2 can differ from it in the last bit; a grid built
    with this one is bit-identical to a builder that calls the C library."""
    return _SCALAR_ATAN2(y, x).astype(np.float64)


def arc(a, b, atan2=np.arctan2):
    """Geodesic arc angle between unit vectors (last axis)."""
    c = np.cross(a, b)
    return atan2(np.sqrt(np.sum(c * c, axis=-1)), np.sum(a * b, axis=-1))


def spring_dynamics(P, nbr, deg, g, k=100.0, beta=1.15, alpha=1.0, dt=0.01,
                    tol=1e-5, max_iter=100000, atan2=np.arctan2):
    """Relax the hexagon points with damped springs; pentagons stay fixed.

    dv/dt = sum_i k (d_i - dbar_spr) e_i - alpha v,  dP/dt = v, with natural
    length dbar_spr = beta 2 pi / (10 2^(g-1)) on the unit sphere.  Symplectic
    Euler in time; the velocity is kept tangent and the point renormalised.
    Returns (P, iterations, converged).
    """
    P = P.copy()
    moving = np.nonzero(deg == 6)[0]
    nb = nbr[moving]
    dbar = beta * 2.0 * np.pi / (10.0 * 2.0 ** (g - 1))
    v = np.zeros((len(moving), 3))
    for it in range(1, max_iter + 1):
        p0 = P[moving]
        pi = P[nb]
        d = arc(p0[:, None, :], pi, atan2)
        dot = np.sum(p0[:, None, :] * pi, axis=-1)
        e = nrm(pi - dot[..., None] * p0[:, None, :])
        force = np.sum(k * (d - dbar)[..., None] * e, axis=1)
        v = v + dt * (force - alpha * v)
        v = v - np.sum(v * p0, axis=-1, keepdims=True) * p0
        pnew = nrm(p0 + dt * v)
        move = np.sqrt(np.max(np.sum((pnew - p0) ** 2, axis=-1)))
        P[moving] = pnew
        if move < tol:
            return P, it, True
    return P, max_iter, False


# ---------------------------------------------------------------------------
# Centroid equation (Sec. 2.2) and spherical triangle areas
# ---------------------------------------------------------------------------
def polygon_centroid(verts, atan2=np.arctan2):
    """Centroid direction of spherical polygon(s) verts[..., n, 3] (CCW)."""
    nxt = np.roll(verts, -1, axis=-2)
    c = np.cross(verts, nxt)
    cn = np.sqrt(np.sum(c * c, axis=-1))
    theta = atan2(cn, np.sum(verts * nxt, axis=-1))
    return nrm(np.sum(c / cn[..., None] * theta[..., None], axis=-2))


def tri_area(a, b, c, atan2=np.arctan2):
    """Spherical triangle area (Van Oosterom and Strackee)."""
    num = np.abs(np.sum(a * np.cross(b, c), axis=-1))
    den = 1.0 + np.sum(a * b, axis=-1) + np.sum(b * c, axis=-1) + np.sum(c * a, axis=-1)
    return 2.0 * atan2(num, den)


class Grid:
    """Grid of one glevel: topology, positions and control-volume geometry.

    Attributes (unit sphere)
      n, nbr[n,6], deg[n], tri[T,3], P[n,3]     points and topology
      C[n,6,3]     control-volume corners (triangle centroids), CCW
      w[n,6,3]     Eq. int_grid weights (w0, wk, wk1) of each corner
      l[n,6], nh[n,6,3]   arc length and outward normal of edge C_k -> C_k+1
      Ac[n], Sc[n,3]      control-volume area and sum_k l_k nhat_k
      tC[T,3], tA[T], tl[T,3], tn[T,3,3], tw[T,3]
                   triangle centroid, area, edge lengths/normals (edge e goes
                   from vertex e to vertex e+1) and corner weights of its
                   three vertices
      corner_tri[n,6]  index of the triangle at corner k of each cell
    """

    def __init__(self, g, smooth=True, k=100.0, beta=1.15, alpha=1.0, dt=0.01,
                 tol=1e-5, max_iter=100000, scalar_atan2=False):
        """scalar_atan2: take every arc angle and area with the C library's
        atan2 (``libm_atan2``) instead of NumPy's vectorised one."""
        self.g = g
        at = libm_atan2 if scalar_atan2 else np.arctan2
        self._atan2 = at
        self.n = n_vertices(g)
        ids = id_table(g)
        self.tri = triangles(g, ids)
        self.nbr, self.deg = neighbour_table(self.tri, self.n)
        P = positions(g)
        self.spring_iters, self.converged = 0, True
        if smooth and g > 0:
            P, self.spring_iters, self.converged = spring_dynamics(
                P, self.nbr, self.deg, g, k, beta, alpha, dt, tol, max_iter, at)
        # Triangle centroids become the control-volume corners.
        tC = polygon_centroid(P[self.tri], at)
        self._corner_map()
        if smooth:
            # Move each point once to the centroid of its control volume.
            C = self._corners(tC)
            newP = np.empty_like(P)
            for d in (5, 6):
                sel = self.deg == d
                newP[sel] = polygon_centroid(C[sel, :d], at)
            P = newP
        self.P = P
        self.tC = tC
        self._geometry()

    def _corner_map(self):
        """corner_tri[i, k]: triangle (i, nbr_k, nbr_k+1)."""
        n = self.n
        tri = self.tri
        key_of = {}
        for t in range(len(tri)):
            p, q, s = tri[t]
            key_of[(p, q)] = t
            key_of[(q, s)] = t
            key_of[(s, p)] = t
        ct = np.full((n, 6), -1, dtype=np.int64)
        for i in range(n):
            d = self.deg[i]
            for kk in range(d):
                ct[i, kk] = key_of[(i, self.nbr[i, kk])]
        self.corner_tri = ct

    def _corners(self, tC):
        C = tC[self.corner_tri]
        C[self.deg == 5, 5] = 0.0
        return C

    def _geometry(self):
        at = self._atan2
        n = self.n
        P, tri = self.P, self.tri
        C = self._corners(self.tC)
        self.C = C
        self.w = np.zeros((n, 6, 3))
        self.l = np.zeros((n, 6))
        self.nh = np.zeros((n, 6, 3))
        self.Ac = np.zeros(n)
        for d in (5, 6):
            sel = np.nonzero(self.deg == d)[0]
            p0 = P[sel][:, None, :]
            nk = self.nbr[sel, :d]
            pk = P[nk]
            pk1 = P[np.roll(nk, -1, axis=1)]
            ck = C[sel, :d]
            ck1 = np.roll(ck, -1, axis=1)
            # Eq. int_grid: A1 (P0,Pk,Ck), A2 (Pk,Pk+1,Ck), A3 (P0,Pk+1,Ck)
            A1 = tri_area(p0, pk, ck, at)
            A2 = tri_area(pk, pk1, ck, at)
            A3 = tri_area(p0, pk1, ck, at)
            tot = A1 + A2 + A3
            self.w[sel, :d, 0] = A2 / tot
            self.w[sel, :d, 1] = A3 / tot
            self.w[sel, :d, 2] = A1 / tot
            self.l[sel, :d] = arc(ck, ck1, at)
            self.nh[sel, :d] = nrm(np.cross(ck1, ck))
            self.Ac[sel] = np.sum(tri_area(p0, ck, ck1, at), axis=1)
        self.Sc = np.sum(self.l[..., None] * self.nh, axis=1)
        # Primal triangles, for the Laplacian (Sec. 4).
        a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
        self.tA = tri_area(a, b, c, at)
        vs = np.stack([a, b, c], axis=1)
        ve = np.roll(vs, -1, axis=1)
        self.tl = arc(vs, ve, at)
        self.tn = nrm(np.cross(ve, vs))
        # Barycentric corner weights of the triangle centroid for its three
        # vertices: each weight is the sub-area opposite that vertex.
        ct = self.tC
        wa = tri_area(b, c, ct, at)
        wb = tri_area(c, a, ct, at)
        wc = tri_area(a, b, ct, at)
        tot = wa + wb + wc
        self.tw = np.stack([wa / tot, wb / tot, wc / tot], axis=1)
