"""Pins of the oracle grid (Sec. 2.1-2.2) against closed forms, brute force
and invariants that the paper and spherical geometry fix."""
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import grid
from tests.conftest import oracle_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.mark.parametrize("g", range(0, 6))
def test_counts_and_euler_characteristic(g):
    """N = 2 + 10 * 4^g (Eq. grid_qts); 12 pentagons, hexagons elsewhere."""
    n = grid.n_vertices(g)
    assert n == 10 * 4 ** g + 2
    tri = grid.triangles(g)
    assert tri.shape == (20 * 4 ** g, 3)
    nbr, deg = grid.neighbour_table(tri, n)
    assert np.sum(deg == 5) == 12
    assert np.sum(deg == 6) == n - 12
    edges = {tuple(sorted(e)) for t in tri for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    assert len(edges) == 30 * 4 ** g
    assert n - len(edges) + len(tri) == 2
    # every undirected edge is in exactly two triangles, once per direction
    directed = {(t[i], t[(i + 1) % 3]) for t in tri for i in range(3)}
    assert len(directed) == 2 * len(edges)
    for a, b in list(directed)[:2000]:
        assert (b, a) in directed
    # neighbour cycles close and start at the smallest id
    for i in range(n):
        d = deg[i]
        row = nbr[i, :d]
        assert len(set(row)) == d and row[0] == row.min()
        if d == 5:
            assert nbr[i, 5] == -1


def test_paper_g5_point_count():
    gold = _golden("paper_constants.txt")
    assert grid.n_vertices(5) == int(gold["n_points_g5"])


@pytest.mark.parametrize("g", [0, 1, 3])
def test_triangles_counter_clockwise(g):
    G = oracle_grid(g, smooth=False)
    P = G.P
    t = G.tri
    det = np.einsum("ij,ij->i", P[t[:, 0]], np.cross(P[t[:, 1]], P[t[:, 2]]))
    assert det.min() > 0.0


def test_pentagons_sit_on_icosahedron_vertices():
    G = oracle_grid(4, smooth=False)
    north, south, upper, lower = grid.icosahedron()
    ico = np.vstack([north, south, upper, lower])
    pent = G.P[G.deg == 5]
    d = cKDTree(ico).query(pent)[0]
    assert d.max() < 1e-15


def _brute_force_points(g):
    """Independent construction: split the 20 faces recursively into four,
    projecting every edge mid-point onto the sphere, and dedupe."""
    north, south, upper, lower = grid.icosahedron()
    faces = []
    for k in range(5):
        k1 = (k + 1) % 5
        faces += [(north, upper[k], upper[k1]), (upper[k], lower[k], upper[k1]),
                  (upper[k1], lower[k], lower[k1]), (lower[k], south, lower[k1])]
    for _ in range(g):
        new = []
        for a, b, c in faces:
            ab = (a + b) / np.linalg.norm(a + b)
            bc = (b + c) / np.linalg.norm(b + c)
            ca = (c + a) / np.linalg.norm(c + a)
            new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        faces = new
    pts = np.array([v for f in faces for v in f])
    key = np.round(pts * 1e9).astype(np.int64)
    _, idx = np.unique(key, axis=0, return_index=True)
    return pts[idx]


@pytest.mark.parametrize("g", [2, 4])
def test_recursive_bisection_matches_brute_force(g):
    G = oracle_grid(g, smooth=False)
    ref = _brute_force_points(g)
    assert len(ref) == G.n
    d, _ = cKDTree(ref).query(G.P)
    assert d.max() < 1e-15
    assert np.allclose(np.linalg.norm(G.P, axis=1), 1.0, atol=1e-15)


@pytest.mark.parametrize("smooth,tol", [(False, 1e-14), (True, 1e-12)])
def test_72_degree_rotation_symmetry(smooth, tol):
    G = oracle_grid(4, smooth=smooth)
    c, s = np.cos(2 * np.pi / 5), np.sin(2 * np.pi / 5)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    d, _ = cKDTree(G.P).query(G.P @ R.T)
    assert d.max() < tol


@pytest.mark.parametrize("smooth", [False, True])
def test_area_sums_are_4pi(smooth):
    G = oracle_grid(4, smooth=smooth)
    assert abs(G.Ac.sum() - 4 * np.pi) < 1e-12
    assert abs(G.tA.sum() - 4 * np.pi) < 1e-12
    assert G.Ac.min() > 0


def test_interpolation_subareas_sum_to_triangle():
    """A1 + A2 + A3 of Eq. int_grid equals the area of (P0, Pk, Pk+1)."""
    G = oracle_grid(3, smooth=True)
    for i in range(0, G.n, 7):
        d = G.deg[i]
        for k in range(d):
            a, b = G.nbr[i, k], G.nbr[i, (k + 1) % d]
            p0, pk, pk1, ck = G.P[i], G.P[a], G.P[b], G.C[i, k]
            tot = (grid.tri_area(p0, pk, ck) + grid.tri_area(pk, pk1, ck)
                   + grid.tri_area(p0, pk1, ck))
            assert abs(tot - grid.tri_area(p0, pk, pk1)) < 1e-15
            assert abs(G.w[i, k].sum() - 1.0) < 1e-14 and G.w[i, k].min() > 0


def test_edges_shared_between_neighbours():
    """The edge between cells i and nbr_k is C_{k-1} -> C_k; both sides see
    the same length and opposite normals."""
    G = oracle_grid(3, smooth=True)
    for i in range(G.n):
        d = G.deg[i]
        for k in range(d):
            j = G.nbr[i, k]
            dj = G.deg[j]
            m = list(G.nbr[j, :dj]).index(i)
            ei, ej = (k - 1) % d, (m - 1) % dj
            assert abs(G.l[i, ei] - G.l[j, ej]) < 1e-15
            assert np.abs(G.nh[i, ei] + G.nh[j, ej]).max() < 1e-14


def _quad_centroid(verts, centre, levels=6):
    """Brute force int r dA over a simple spherical polygon: signed fan of
    triangles from ``centre``, each subdivided into 4^levels small triangles,
    midpoint rule."""
    total = np.zeros(3)
    n = len(verts)
    for k in range(n):
        faces = [(centre, verts[k], verts[(k + 1) % n])]
        for _ in range(levels):
            new = []
            for a, b, c in faces:
                ab, bc, ca = grid.nrm(a + b), grid.nrm(b + c), grid.nrm(c + a)
                new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
            faces = new
        f = np.array(faces)
        sign = np.sign(np.einsum("ij,ij->i", f[:, 0], np.cross(f[:, 1], f[:, 2])))
        area = sign * grid.tri_area(f[:, 0], f[:, 1], f[:, 2])
        mid = grid.nrm(f.sum(axis=1))
        total += np.sum(area[:, None] * mid, axis=0)
    return grid.nrm(total)


def test_centroid_formula_matches_quadrature():
    rs = np.random.default_rng(11)
    for n in (3, 5, 6):
        for _ in range(3):
            c = grid.nrm(rs.normal(size=3))
            t1 = grid.nrm(np.cross(c, rs.normal(size=3)))
            t2 = np.cross(c, t1)
            ang = np.sort(rs.uniform(0, 2 * np.pi, n))
            rad = rs.uniform(0.05, 0.15, n)
            verts = grid.nrm(c + rad[:, None] * (np.cos(ang)[:, None] * t1 + np.sin(ang)[:, None] * t2))
            got = grid.polygon_centroid(verts[None])[0]
            ref = _quad_centroid(verts, c)
            assert np.linalg.norm(got - ref) < 1e-8


def test_regular_polygon_centroid_is_its_centre():
    c = grid.nrm(np.array([0.3, -0.2, 0.9]))
    t1 = grid.nrm(np.cross(c, [1.0, 0, 0]))
    t2 = np.cross(c, t1)
    ang = 2 * np.pi * np.arange(6) / 6 + 0.1
    verts = grid.nrm(c + 0.1 * (np.cos(ang)[:, None] * t1 + np.sin(ang)[:, None] * t2))
    assert np.linalg.norm(grid.polygon_centroid(verts[None])[0] - c) < 1e-15


def test_spring_dynamics_stops_by_rule_and_keeps_pentagons():
    G0 = oracle_grid(4, smooth=False)
    P, it, ok = grid.spring_dynamics(G0.P, G0.nbr, G0.deg, 4, k=100.0)
    assert ok and 10 < it < 100000
    pent = G0.deg == 5
    assert np.array_equal(P[pent], G0.P[pent])
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0, atol=1e-14)


def test_mean_spacing_example_from_paper():
    gold = _golden("paper_constants.txt")
    dbar_km = grid.mean_spacing(5, 7.0e7) / 1e3
    assert abs(dbar_km - gold["dbar_jupiter_g5_km"]) < 1.0
    assert abs(np.degrees(grid.mean_angle(5)) - gold["thetabar_g5_deg"]) < 0.05


def test_spring_relaxation_approaches_a_force_balance():
    """Sec. 2.2: the relaxation drives each hexagon point toward a balance of
    its springs.  When the paper's rule stops it (steps < 1e-5) the largest
    net force is a few percent of a single spring's force; with a 100x
    tighter rule it falls by more than 100x.  The tangent direction is
    written here through cross products, (p0 x pk) x p0, independently of
    the oracle's projection."""
    G0 = oracle_grid(4, smooth=False)
    k = 100.0
    dbar = 1.15 * 2 * np.pi / (10 * 2 ** 3)
    hexes = np.flatnonzero(G0.deg == 6)

    def worst_net_force(tol):
        P, it, ok = grid.spring_dynamics(G0.P, G0.nbr, G0.deg, 4, k=k, tol=tol)
        assert ok
        net, single = [], []
        for c in hexes:
            p0 = P[c]
            F = np.zeros(3)
            for q in G0.nbr[c]:
                pk = P[q]
                t = np.cross(np.cross(p0, pk), p0)
                t /= np.linalg.norm(t)
                d = np.arctan2(np.linalg.norm(np.cross(p0, pk)), p0 @ pk)
                F += k * (d - dbar) * t
                single.append(abs(k * (d - dbar)))
            net.append(np.linalg.norm(F))
        return max(net) / np.median(single)

    loose, tight = worst_net_force(1e-5), worst_net_force(1e-7)
    assert loose < 0.05
    assert tight < loose / 100
