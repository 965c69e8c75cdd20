// Host construction of the icosahedral grid and its finite-volume operator
// coefficients (Sec. 2.1-2.2 of Mendonca et al. 2016).
//
//  * icosahedron with vertices at the poles; upper ring at latitude
//    atan(1/2), longitudes 2 pi k/5; lower ring at -atan(1/2), shifted pi/5;
//  * ten rhombi, each refined by recursive edge bisection (Fig. icogrid);
//  * canonical column ids and counter-clockwise neighbour cycles;
//  * spring dynamics (Eqs. spring_force, spr_vel, dbar) on the hexagon points;
//  * control-volume corners at the triangle centroids, cell points moved once
//    to the control-volume centroids (centroid equation, arc-angle form);
//  * Eq. int_grid corner weights, Eqs. flx_div / div_gauss / grad folded into
//    per-column coefficient vectors, and the triangle-gradient Laplacian of
//    Sec. 4 folded into per-column neighbour weights.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace thor {
namespace {

inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline Vec3 cross(Vec3 a, Vec3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(Vec3 a) { return std::sqrt(dot(a, a)); }
inline Vec3 unit(Vec3 a) {
  double n = norm(a);
  return {a.x / n, a.y / n, a.z / n};
}

// Great-circle angle between unit vectors.
inline double arc_angle(Vec3 a, Vec3 b) { return std::atan2(norm(cross(a, b)), dot(a, b)); }

// Spherical triangle area (Van Oosterom and Strackee 1983).
inline double sph_area(Vec3 a, Vec3 b, Vec3 c) {
  double num = std::fabs(dot(a, cross(b, c)));
  double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
  return 2.0 * std::atan2(num, den);
}

// Centroid direction of a counter-clockwise spherical polygon: the area
// integral of r equals half the sum of edge-plane normals times arc angles.
Vec3 sph_centroid(const Vec3 *v, int n) {
  Vec3 s{0, 0, 0};
  for (int i = 0; i < n; ++i) {
    Vec3 a = v[i], b = v[(i + 1) % n];
    Vec3 c = cross(a, b);
    double cn = norm(c);
    double th = std::atan2(cn, dot(a, b));
    Vec3 nc{c.x / cn, c.y / cn, c.z / cn};
    s = s + th * nc;
  }
  return unit(s);
}

struct Ico {
  Vec3 north, south, up[5], lo[5];
};

Ico make_icosahedron() {
  Ico I;
  const double lat = std::atan(0.5);
  const double pi = M_PI;
  I.north = {0, 0, 1};
  I.south = {0, 0, -1};
  for (int k = 0; k < 5; ++k) {
    double lu = 2 * pi * k / 5, ll = 2 * pi * k / 5 + pi / 5;
    I.up[k] = {std::cos(lat) * std::cos(lu), std::cos(lat) * std::sin(lu), std::sin(lat)};
    I.lo[k] = {std::cos(lat) * std::cos(ll), std::cos(lat) * std::sin(ll), -std::sin(lat)};
  }
  return I;
}

// Rhombus r corners in the order top, left, bottom, right; lattice (a, b) has
// top (0,0), left (M,0), right (0,M), bottom (M,M).
std::array<Vec3, 4> rhombus(const Ico &I, int r) {
  int k = r % 5, k1 = (k + 1) % 5;
  if (r < 5) return {I.north, I.up[k], I.lo[k], I.up[k1]};
  return {I.up[k1], I.lo[k], I.south, I.lo[k1]};
}

// Lattice of one rhombus after `levels` bisections, row-major [(M+1)^2].
std::vector<Vec3> bisect_lattice(const std::array<Vec3, 4> &c, int levels) {
  int m = 1;
  std::vector<Vec3> cur = {c[0], c[3], c[1], c[2]};  // (0,0) (0,1) (1,0) (1,1)
  for (int l = 0; l < levels; ++l) {
    int m2 = 2 * m, w = m + 1, w2 = m2 + 1;
    std::vector<Vec3> nxt((size_t)w2 * w2);
    auto O = [&](int a, int b) -> const Vec3 & { return cur[(size_t)a * w + b]; };
    for (int a = 0; a <= m; ++a)
      for (int b = 0; b <= m; ++b) nxt[(size_t)(2 * a) * w2 + 2 * b] = O(a, b);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b <= m; ++b) nxt[(size_t)(2 * a + 1) * w2 + 2 * b] = unit(O(a, b) + O(a + 1, b));
    for (int a = 0; a <= m; ++a)
      for (int b = 0; b < m; ++b) nxt[(size_t)(2 * a) * w2 + 2 * b + 1] = unit(O(a, b) + O(a, b + 1));
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b)
        nxt[(size_t)(2 * a + 1) * w2 + 2 * b + 1] = unit(O(a + 1, b) + O(a, b + 1));
    cur.swap(nxt);
    m = m2;
  }
  return cur;
}

// Canonical id of lattice point (a, b) of rhombus r, following points on the
// unowned edges (a = 0, b = M) into the rhombus that owns them.
int64_t point_id(int r, int a, int b, int M) {
  const int64_t MM = (int64_t)M * M;
  for (;;) {
    bool north = r < 5;
    int k = r % 5, k1 = (k + 1) % 5;
    if (north && a == 0 && b == 0) return 10 * MM;
    if (!north && a == M && b == M) return 10 * MM + 1;
    if (a == 0) {
      if (north) { r = k1; a = b; b = 0; }
      else { r = k1; a = M; }
      continue;
    }
    if (b == M) {
      if (north) { r = 5 + k; b = 0; }
      else { r = 5 + k1; b = a; a = M; }
      continue;
    }
    return r * MM + (int64_t)(a - 1) * M + b;
  }
}

}  // namespace

int build_grid(const thor_grid_params &p, Grid &G) {
  const int g = p.glevel;
  const int M = 1 << g;
  const int64_t n = 10LL * M * M + 2;
  G.glevel = g;
  G.smooth = p.smooth;
  G.n = n;
  const Ico I = make_icosahedron();

  // Points and triangles from the ten rhombus lattices.
  std::vector<Vec3> P(n);
  std::vector<std::array<int64_t, 3>> tris;
  tris.reserve((size_t)20 * M * M);
  for (int r = 0; r < 10; ++r) {
    std::vector<Vec3> lat = bisect_lattice(rhombus(I, r), g);
    const int w = M + 1;
    std::vector<int64_t> id((size_t)w * w);
    for (int a = 0; a <= M; ++a)
      for (int b = 0; b <= M; ++b) id[(size_t)a * w + b] = point_id(r, a, b, M);
    for (int a = 1; a <= M; ++a)
      for (int b = 0; b < M; ++b) P[id[(size_t)a * w + b]] = lat[(size_t)a * w + b];
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b) {
        int64_t p00 = id[(size_t)a * w + b], p10 = id[(size_t)(a + 1) * w + b];
        int64_t p01 = id[(size_t)a * w + b + 1], p11 = id[(size_t)(a + 1) * w + b + 1];
        tris.push_back({p00, p10, p01});
        tris.push_back({p10, p11, p01});
      }
  }
  P[10LL * M * M] = I.north;
  P[10LL * M * M + 1] = I.south;

  // Around each point, every counter-clockwise triangle (p, q, s) says that
  // s follows q.  Chain the successors from the smallest neighbour id.
  std::vector<std::array<int64_t, 6>> from(n), to(n);
  std::vector<int> cnt(n, 0);
  auto add = [&](int64_t c, int64_t f, int64_t t) {
    int i = cnt[c]++;
    from[c][i] = f;
    to[c][i] = t;
  };
  for (auto &t : tris) {
    add(t[0], t[1], t[2]);
    add(t[1], t[2], t[0]);
    add(t[2], t[0], t[1]);
  }
  G.nbr.assign((size_t)n * 6, -1);
  G.deg.assign(n, 0);
  for (int64_t c = 0; c < n; ++c) {
    int d = cnt[c];
    G.deg[c] = (uint8_t)d;
    int64_t cur = *std::min_element(from[c].begin(), from[c].begin() + d);
    for (int k = 0; k < d; ++k) {
      G.nbr[(size_t)c * 6 + k] = (int32_t)cur;
      int j = 0;
      while (from[c][j] != cur) ++j;
      cur = to[c][j];
    }
  }

  // Spring dynamics on the hexagon points (pentagon points stay fixed).
  G.spring_iters = 0;
  G.converged = true;
  G.first_force = 0.0;
  if (p.smooth && g > 0) {
    const double dspr = p.beta * 2.0 * M_PI / (10.0 * std::ldexp(1.0, g - 1));
    std::vector<int64_t> mov;
    for (int64_t c = 0; c < n; ++c)
      if (G.deg[c] == 6) mov.push_back(c);
    std::vector<Vec3> vel(mov.size(), Vec3{0, 0, 0}), nxt(mov.size());
    G.converged = false;
    // Every point's update reads only the previous positions, so the points
    // are split over host threads; the result does not depend on the split.
    const size_t nm = mov.size();
    const int nt = (int)std::max<size_t>(1, std::min<size_t>({(size_t)std::thread::hardware_concurrency(),
                                                               (size_t)16, nm / 4096 + 1}));
    std::vector<double> part(nt), pforce(nt);
    auto sweep = [&](int t) {
      const size_t lo = nm * t / nt, hi = nm * (t + 1) / nt;
      double mm = 0.0, ff = 0.0;
      for (size_t m = lo; m < hi; ++m) {
        const Vec3 p0 = P[mov[m]];
        Vec3 F{0, 0, 0};
        for (int k = 0; k < 6; ++k) {
          const Vec3 pk = P[G.nbr[(size_t)mov[m] * 6 + k]];
          double d = arc_angle(p0, pk);
          Vec3 e = unit(pk - dot(p0, pk) * p0);
          F = F + (p.k * (d - dspr)) * e;
        }
        ff = std::max(ff, dot(F, F));
        Vec3 v = vel[m] + p.dt * (F - p.alpha * vel[m]);
        v = v - dot(v, p0) * p0;
        vel[m] = v;
        Vec3 q = unit(p0 + p.dt * v);
        Vec3 dq = q - p0;
        mm = std::max(mm, dot(dq, dq));
        nxt[m] = q;
      }
      part[t] = mm;
      pforce[t] = ff;
    };
    for (int it = 1; it <= p.max_iter; ++it) {
      if (nt == 1) {
        sweep(0);
      } else {
        std::vector<std::thread> pool;
        for (int t = 1; t < nt; ++t) pool.emplace_back(sweep, t);
        sweep(0);
        for (auto &th : pool) th.join();
      }
      double maxmove2 = 0.0;
      for (double v : part) maxmove2 = std::max(maxmove2, v);
      if (it == 1) {
        double f2 = 0.0;
        for (double v : pforce) f2 = std::max(f2, v);
        // largest spring force of the first step relative to k times the
        // natural length: ~1e-16 for points already in equilibrium
        G.first_force = std::sqrt(f2) / (p.k * dspr);
      }
      for (size_t m = 0; m < nm; ++m) P[mov[m]] = nxt[m];
      G.spring_iters = it;
      if (std::sqrt(maxmove2) < p.tol) {
        G.converged = true;
        break;
      }
    }
  }

  // Triangle centroids become the control-volume corners; corner k of cell
  // c is the triangle (c, nbr_k, nbr_k+1).
  const size_t T = tris.size();
  std::vector<Vec3> tc(T);
  for (size_t t = 0; t < T; ++t) {
    Vec3 v[3] = {P[tris[t][0]], P[tris[t][1]], P[tris[t][2]]};
    tc[t] = sph_centroid(v, 3);
  }
  // corner triangle lookup: the triangle whose directed edge (c -> nbr_k) is
  // followed by nbr_k+1 around c.
  std::vector<std::array<int64_t, 6>> ctri(n);
  std::vector<std::array<int, 6>> cslot(n);   // position of c inside that triangle
  for (size_t t = 0; t < T; ++t)
    for (int v = 0; v < 3; ++v) {
      int64_t c = tris[t][v], q = tris[t][(v + 1) % 3];
      int d = G.deg[c];
      for (int k = 0; k < d; ++k)
        if (G.nbr[(size_t)c * 6 + k] == q) {
          ctri[c][k] = (int64_t)t;
          cslot[c][k] = v;
        }
    }
  if (p.smooth) {
    std::vector<Vec3> Pn(n);
    for (int64_t c = 0; c < n; ++c) {
      Vec3 cv[6];
      int d = G.deg[c];
      for (int k = 0; k < d; ++k) cv[k] = tc[ctri[c][k]];
      Pn[c] = sph_centroid(cv, d);
    }
    P.swap(Pn);
  }
  G.pos = P;

  // Per-triangle primal gradient weights (Eq. grad on a triangle): the
  // gradient at the corner is sum_v bt[t][v] * s_v (unit sphere).
  std::vector<std::array<Vec3, 3>> bt(T);
  for (size_t t = 0; t < T; ++t) {
    Vec3 v[3] = {P[tris[t][0]], P[tris[t][1]], P[tris[t][2]]};
    double At = sph_area(v[0], v[1], v[2]);
    Vec3 ln[3];   // l_e n_e of edge e: v[e] -> v[e+1], outward
    Vec3 S{0, 0, 0};
    for (int e = 0; e < 3; ++e) {
      Vec3 a = v[e], b = v[(e + 1) % 3];
      ln[e] = arc_angle(a, b) * unit(cross(b, a));
      S = S + ln[e];
    }
    // centroid value by area weights of the sub-triangles opposite each vertex
    double wa = sph_area(v[1], v[2], tc[t]);
    double wb = sph_area(v[2], v[0], tc[t]);
    double wc = sph_area(v[0], v[1], tc[t]);
    double ws = wa + wb + wc;
    double tw[3] = {wa / ws, wb / ws, wc / ws};
    for (int i = 0; i < 3; ++i) {
      Vec3 s = 0.5 * (ln[i] + ln[(i + 2) % 3]) - tw[i] * S;
      bt[t][i] = (1.0 / At) * s;
    }
  }

  // Control-volume geometry and folded operator coefficients.
  G.area.assign(n, 0.0);
  G.div_coef.assign((size_t)n * 21, 0.0);
  G.lap_coef.assign((size_t)n * 6, 0.0);
  for (int64_t c = 0; c < n; ++c) {
    const int d = G.deg[c];
    const int32_t *nb = &G.nbr[(size_t)c * 6];
    const Vec3 p0 = P[c];
    Vec3 C[6];
    for (int k = 0; k < d; ++k) C[k] = tc[ctri[c][k]];
    double Ac = 0.0;
    Vec3 ln[6];
    double w0[6], wk[6], wk1[6];
    for (int k = 0; k < d; ++k) {
      int k1 = (k + 1) % d;
      Vec3 pk = P[nb[k]], pk1 = P[nb[k1]];
      Ac += sph_area(p0, C[k], C[k1]);
      ln[k] = arc_angle(C[k], C[k1]) * unit(cross(C[k1], C[k]));
      // Eq. int_grid: A1 (P0,Pk,Ck), A2 (Pk,Pk+1,Ck), A3 (P0,Pk+1,Ck)
      double A1 = sph_area(p0, pk, C[k]);
      double A2 = sph_area(pk, pk1, C[k]);
      double A3 = sph_area(p0, pk1, C[k]);
      double As = A1 + A2 + A3;
      w0[k] = A2 / As;
      wk[k] = A3 / As;
      wk1[k] = A1 / As;
    }
    G.area[c] = Ac;
    // h_k: weight of the corner-k value in the Gauss sum (edges k-1 and k)
    Vec3 h[6];
    for (int k = 0; k < d; ++k) h[k] = (0.5 / Ac) * (ln[k] + ln[(k + d - 1) % d]);
    double *dc = &G.div_coef[(size_t)c * 21];
    Vec3 e0{0, 0, 0};
    for (int k = 0; k < d; ++k) e0 = e0 + w0[k] * h[k];
    dc[0] = e0.x; dc[1] = e0.y; dc[2] = e0.z;
    for (int j = 0; j < d; ++j) {
      int jm = (j + d - 1) % d;
      Vec3 ej = wk[j] * h[j] + wk1[jm] * h[jm];
      dc[3 * (j + 1) + 0] = ej.x;
      dc[3 * (j + 1) + 1] = ej.y;
      dc[3 * (j + 1) + 2] = ej.z;
    }
    // Laplacian: sum_k h_k . G_k, G_k = triangle gradient at corner k.
    double *lc = &G.lap_coef[(size_t)c * 6];
    for (int j = 0; j < d; ++j) {
      int jm = (j + d - 1) % d;
      // neighbour j is vertex (slot+1) of corner-j triangle and vertex
      // (slot+2) of the corner-(j-1) triangle
      const auto &bj = bt[ctri[c][j]];
      const auto &bm = bt[ctri[c][jm]];
      lc[j] = dot(h[j], bj[(cslot[c][j] + 1) % 3]) + dot(h[jm], bm[(cslot[c][jm] + 2) % 3]);
    }
  }
  // Divergence damping acts as lap(grad D): fold the two stencils into one
  // over the two-ring of each column (at most 18 other columns):
  //   lap(grad D)(c) = (1/r^3) sum_m w_m (D_m - D_c).
  G.dd_idx.assign((size_t)n * kRing2, -1);
  G.dd_w.assign((size_t)n * kRing2 * 3, 0.0);
  for (int64_t c = 0; c < n; ++c) {
    int32_t *idx = &G.dd_idx[(size_t)c * kRing2];
    double *wv = &G.dd_w[(size_t)c * kRing2 * 3];
    int cnt = 0;
    auto slot = [&](int64_t m) -> int {
      for (int q = 0; q < cnt; ++q)
        if (idx[q] == m) return q;
      idx[cnt] = (int32_t)m;
      return cnt++;
    };
    // weight of D_m in G(y) = sum_i e^y_i (D(n^y_i) - D(y)), scaled by s
    auto add_grad = [&](int64_t y, double s) {
      const double *dc = &G.div_coef[(size_t)y * 21];
      for (int i = 0; i < G.deg[y]; ++i) {
        const int64_t m = G.nbr[(size_t)y * 6 + i];
        const double *e = dc + 3 * (i + 1);
        if (m != c) {
          const int q = slot(m);
          for (int k = 0; k < 3; ++k) wv[3 * q + k] += s * e[k];
        }
        if (y != c) {
          const int q = slot(y);
          for (int k = 0; k < 3; ++k) wv[3 * q + k] -= s * e[k];
        }
      }
    };
    const double *lc = &G.lap_coef[(size_t)c * 6];
    for (int j = 0; j < G.deg[c]; ++j) add_grad(G.nbr[(size_t)c * 6 + j], lc[j]);
    double lsum = 0.0;
    for (int j = 0; j < G.deg[c]; ++j) lsum += lc[j];
    add_grad(c, -lsum);
    if (cnt > kRing2) return THOR_EINVAL;
  }
  return THOR_OK;
}

}  // namespace thor

extern "C" {

void thor_grid_params_default(int glevel, thor_grid_params *p) {
  if (!p) return;
  p->glevel = glevel;
  p->smooth = 1;
  p->k = 100.0;
  p->beta = 1.15;
  p->alpha = 1.0;
  p->dt = 0.01;
  p->tol = 1e-5;
  p->max_iter = 100000;
}

int thor_grid_build(const thor_grid_params *p, thor_grid **out) {
  thor::clear_error();
  if (!p || !out) { thor::set_error("thor_grid_build: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  if (p->glevel < 0 || p->glevel > 8) { thor::set_error("thor_grid_build: glevel must be 0..8"); return THOR_EINVAL; }
  if (p->smooth != 0 && p->smooth != 1) { thor::set_error("thor_grid_build: smooth must be 0 or 1"); return THOR_EINVAL; }
  if (p->smooth && !(p->k > 0 && p->beta > 0 && p->alpha >= 0 && p->dt > 0 && p->tol > 0 && p->max_iter > 0)) {
    thor::set_error("thor_grid_build: spring parameters must be positive");
    return THOR_EINVAL;
  }
  thor_grid *g = new (std::nothrow) thor_grid;
  if (!g) { thor::set_error("thor_grid_build: out of host memory"); return THOR_ENOMEM; }
  try {
    if (thor::build_grid(*p, g->g) != THOR_OK) {
      delete g;
      thor::set_error("thor_grid_build: two-ring stencil larger than expected");
      return THOR_EINVAL;
    }
  } catch (const std::bad_alloc &) {
    delete g;
    thor::set_error("thor_grid_build: out of host memory");
    return THOR_ENOMEM;
  }
  *out = g;
  if (!g->g.converged) {
    thor::set_error("thor_grid_build: spring dynamics reached max_iter");
    return THOR_ENOTCONV;
  }
  if (p->smooth && p->glevel > 0 && g->g.spring_iters <= 1 && g->g.first_force > 1e-9) {
    thor::set_error("thor_grid_build: spring dynamics stopped after its first step (every point moved less than "
                    "tol) with the points out of equilibrium; no point was relaxed, a larger k relaxes this grid");
    return THOR_ENOTSMOOTH;
  }
  return THOR_OK;
}

int thor_grid_info(const thor_grid *g, int64_t *n_col, int *n_pent, int *spring_iters) {
  thor::clear_error();
  if (!g) { thor::set_error("thor_grid_info: NULL grid"); return THOR_EINVAL; }
  if (n_col) *n_col = g->g.n;
  if (n_pent) {
    int c = 0;
    for (auto d : g->g.deg) c += (d == 5);
    *n_pent = c;
  }
  if (spring_iters) *spring_iters = g->g.spring_iters;
  return THOR_OK;
}

int thor_grid_export(const thor_grid *g, int32_t *nbr, double *xyz, double *area) {
  thor::clear_error();
  if (!g) { thor::set_error("thor_grid_export: NULL grid"); return THOR_EINVAL; }
  const auto &G = g->g;
  if (nbr) std::copy(G.nbr.begin(), G.nbr.end(), nbr);
  if (xyz)
    for (int64_t c = 0; c < G.n; ++c) {
      xyz[3 * c] = G.pos[c].x;
      xyz[3 * c + 1] = G.pos[c].y;
      xyz[3 * c + 2] = G.pos[c].z;
    }
  if (area) std::copy(G.area.begin(), G.area.end(), area);
  return THOR_OK;
}

int thor_grid_coefficients(const thor_grid *g, double *div_coef, double *lap_coef) {
  thor::clear_error();
  if (!g) { thor::set_error("thor_grid_coefficients: NULL grid"); return THOR_EINVAL; }
  if (div_coef) std::copy(g->g.div_coef.begin(), g->g.div_coef.end(), div_coef);
  if (lap_coef) std::copy(g->g.lap_coef.begin(), g->g.lap_coef.end(), lap_coef);
  return THOR_OK;
}

int thor_grid_damping_coefficients(const thor_grid *g, int32_t *idx, double *w) {
  thor::clear_error();
  if (!g) { thor::set_error("thor_grid_damping_coefficients: NULL grid"); return THOR_EINVAL; }
  if (idx) std::copy(g->g.dd_idx.begin(), g->g.dd_idx.end(), idx);
  if (w) std::copy(g->g.dd_w.begin(), g->g.dd_w.end(), w);
  return THOR_OK;
}

void thor_grid_free(thor_grid *g) { delete g; }

}  // extern "C"
