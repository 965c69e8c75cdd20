// HIP kernels of the HEVI dynamical-core step for gfx950 (MI355X).
//
// Paper: Mendonca et al. 2016 (arXiv:1607.05535), Sec. 2-5.
//
// Work mappings.  Column data is contiguous in memory ([col][lev]).
//  * Gather kernels (acoustic phase M, the gather half of phase V, slow
//    terms, per-large-step terms): a lane owns kHq = 4 consecutive levels of
//    one column, ceil(L / 4) lanes per column.  A neighbour row is read with
//    16-byte loads, per-column stencil weights are loaded once per 4 cells,
//    and a vertical neighbour is a register or, across a lane boundary, one
//    cross-lane shuffle.
//  * Vertical solve (phase V): a wavefront covers cpw = floor(64 / L) whole
//    columns with lane = (col - first col) * L + lev, so the implicit system
//    of a column is solved in registers by cyclic reduction across its lanes
//    (ceil(log2 L) shuffle rounds), an exact direct solver of the same
//    tridiagonal the Thomas algorithm solves.  Its horizontal divergences
//    are gathered with the same mapping: staging them through LDS from the
//    gather mapping leaves 4x fewer wavefronts, each solving 4 column groups
//    in turn, and measured slower.
//
// Horizontal stencils use folded coefficients built on the host:
//   div F = (1/r) sum_{j=0..6} c_j . F_j                   (Eqs. flx_div, int_grid, div_gauss)
//   grad s = (1/r) sum_{j=1..6} c_j (s_j - s_0)            (Eq. grad; the curvature term
//                                                           cancels the constant part)
//   lap s = (1/r^2) sum_{j=1..6} l_j (s_j - s_0)           (Sec. 4 triangle-gradient form)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "kernels.h"
#include "powd.h"

// Wavefronts per SIMD that the phase-M kernel is compiled for, as both the
// minimum and the maximum (register budget 512 / n): scheduled for that
// budget the two-ring gathers keep many loads in flight per wavefront
// (FP64: 33 us at 2 against 36 us at 3 and 43 us when the compiler is left
// to aim for 4, at g6 L32).
#define HMOM_OCC_D 2
#ifndef HMOM_OCC_F
#define HMOM_OCC_F 4
#endif
// Two-ring rows of D that k_hmom loads together, FP64 and mixed.
#ifndef HMOM_DU_D
#define HMOM_DU_D 6
#endif
#ifndef HMOM_DU_F
#define HMOM_DU_F 18
#endif
#ifndef HMOM_PU
#define HMOM_PU 6
#endif
// Neighbours whose rows the slow-terms kernel loads together (1; 2 and 3
// measured no faster in FP64 and slower in the mixed form at g6 L32).
#ifndef SLOW_NU
#define SLOW_NU 1
#endif
// Minimum wavefronts per SIMD of k_large1 in FP64 and in mixed precision.
#ifndef LARGE1_OCC_D
#define LARGE1_OCC_D 2
#endif
#ifndef LARGE1_OCC_F
#define LARGE1_OCC_F 2
#endif
#ifndef VERT4_OCC
#define VERT4_OCC 2
#endif
#ifndef VERT4_UNROLL
#define VERT4_UNROLL 3
#endif

namespace thor {
namespace {

struct Lane {
  int lane, lev, col;   // col is clamped to a valid column for loads
  bool store;           // this lane owns a real (col, lev)
  bool real_col;        // lane belongs to one of the wavefront's cpw columns
};

// Workgroups are dispatched round-robin over the XCDs, each with its own L2.
// Renumber them so that XCD x works on one contiguous range of the work: the
// neighbours a column gathers from (ids +-1, +-2^g) then sit in the same L2.
// The launched count is a multiple of kXcds.
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x / kXcds;
  return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

// Lane of logical workgroup lb (blockDim.x / 64 wavefronts per workgroup).
__device__ __forceinline__ Lane map_lane(const Consts &c, int lb) {
  Lane r;
  r.lane = threadIdx.x & 63;
  const int wave = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int cw = r.lane / c.L;
  r.lev = r.lane - cw * c.L;
  int col = wave * c.cpw + cw;
  r.real_col = cw < c.cpw;
  r.store = r.real_col && col < c.N;
  r.col = col < c.N ? col : c.N - 1;
  return r;
}

__device__ __forceinline__ double shfl(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, 64); }

template <typename H>
__device__ __forceinline__ H eos(double rth, const Consts &c) {
  return (H)(c.p_ref * powd(c.Rd * rth / c.p_ref, c.gamma));
}

// Distance from the planet's centre of level centres and interfaces; the
// radial spacing rdz is dz, or 0 in the shallow-atmosphere form (the planet
// radius at every level).
__device__ __forceinline__ double radius_c(const Consts &c, int lev) { return c.radius + (lev + 0.5) * c.rdz; }
__device__ __forceinline__ double radius_i(const Consts &c, int lev) { return c.radius + lev * c.rdz; }

// 1 / x from the hardware reciprocal estimate refined by two Newton steps
// (within an ulp or two of the quotient; for the geometric factors and the
// pivots of the column solve, where no correctly rounded quotient is needed).
__device__ __forceinline__ double rcpd(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Neighbour ids of a column; a pentagon's missing 6th neighbour points at the
// column itself (its coefficients are zero).
__device__ __forceinline__ void load_nbr(const int32_t *nbr, int col, int nb[6]) {
  const int32_t *p = nbr + (size_t)col * 6;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    int v = p[j];
    nb[j] = v < 0 ? col : v;
  }
}

// ---------------------------------------------------------------------------
// Acoustic phase H: explicit horizontal momentum (Eq. mom2) with the
// deviation-pressure gradient, slow forcing and divergence damping, then the
// horizontal projection (Eq. proj_h).
// ---------------------------------------------------------------------------
// Lane of the phase-M mapping: kHq consecutive levels [lev0, lev0 + nv) of
// one column.
struct HLane {
  int col, lev0, nv;
  bool store;
};

__device__ __forceinline__ HLane map_hlane(const Consts &c, int lb) {
  HLane r;
  const int lane = threadIdx.x & 63;
  const int wave = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int cw = lane / c.hlpc;
  const int sub = lane - cw * c.hlpc;
  const int col = wave * c.hcpw + cw;
  r.lev0 = sub * kHq;
  r.nv = min(kHq, c.L - r.lev0);
  r.store = cw < c.hcpw && col < c.N && r.nv > 0;
  r.col = col < c.N ? col : c.N - 1;
  return r;
}

// kHq consecutive values starting at p.  VEC: p is 16-byte aligned and all
// kHq are readable (the state rows have stride S, a multiple of kHq; levels
// from L up are padding); else only the first nv are read.
template <bool VEC>
__device__ __forceinline__ void ld4(const double *p, int nv, double v[kHq]) {
  if (VEC) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else {
#pragma unroll
    for (int q = 0; q < kHq; ++q) v[q] = q < nv ? p[q] : 0.0;
  }
}
template <bool VEC>
__device__ __forceinline__ void ld4(const float *p, int nv, float v[kHq]) {
  if (VEC) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
#pragma unroll
    for (int q = 0; q < kHq; ++q) v[q] = q < nv ? p[q] : 0.0f;
  }
}
// ---------------------------------------------------------------------------
// Cubic vertical interpolation (the Lagrange interpolation of Sec. 2.1 with
// k = 3 on the equally spaced levels).  Centre values to interface j from
// the centres j-2..j+1, weights (-1, 9, 9, -1)/16; at the first interior
// interface (j = 1) from centres 0..3, (5, 15, -5, 1)/16; at the last
// (j = L-1) from centres L-4..L-1, (1, -5, 15, 5)/16.  Interface values to
// centre c the same way: interfaces c-1..c+2, or 0..3 (c = 0), or L-3..L
// (c = L-1), ground and lid included.  Needs L >= 4.
// ---------------------------------------------------------------------------
// The gather mapping's window of a per-level field around a lane's kHq
// levels: win[i] = value at level lev0 - 3 + i (i = 0..9), from the lane,
// the lane below (levels lev0-3..lev0-1) and the lane above (lev0+4 ..
// lev0+6); levels below 0 or from `top` up read as 0 (top = L: for centre
// fields the column's end, for interface fields the lid, which carries
// nothing).  Every lane calls it (shuffles).
template <typename T>
__device__ __forceinline__ void level_window(const T v[kHq], int lev0, int top, int lm, int lp, T win[10]) {
  win[0] = shfl(v[1], lm);
  win[1] = shfl(v[2], lm);
  win[2] = shfl(v[3], lm);
#pragma unroll
  for (int q = 0; q < kHq; ++q) win[3 + q] = v[q];
  win[7] = shfl(v[0], lp);
  win[8] = shfl(v[1], lp);
  win[9] = shfl(v[2], lp);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const int lev = lev0 - 3 + i;
    if (lev < 0 || lev >= top) win[i] = (T)0;
  }
}
// Interface j from the centre window (centre j at win[b], b = j - lev0 + 3).
template <typename T>
__device__ __forceinline__ T cubic_c2i(const T *win, int j, int L) {
  const bool bot = j == 1, top = j == L - 1;
  const T t0 = top ? (T)(1.0 / 16) : (T)0;
  const T t1 = top ? (T)(-5.0 / 16) : (bot ? (T)0 : (T)(-1.0 / 16));
  const T t2 = top ? (T)(15.0 / 16) : (bot ? (T)(5.0 / 16) : (T)(9.0 / 16));
  const T t3 = top ? (T)(5.0 / 16) : (bot ? (T)(15.0 / 16) : (T)(9.0 / 16));
  const T t4 = top ? (T)0 : (bot ? (T)(-5.0 / 16) : (T)(-1.0 / 16));
  const T t5 = bot ? (T)(1.0 / 16) : (T)0;
  // win points at centre j - 3
  return t0 * win[0] + t1 * win[1] + t2 * win[2] + t3 * win[3] + t4 * win[4] + t5 * win[5];
}
// Centre c from the interface window (win points at interface c - 2).
template <typename T>
__device__ __forceinline__ T cubic_i2c(const T *win, int c, int L) {
  const bool bot = c == 0, top = c == L - 1;
  const T t0 = top ? (T)(1.0 / 16) : (T)0;
  const T t1 = top ? (T)(-5.0 / 16) : (bot ? (T)0 : (T)(-1.0 / 16));
  const T t2 = top ? (T)(15.0 / 16) : (bot ? (T)(5.0 / 16) : (T)(9.0 / 16));
  const T t3 = top ? (T)(5.0 / 16) : (bot ? (T)(15.0 / 16) : (T)(9.0 / 16));
  const T t4 = top ? (T)0 : (bot ? (T)(-5.0 / 16) : (T)(-1.0 / 16));
  const T t5 = bot ? (T)(1.0 / 16) : (T)0;
  return t0 * win[0] + t1 * win[1] + t2 * win[2] + t3 * win[3] + t4 * win[4] + t5 * win[5];
}

template <bool VEC>
__device__ __forceinline__ void st4(double *p, int nv, const double v[kHq]) {
  if (VEC) {
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
  } else {
#pragma unroll
    for (int q = 0; q < kHq; ++q)
      if (q < nv) p[q] = v[q];
  }
}
template <bool VEC>
__device__ __forceinline__ void st4(float *p, int nv, const float v[kHq]) {
  if (VEC) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int q = 0; q < kHq; ++q)
      if (q < nv) p[q] = v[q];
  }
}

// Phase M of one lane's kHq levels.  FIRST (the first substep: p* = 0, D
// of the [t] state) and DD (divergence damping) are compile-time (0 or 1)
// in the single-state kernel, so each form is straight-line code whose
// gathers are unrolled (the six p* rows; the 18 two-ring D rows six at a
// time in FP64, all together in the mixed form): the scheduler can put
// the rows of both gathers and of M, S_M in flight together (FP64
// unchanged, mixed 17.4 -> 15.9 us at g6 L32).  The
// ensemble kernel passes -1 for both (runtime flags, partly unrolled
// gathers): there the four forms measured slower (1.31 -> 1.38-1.45 ms per
// launch over 64 planets).  Every form adds its terms in the same order (j,
// m ascending), so all give the same bits.
template <typename H, bool VEC, int FIRST_, int DD_>
__device__ __forceinline__ void hmom_cells(const Fields<H> &f, const Consts &c, const HLane &ln, double dtau,
                                           int first_rt) {
  const bool FIRST = FIRST_ < 0 ? first_rt != 0 : FIRST_ != 0;
  const bool DD = DD_ < 0 ? c.div_damp != 0 : DD_ != 0;
  const int col = ln.col, nv = ln.nv;
  const size_t idx = (size_t)col * c.S + ln.lev0;
  int nb[6];
  if (!FIRST) load_nbr(f.nbr, col, nb);
  int ring[kRing2];
  if (DD) {
    const int32_t *di = f.ddi + (size_t)col * kRing2;
#pragma unroll
    for (int m = 0; m < kRing2; ++m) {
      const int v = di[m];
      ring[m] = v < 0 ? col : v;
    }
  }
  const H *dc = f.dc + (size_t)col * 21;
  H ir[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) ir[q] = (H)1 / (H)radius_c(c, ln.lev0 + q);
  H gx[kHq], gy[kHq], gz[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) gx[q] = gy[q] = gz[q] = 0;
  if (!FIRST) {
    // (1/r) sum_j c_j (p*_j - p*_0)
    H s0[kHq];
    ld4<VEC>(f.ps + idx, nv, s0);
#pragma unroll(FIRST_ < 0 ? 2 : HMOM_PU)
    for (int j = 0; j < 6; ++j) {
      H sj[kHq];
      ld4<VEC>(f.ps + (size_t)nb[j] * c.S + ln.lev0, nv, sj);
      const H cx = dc[3 * (j + 1)], cy = dc[3 * (j + 1) + 1], cz = dc[3 * (j + 1) + 2];
#pragma unroll
      for (int q = 0; q < kHq; ++q) {
        const H d = sj[q] - s0[q];
        gx[q] += cx * d;
        gy[q] += cy * d;
        gz[q] += cz * d;
      }
    }
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      gx[q] *= ir[q];
      gy[q] *= ir[q];
      gz[q] *= ir[q];
    }
  }
  H ddx[kHq], ddy[kHq], ddz[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) ddx[q] = ddy[q] = ddz[q] = 0;
  if (DD) {
    // -Kd lap(grad D) over the two-ring, D of the current small-step state
    const H *D = FIRST ? f.Dt : f.D;
    const H *dw = f.ddw + (size_t)col * kRing2 * 3;
    H d0[kHq];
    ld4<VEC>(D + idx, nv, d0);
#pragma unroll(DD_ < 0 ? 6 : sizeof(H) == 8 ? HMOM_DU_D : HMOM_DU_F)
    for (int m = 0; m < kRing2; ++m) {
      H dm[kHq];
      ld4<VEC>(D + (size_t)ring[m] * c.S + ln.lev0, nv, dm);
      const H wx = dw[3 * m], wy = dw[3 * m + 1], wz = dw[3 * m + 2];
#pragma unroll
      for (int q = 0; q < kHq; ++q) {
        const H dd = dm[q] - d0[q];
        ddx[q] += wx * dd;
        ddy[q] += wy * dd;
        ddz[q] += wz * dd;
      }
    }
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const H s = (H)(-c.Kd) * ir[q] * ir[q] * ir[q];
      ddx[q] *= s;
      ddy[q] *= s;
      ddz[q] *= s;
    }
  }
  const H *rh = f.rhat + (size_t)col * 3;
  const H rx = rh[0], ry = rh[1], rz = rh[2];
  const H dt = (H)dtau;
  H mx[kHq], my[kHq], mz[kHq], sx[kHq], sy[kHq], sz[kHq];
  ld4<VEC>((FIRST ? f.Mx_t : f.Mx) + idx, nv, mx);
  ld4<VEC>((FIRST ? f.My_t : f.My) + idx, nv, my);
  ld4<VEC>((FIRST ? f.Mz_t : f.Mz) + idx, nv, mz);
  ld4<VEC>(f.SMx + idx, nv, sx);
  ld4<VEC>(f.SMy + idx, nv, sy);
  ld4<VEC>(f.SMz + idx, nv, sz);
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const H ax = mx[q] + dt * (-gx[q] + sx[q] + ddx[q]);
    const H ay = my[q] + dt * (-gy[q] + sy[q] + ddy[q]);
    const H az = mz[q] + dt * (-gz[q] + sz[q] + ddz[q]);
    const H mr = ax * rx + ay * ry + az * rz;
    mx[q] = ax - mr * rx;
    my[q] = ay - mr * ry;
    mz[q] = az - mr * rz;
  }
  st4<VEC>(f.Mx + idx, nv, mx);
  st4<VEC>(f.My + idx, nv, my);
  st4<VEC>(f.Mz + idx, nv, mz);
}

template <typename H, bool FORMS>
__device__ __forceinline__ void b_hmom(const Fields<H> &f, const Consts &c, const HLane &ln, double dtau,
                                       int first) {
  if (!ln.store) return;
  // rows of stride S: whole groups of kHq
  if (!FORMS) {
    hmom_cells<H, true, -1, -1>(f, c, ln, dtau, first);
  } else if (first) {
    if (c.div_damp)
      hmom_cells<H, true, 1, 1>(f, c, ln, dtau, first);
    else
      hmom_cells<H, true, 1, 0>(f, c, ln, dtau, first);
  } else {
    if (c.div_damp)
      hmom_cells<H, true, 0, 1>(f, c, ln, dtau, first);
    else
      hmom_cells<H, true, 0, 0>(f, c, ln, dtau, first);
  }
}

// ---------------------------------------------------------------------------
// Physics after the dynamics (Sec. 5), backward Euler at fixed density, on
// one cell: the relaxation of T (Eq. im_eq_t) for the configured forcing.
// Takes and returns the cell's pressure; p0, T0 are the pressure and
// temperature of the column's lowest cell (for p_s); sigma receives p / p_s
// of the input state (Held-Suarez only, for the friction).
//   NEWTONIAN:   K_T = 1 / tau toward the day/night T_eq;
//   HOT_JUPITER: K_T = 1 / tau toward Eqs. teq-hj, btrop, tvert, sigma from
//                the surface pressure the lowest cell implies at constant T;
//   HELD_SUAREZ: K_T and T_eq of Sec. 7.1 with the same sigma.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double physics_p(const Consts &c, const double *teq, int col, int lev, double rho,
                                            double p, double p0, double T0, double &sigma) {
  const double dz = c.dz;
  if (c.forcing == THOR_FORCING_NEWTONIAN) {
    const double kt = c.dt / c.tau;
    const double T = p / (rho * c.Rd);
    const double Tn = (T + kt * teq[col]) / (1.0 + kt);
    p = rho * c.Rd * Tn;
  } else if (c.forcing == THOR_FORCING_HOT_JUPITER) {
    const double kt = c.dt / c.tau;
    const double T = p / (rho * c.Rd);
    const double ps = p0 * exp(c.grav * (0.5 * dz) / (c.Rd * T0));
    const double z = (lev + 0.5) * dz, zs = c.hj_zstrat;
    double Teq;
    if (z <= zs) {
      const double a = c.hj_lapse * (z - zs) / 2.0;
      const double tv = c.hj_Tsurf - c.hj_lapse * (zs + (z - zs) / 2.0) + sqrt(a * a + c.hj_dTstrat * c.hj_dTstrat);
      const double beta = sin(M_PI * (p / ps - c.hj_sstrat) / (2.0 * (1.0 - c.hj_sstrat)));
      Teq = tv + beta * c.hj_dTep * teq[col];
    } else {
      Teq = c.hj_Tsurf - c.hj_lapse * zs + c.hj_dTstrat;
    }
    const double Tn = (T + kt * Teq) / (1.0 + kt);
    p = rho * c.Rd * Tn;
  } else if (c.forcing == THOR_FORCING_HELD_SUAREZ) {
    const double T = p / (rho * c.Rd);
    const double ps = p0 * exp(c.grav * (0.5 * dz) / (c.Rd * T0));
    sigma = p / ps;
    const double s2 = teq[col] * teq[col], c2 = 1.0 - s2;
    const double ramp = fmax(0.0, (sigma - c.hs_sb) / (1.0 - c.hs_sb));
    const double KT = c.hs_ka + (c.hs_ks - c.hs_ka) * ramp * c2 * c2;
    const double x = p / c.hs_pstar;
    const double Teq = fmax(c.hs_Tmin, (c.hs_Ttop - c.hs_dTy * s2 - c.hs_dthz * log(x) * c2) * pow(x, c.Rd / c.Cp));
    const double kt = c.dt * KT;
    const double Tn = (T + kt * Teq) / (1.0 + kt);
    p = rho * c.Rd * Tn;
  }
  return p;
}

// ---------------------------------------------------------------------------
// Acoustic phase V: horizontal mass and theta fluxes of the new momentum,
// then the HEVI vertical-momentum tridiagonal (Eqs. dens2, momr2, pt2
// combined), its solution, and the density / rho-theta updates with the new
// W; pressure from the nonlinear equation of state (Eq. theta_to_p).
// ---------------------------------------------------------------------------
template <typename H, bool LAST, int ORD = 1>
__device__ __forceinline__ void b_vert(const Fields<H> &f, const Consts &c, const Lane &ln, double dtau, int first) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dc = f.dc + (size_t)col * 21;

  // horizontal divergences of M and theta_L M
  H drho, dth;
  {
    H mx = f.Mx[idx], my = f.My[idx], mz = f.Mz[idx];
    H t = dc[0] * mx + dc[1] * my + dc[2] * mz;
    drho = t;
    dth = f.thL[idx] * t;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      size_t nj = (size_t)nb[j] * c.S + lev;
      H u = dc[3 * (j + 1)] * f.Mx[nj] + dc[3 * (j + 1) + 1] * f.My[nj] + dc[3 * (j + 1) + 2] * f.Mz[nj];
      drho += u;
      dth += f.thL[nj] * u;
    }
    const H ir = (H)1 / (H)radius_c(c, lev);
    drho *= ir;
    dth *= ir;
  }

  const double *rho_in = first ? f.rho_t : f.rho;
  const double *rth_in = first ? f.rth_t : f.rth;
  const double *W_in = first ? f.W_t : f.W;
  const double rho0 = rho_in[idx];
  const double rth0 = rth_in[idx];
  const double Wj = lev == 0 ? 0.0 : W_in[idx];
  const double ps_in = first ? 0.0 : (double)f.ps[idx];
  const double pt = f.p_t[idx];
  const double gam = (double)f.Gam[idx];
  const double thC = (double)f.thL[idx];
  const double Drho = (double)drho, Dth = (double)dth;
  const double Hrth = (double)f.Hrth[idx];
  const double rho_hat = rho0 + dtau * (-Drho + (double)f.Hrho[idx]);
  const double rth_hat = rth0 + dtau * (-Dth + Hrth);
  const double phs = ps_in + dtau * gam * (-Dth + Hrth);   // p-hat minus p[t]
  const double rhs = rho_hat - f.rho_t[idx];              // rho-hat minus rho[t]

  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  double thI;   // theta at interface lev
  if (ORD == 3) {
    double tw[6];   // centres lev-3 .. lev+2 of the column (0 outside it)
#pragma unroll
    for (int o = -3; o <= 2; ++o) {
      const int src = min(max(ln.lane + o, 0), 63);
      const double v = shfl(thC, src);
      tw[o + 3] = (lev + o < 0 || lev + o >= L) ? 0.0 : v;
    }
    thI = cubic_c2i(tw, lev, L);
  } else {
    thI = 0.5 * (shfl(thC, lm) + thC);
  }
  const double thI_m = shfl(thI, lm);
  const double thI_p = shfl(thI, lp);
  const double gam_m = shfl(gam, lm);
  const double phs_m = shfl(phs, lm);
  const double rhs_m = shfl(rhs, lm);

  const double dz = c.dz;
  const double rI = radius_i(c, lev), rI1 = rI + c.rdz;
  const double rC = radius_c(c, lev);
  const double irc2dz = 1.0 / (rC * rC * dz);
  const double gp = rI1 * rI1 * irc2dz, gm = rI * rI * irc2dz;
  const double ap = dtau * gp;         // alpha+ of cell lev
  const double am = dtau * gm;         // alpha- of cell lev
  const double ap_m = shfl(ap, lm);    // alpha+ of cell lev-1
  const double am_m = shfl(am, lm);    // alpha- of cell lev-1
  const double c1 = dtau / dz, c2 = 0.5 * c.grav * dtau;

  // first term of the row's right-hand side: the old W and its slow
  // forcing, or in the hydrostatic form (no vertical acceleration, so W
  // leaves the end of the substep balanced) only the [t] imbalance of
  // interface lev
  double d0;
  if (c.hydrostatic) {
    const double rt = f.rho_t[idx];
    const double pt_m = shfl(pt, lm), rt_m = shfl(rt, lm);
    d0 = dtau * (-(pt - pt_m) / dz - 0.5 * c.grav * (rt_m + rt));
  } else {
    d0 = Wj + dtau * f.SW[idx];
  }
  double a = 0.0, b = 1.0, cc = 0.0, d = 0.0;
  if (ln.real_col && lev > 0) {
    a = lev == 1 ? 0.0 : -c1 * gam_m * am_m * thI_m + c2 * am_m;
    b = c.hydrostatic ? c1 * thI * (gam * am + gam_m * ap_m) + c2 * (am - ap_m)
                      : 1.0 + c1 * thI * (gam * am + gam_m * ap_m) + c2 * (am - ap_m);
    cc = lev == L - 1 ? 0.0 : -c1 * gam * ap * thI_p - c2 * ap;
    d = d0 - c1 * (phs - phs_m) - c2 * (rhs_m + rhs);
  }
  // cyclic reduction: after the round with stride s every row couples only
  // to rows lev -/+ 2s of the same column
  for (int s = 1; s < L; s <<= 1) {
    const bool lo = ln.real_col && lev >= s, hi = ln.real_col && lev + s < L;
    const int sl = lo ? ln.lane - s : ln.lane;
    const int sh = hi ? ln.lane + s : ln.lane;
    const double rb = 1.0 / b;
    const double a_l = shfl(a, sl), rb_l = shfl(rb, sl), c_l = shfl(cc, sl), d_l = shfl(d, sl);
    const double a_h = shfl(a, sh), rb_h = shfl(rb, sh), c_h = shfl(cc, sh), d_h = shfl(d, sh);
    const double k1 = lo ? a * rb_l : 0.0;
    const double k2 = hi ? cc * rb_h : 0.0;
    const double na = lo ? -a_l * k1 : 0.0;
    const double nc = hi ? -c_h * k2 : 0.0;
    b = b - (lo ? c_l * k1 : 0.0) - (hi ? a_h * k2 : 0.0);
    d = d - (lo ? d_l * k1 : 0.0) - (hi ? d_h * k2 : 0.0);
    a = na;
    cc = nc;
  }
  const double Wn = lev == 0 ? 0.0 : d / b;
  double Wp = shfl(Wn, lp);
  if (lev == L - 1) Wp = 0.0;

  const double rho_new = rho_hat - ap * Wp + am * Wn;
  double rth_new = rth_hat - ap * thI_p * Wp + am * thI * Wn;
  double p = c.p_ref * powd(c.Rd * rth_new / c.p_ref, c.gamma);
  double hs_sigma = 0.0;
  if (LAST && c.forcing != THOR_FORCING_NONE) {
    const int l0 = ln.lane - lev;   // the column's lowest cell
    const double p0 = shfl(p, l0), T0 = shfl(p / (rho_new * c.Rd), l0);
    p = physics_p(c, f.teq, col, lev, rho_new, p, p0, T0, hs_sigma);
    rth_new = c.p_ref / c.Rd * powd(p / c.p_ref, 1.0 / c.gamma);
  }
  const double D3 = Drho + (gp * Wp - gm * Wn);
  if (ln.store) {
    f.rho[idx] = rho_new;
    f.rth[idx] = rth_new;
    f.W[idx] = Wn;
    f.ps[idx] = (H)(p - pt);
    // after the last substep D is not read again; the Held-Suarez friction
    // takes sigma from it
    f.D[idx] = (H)(LAST && c.forcing == THOR_FORCING_HELD_SUAREZ ? hs_sigma : D3);
  }
}

// ---------------------------------------------------------------------------
// Phase V with two levels per lane (32 < L <= 64: with one level per lane a
// wavefront would hold a single column and leave 64 - L lanes idle).  Lane
// `sub` of a column owns levels 2 sub and 2 sub + 1 and the tridiagonal rows
// of interfaces 2 sub and 2 sub + 1; ceil(L / 2) lanes per column,
// floor(64 / ceil(L / 2)) columns per wavefront.  The same arithmetic as
// b_vert per cell; the solve first eliminates the odd rows inside each lane
// (one step of cyclic reduction), runs cyclic reduction on the even rows
// across the lanes, then recovers the odd unknowns.
// ---------------------------------------------------------------------------
struct Lane2 {
  int lane, sub, lev0, col;
  bool real_col;   // lane belongs to one of the wavefront's columns
  bool store;      // ... and that column exists
};

__device__ __forceinline__ Lane2 map_lane2(const Consts &c, int lb) {
  Lane2 r;
  r.lane = threadIdx.x & 63;
  const int wave = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int cw = r.lane / c.vlpc;
  r.sub = r.lane - cw * c.vlpc;
  r.lev0 = 2 * r.sub;
  int col = wave * c.vcpw + cw;
  r.real_col = cw < c.vcpw;
  r.store = r.real_col && col < c.N;
  r.col = col < c.N ? col : c.N - 1;
  return r;
}

template <typename H, bool LAST>
__device__ __forceinline__ void b_vert2(const Fields<H> &f, const Consts &c, const Lane2 &ln, double dtau,
                                        int first) {
  const int L = c.L, col = ln.col, lev0 = ln.lev0;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dc = f.dc + (size_t)col * 21;
  const double *rho_in = first ? f.rho_t : f.rho;
  const double *rth_in = first ? f.rth_t : f.rth;
  const double *W_in = first ? f.W_t : f.W;
  const double dz = c.dz;
  const double c1 = dtau / dz, c2 = 0.5 * c.grav * dtau;

  // per level of the lane (q = 0, 1); a level past the column's top is
  // loaded from the top level and never stored
  double Drho[2], rho_hat[2], rth_hat[2], phs[2], rhs[2], gam[2], thC[2], pt[2], rt[2], d0[2];
  // radial factors of cell k: g+ = r_I(k+1)^2 / (r_C^2 dz), g- = r_I(k)^2 / (r_C^2 dz)
  auto gpm = [&](int k, double &gpk, double &gmk) {
    const double rI = radius_i(c, k), rI1 = rI + c.rdz;
    const double rC = radius_c(c, k);
    const double irc2dz = 1.0 / (rC * rC * dz);
    gpk = rI1 * rI1 * irc2dz;
    gmk = rI * rI * irc2dz;
  };
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int lev = min(lev0 + q, L - 1);
    const size_t idx = (size_t)col * c.S + lev;
    H drho, dth;
    {
      H mx = f.Mx[idx], my = f.My[idx], mz = f.Mz[idx];
      H t = dc[0] * mx + dc[1] * my + dc[2] * mz;
      drho = t;
      dth = f.thL[idx] * t;
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        size_t nj = (size_t)nb[j] * c.S + lev;
        H u = dc[3 * (j + 1)] * f.Mx[nj] + dc[3 * (j + 1) + 1] * f.My[nj] + dc[3 * (j + 1) + 2] * f.Mz[nj];
        drho += u;
        dth += f.thL[nj] * u;
      }
      const H ir = (H)1 / (H)radius_c(c, lev);
      drho *= ir;
      dth *= ir;
    }
    const double rho0 = rho_in[idx];
    const double rth0 = rth_in[idx];
    const double Wj = lev == 0 ? 0.0 : W_in[idx];
    const double ps_in = first ? 0.0 : (double)f.ps[idx];
    pt[q] = f.p_t[idx];
    gam[q] = (double)f.Gam[idx];
    thC[q] = (double)f.thL[idx];
    Drho[q] = (double)drho;
    const double Dth = (double)dth;
    const double Hrth = (double)f.Hrth[idx];
    rho_hat[q] = rho0 + dtau * (-Drho[q] + (double)f.Hrho[idx]);
    rth_hat[q] = rth0 + dtau * (-Dth + Hrth);
    phs[q] = ps_in + dtau * gam[q] * (-Dth + Hrth);
    rt[q] = f.rho_t[idx];
    rhs[q] = rho_hat[q] - rt[q];
    d0[q] = c.hydrostatic ? 0.0 : Wj + dtau * f.SW[idx];
  }
  // values of level lev0 - 1 (the lane below's second level)
  const double thC_m = shfl(thC[1], lm), gam_m0 = shfl(gam[1], lm), phs_m0 = shfl(phs[1], lm);
  const double rhs_m0 = shfl(rhs[1], lm);
  if (c.hydrostatic) {
    // the [t] imbalance of interfaces lev0 and lev0 + 1
    const double pt_m0 = shfl(pt[1], lm), rt_m0 = shfl(rt[1], lm);
    d0[0] = dtau * (-(pt[0] - pt_m0) / dz - 0.5 * c.grav * (rt_m0 + rt[0]));
    d0[1] = dtau * (-(pt[1] - pt[0]) / dz - 0.5 * c.grav * (rt[0] + rt[1]));
  }
  // theta at interfaces lev0, lev0 + 1, and at lev0 - 1, lev0 + 2
  double thI[2];
  thI[0] = 0.5 * (thC_m + thC[0]);
  thI[1] = 0.5 * (thC[0] + thC[1]);
  const double thI_lo = shfl(thI[1], lm), thI_hi = shfl(thI[0], lp);

  double a[2], b[2], cc[2], d[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int lev = lev0 + q;
    const double thIm = q ? thI[0] : thI_lo, thIp = q ? thI_hi : thI[1];
    const double gamm = q ? gam[0] : gam_m0, phsm = q ? phs[0] : phs_m0, rhsm = q ? rhs[0] : rhs_m0;
    double gpq, gmq, gpm1, gmm1;
    gpm(min(lev, L - 1), gpq, gmq);
    gpm(max(min(lev, L - 1) - 1, 0), gpm1, gmm1);
    const double ap = dtau * gpq, am = dtau * gmq, apm = dtau * gpm1, amm = dtau * gmm1;
    a[q] = 0.0;
    b[q] = 1.0;
    cc[q] = 0.0;
    d[q] = 0.0;
    if (ln.real_col && lev > 0 && lev < L) {
      a[q] = lev == 1 ? 0.0 : -c1 * gamm * amm * thIm + c2 * amm;
      b[q] = c.hydrostatic ? c1 * thI[q] * (gam[q] * am + gamm * apm) + c2 * (am - apm)
                           : 1.0 + c1 * thI[q] * (gam[q] * am + gamm * apm) + c2 * (am - apm);
      cc[q] = lev == L - 1 ? 0.0 : -c1 * gam[q] * ap * thIp - c2 * ap;
      d[q] = d0[q] - c1 * (phs[q] - phsm) - c2 * (rhsm + rhs[q]);
    }
  }
  // eliminate the odd rows: the lane's row 2 sub + 1 and the lane below's
  const int lpc = c.vlpc;
  const bool lo1 = ln.real_col && ln.sub > 0;
  const double r1 = 1.0 / b[1];
  const double a1p = shfl(a[1], lm), b1p = shfl(b[1], lm), c1p = shfl(cc[1], lm), d1p = shfl(d[1], lm);
  const double r1p = 1.0 / b1p;
  double A = lo1 ? -a[0] * a1p * r1p : 0.0;
  double B = b[0] - (lo1 ? a[0] * c1p * r1p : 0.0) - cc[0] * a[1] * r1;
  double C = -cc[0] * cc[1] * r1;
  double D = d[0] - (lo1 ? a[0] * d1p * r1p : 0.0) - cc[0] * d[1] * r1;
  // cyclic reduction of the even rows across the column's lanes
  for (int s = 1; s < lpc; s <<= 1) {
    const bool lo = ln.real_col && ln.sub >= s, hi = ln.real_col && ln.sub + s < lpc;
    const int sl = lo ? ln.lane - s : ln.lane;
    const int sh = hi ? ln.lane + s : ln.lane;
    const double rb = 1.0 / B;
    const double a_l = shfl(A, sl), rb_l = shfl(rb, sl), c_l = shfl(C, sl), d_l = shfl(D, sl);
    const double a_h = shfl(A, sh), rb_h = shfl(rb, sh), c_h = shfl(C, sh), d_h = shfl(D, sh);
    const double k1 = lo ? A * rb_l : 0.0;
    const double k2 = hi ? C * rb_h : 0.0;
    const double na = lo ? -a_l * k1 : 0.0;
    const double nc = hi ? -c_h * k2 : 0.0;
    B = B - (lo ? c_l * k1 : 0.0) - (hi ? a_h * k2 : 0.0);
    D = D - (lo ? d_l * k1 : 0.0) - (hi ? d_h * k2 : 0.0);
    A = na;
    C = nc;
  }
  const double x0 = D / B;                                     // interface lev0
  const bool hi1 = ln.real_col && ln.sub + 1 < lpc;
  const double x2n = shfl(x0, lp);
  const double x2 = hi1 ? x2n : 0.0;                           // interface lev0 + 2
  const double x1 = (d[1] - a[1] * x0 - cc[1] * x2) * r1;      // interface lev0 + 1
  double Wn[2], Wp[2];
  Wn[0] = lev0 == 0 ? 0.0 : x0;
  Wn[1] = lev0 + 1 < L ? x1 : 0.0;
  Wp[0] = Wn[1];
  Wp[1] = lev0 + 2 < L ? x2 : 0.0;

  double rho_new[2], rth_new[2], p[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double thIp = q ? thI_hi : thI[1];
    double gpq, gmq;
    gpm(min(lev0 + q, L - 1), gpq, gmq);
    const double ap = dtau * gpq, am = dtau * gmq;
    rho_new[q] = rho_hat[q] - ap * Wp[q] + am * Wn[q];
    rth_new[q] = rth_hat[q] - ap * thIp * Wp[q] + am * thI[q] * Wn[q];
    p[q] = c.p_ref * powd(c.Rd * rth_new[q] / c.p_ref, c.gamma);
  }
  double hs_sigma[2] = {0.0, 0.0};
  if (LAST && c.forcing != THOR_FORCING_NONE) {
    const int l0 = ln.lane - ln.sub;   // the column's first lane holds its lowest cell
    const double p0 = shfl(p[0], l0), T0 = shfl(p[0] / (rho_new[0] * c.Rd), l0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int lev = min(lev0 + q, L - 1);
      p[q] = physics_p(c, f.teq, col, lev, rho_new[q], p[q], p0, T0, hs_sigma[q]);
      rth_new[q] = c.p_ref / c.Rd * powd(p[q] / c.p_ref, 1.0 / c.gamma);
    }
  }
  if (!ln.store) return;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int lev = lev0 + q;
    if (lev >= L) continue;
    const size_t idx = (size_t)col * c.S + lev;
    double gpq, gmq;
    gpm(lev, gpq, gmq);
    const double D3 = Drho[q] + (gpq * Wp[q] - gmq * Wn[q]);
    f.rho[idx] = rho_new[q];
    f.rth[idx] = rth_new[q];
    f.W[idx] = Wn[q];
    f.ps[idx] = (H)(p[q] - pt[q]);
    f.D[idx] = (H)(LAST && c.forcing == THOR_FORCING_HELD_SUAREZ ? hs_sigma[q] : D3);
  }
}

// ---------------------------------------------------------------------------
// Phase V on the gather mapping: a lane owns kHq = 4 consecutive levels
// lev0..lev0+3 of one column (hlpc = ceil(L / 4) lanes per column, hcpw
// columns per wavefront) and the tridiagonal rows of interfaces lev0..lev0+3.
// Every row moves in 16-byte loads and the per-column stencil data is loaded
// once per 4 cells.  The same arithmetic per cell as b_vert; the solve
// eliminates inside the lane first, by two steps of odd-even (cyclic)
// reduction: the odd rows (lev0+1, lev0+3; the second needs the row below
// the lane, lev0-1, from the lane below), then row lev0+2, which leaves row
// lev0 of each lane coupled to row lev0 of the lanes below and above.
// Cyclic reduction across the column's lanes solves those (ceil(log2 hlpc)
// shuffle rounds), and back substitution recovers rows lev0+2, then
// lev0+1 and lev0+3.  Rows of the ground (interface 0), of levels from L up
// (a partly filled top lane) and of lanes outside the wavefront's columns
// are identity rows (W = 0) whose coefficients are constants, so padding
// levels never reach a real cell; only levels below L are stored.
// ---------------------------------------------------------------------------
struct VLane {
  int lane, sub, lev0, nv, col;
  bool real_col;   // lane belongs to one of the wavefront's columns
  bool store;      // ... and that column exists
};

__device__ __forceinline__ VLane map_vlane(const Consts &c, int lb) {
  VLane r;
  r.lane = threadIdx.x & 63;
  const int wave = lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int cw = r.lane / c.hlpc;
  r.sub = r.lane - cw * c.hlpc;
  r.lev0 = r.sub * kHq;
  r.nv = min(kHq, c.L - r.lev0);
  const int col = wave * c.hcpw + cw;
  r.real_col = cw < c.hcpw;
  r.store = r.real_col && col < c.N;
  r.col = col < c.N ? col : c.N - 1;
  return r;
}

// ANEL (the anelastic switch): the density update takes the divergence of
// the reference-density mass flux, fC M horizontally and fI W vertically,
// and the buoyancy terms of the tridiagonal the matching fI W; the
// divergence-damping D keeps the plain momentum divergence.
template <typename H, bool LAST, bool ANEL = false>
__device__ __forceinline__ void b_vert4(const Fields<H> &f, const Consts &c, const VLane &ln, double dtau,
                                        int first) {
  const int L = c.L, col = ln.col, lev0 = ln.lev0;
  const size_t idx = (size_t)col * c.S + lev0;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dc = f.dc + (size_t)col * 21;

  // radial factors g+ = r_I(k+1)^2 / (r_C^2 dz), g- = r_I(k)^2 / (r_C^2 dz)
  // and 1 / r_C of cells lev0 - 1 .. lev0 + 3 (index k - lev0 + 1)
  const double idz = 1.0 / c.dz;
  double gp[kHq + 1], gm[kHq + 1], irc[kHq + 1];
#pragma unroll
  for (int k = 0; k <= kHq; ++k) {
    const int lev = lev0 - 1 + k;
    const double rI = radius_i(c, lev), rI1 = rI + c.rdz;
    irc[k] = rcpd(radius_c(c, lev));
    const double irc2dz = irc[k] * irc[k] * idz;
    gp[k] = rI1 * rI1 * irc2dz;
    gm[k] = rI * rI * irc2dz;
  }

  // horizontal divergences of M and theta_L M (ANEL: and of fC M)
  H drho[kHq], dth[kHq], thl[kHq], dmass[kHq];
  {
    H mx[kHq], my[kHq], mz[kHq], fc[kHq];
    ld4<true>(f.Mx + idx, kHq, mx);
    ld4<true>(f.My + idx, kHq, my);
    ld4<true>(f.Mz + idx, kHq, mz);
    ld4<true>(f.thL + idx, kHq, thl);
    if (ANEL) ld4<true>(f.fC + idx, kHq, fc);
    const H c0x = dc[0], c0y = dc[1], c0z = dc[2];
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const H t = c0x * mx[q] + c0y * my[q] + c0z * mz[q];
      drho[q] = t;
      dth[q] = thl[q] * t;
      if (ANEL) dmass[q] = fc[q] * t;
    }
#pragma unroll VERT4_UNROLL
    for (int j = 0; j < 6; ++j) {
      const size_t nj = (size_t)nb[j] * c.S + lev0;
      H nx[kHq], ny[kHq], nz[kHq], nt[kHq], nf[kHq];
      ld4<true>(f.Mx + nj, kHq, nx);
      ld4<true>(f.My + nj, kHq, ny);
      ld4<true>(f.Mz + nj, kHq, nz);
      ld4<true>(f.thL + nj, kHq, nt);
      if (ANEL) ld4<true>(f.fC + nj, kHq, nf);
      const H cx = dc[3 * (j + 1)], cy = dc[3 * (j + 1) + 1], cz = dc[3 * (j + 1) + 2];
#pragma unroll
      for (int q = 0; q < kHq; ++q) {
        const H u = cx * nx[q] + cy * ny[q] + cz * nz[q];
        drho[q] += u;
        dth[q] += nt[q] * u;
        if (ANEL) dmass[q] += nf[q] * u;
      }
    }
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const H ir = (H)irc[q + 1];
      drho[q] *= ir;
      dth[q] *= ir;
      if (ANEL) dmass[q] *= ir;
    }
  }

  // explicit parts of density, rho theta and the deviation pressure
  double rho_hat[kHq], rth_hat[kHq], phs[kHq], rhs[kHq], gam[kHq], thC[kHq], pt[kHq], d0[kHq];
  {
    double rho0[kHq], rth0[kHq], rt[kHq];
    H gh[kHq], hrho[kHq], hrth[kHq], psh[kHq];
    ld4<true>((first ? f.rho_t : f.rho) + idx, kHq, rho0);
    ld4<true>((first ? f.rth_t : f.rth) + idx, kHq, rth0);
    ld4<true>(f.p_t + idx, kHq, pt);
    ld4<true>(f.rho_t + idx, kHq, rt);
    ld4<true>(f.Gam + idx, kHq, gh);
    ld4<true>(f.Hrho + idx, kHq, hrho);
    ld4<true>(f.Hrth + idx, kHq, hrth);
    if (first) {
#pragma unroll
      for (int q = 0; q < kHq; ++q) psh[q] = (H)0;
    } else {
      ld4<true>(f.ps + idx, kHq, psh);
    }
    if (c.hydrostatic) {
      // the [t] imbalance of the lane's interfaces (no vertical acceleration:
      // W leaves the end of the substep balanced)
      const double pt_m = shfl(pt[3], lm), rt_m = shfl(rt[3], lm);
#pragma unroll
      for (int q = 0; q < kHq; ++q) {
        const double ptm = q ? pt[q - 1] : pt_m, rtm = q ? rt[q - 1] : rt_m;
        d0[q] = dtau * (-(pt[q] - ptm) * idz - 0.5 * c.grav * (rtm + rt[q]));
      }
    } else {
      double w0[kHq], sw[kHq];
      ld4<true>((first ? f.W_t : f.W) + idx, kHq, w0);
      ld4<true>(f.SW + idx, kHq, sw);
#pragma unroll
      for (int q = 0; q < kHq; ++q) d0[q] = (lev0 + q == 0 ? 0.0 : w0[q]) + dtau * sw[q];
    }
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      gam[q] = (double)gh[q];
      thC[q] = (double)thl[q];
      const double Dr = (double)(ANEL ? dmass[q] : drho[q]), Dt = (double)dth[q], Hr = (double)hrth[q];
      rho_hat[q] = rho0[q] + dtau * (-Dr + (double)hrho[q]);
      rth_hat[q] = rth0[q] + dtau * (-Dt + Hr);
      phs[q] = (double)psh[q] + dtau * gam[q] * (-Dt + Hr);
      rhs[q] = rho_hat[q] - rt[q];
    }
  }

  // theta at the lane's interfaces and at interface lev0 + 4 (lane above)
  double thI[kHq];
  const double thC_dn = shfl(thC[3], lm);
  thI[0] = ln.sub == 0 ? thC[0] : 0.5 * (thC_dn + thC[0]);   // interface 0 only meets W = 0
#pragma unroll
  for (int q = 1; q < kHq; ++q) thI[q] = 0.5 * (thC[q - 1] + thC[q]);
  const double thI_up = shfl(thI[0], lp);
  const double gam_m = shfl(gam[3], lm), phs_m = shfl(phs[3], lm), rhs_m = shfl(rhs[3], lm);

  const double c1 = dtau * idz, c2 = 0.5 * c.grav * dtau;

  // ANEL: the mass-flux factors of the lane's interfaces and of interfaces
  // lev0 - 1 and lev0 + 4
  double fI[kHq] = {1.0, 1.0, 1.0, 1.0}, fI_dn = 1.0, fI_up = 1.0;
  if (ANEL) {
    ld4<true>(f.fI + idx, kHq, fI);
    fI_dn = shfl(fI[3], lm);
    fI_up = shfl(fI[0], lp);
  }

  // rows of interfaces lev0 + q: a x[j-1] + b x[j] + cc x[j+1] = d
  const double thI_dn = shfl(thI[3], lm);   // interface lev0 - 1
  double a[kHq], b[kHq], cc[kHq], d[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const int j = lev0 + q;
    const double ap = dtau * gp[q + 1], am = dtau * gm[q + 1];   // cell j
    const double apm = dtau * gp[q], amm = dtau * gm[q];         // cell j - 1
    const double gmq = q ? gam[q - 1] : gam_m, phsm = q ? phs[q - 1] : phs_m, rhsm = q ? rhs[q - 1] : rhs_m;
    const double thIm = q ? thI[q - 1] : thI_dn, thIp = q < kHq - 1 ? thI[q + 1] : thI_up;
    // ANEL: the buoyancy terms (c2) see the density change of fI W
    const double fIm = q ? fI[q - 1] : fI_dn, fIp = q < kHq - 1 ? fI[q + 1] : fI_up;
    a[q] = 0.0;
    b[q] = 1.0;
    cc[q] = 0.0;
    d[q] = 0.0;
    if (ln.real_col && j > 0 && j < L) {
      if (ANEL) {
        a[q] = j == 1 ? 0.0 : -c1 * gmq * amm * thIm + c2 * amm * fIm;
        b[q] = c.hydrostatic ? c1 * thI[q] * (gam[q] * am + gmq * apm) + c2 * (am - apm) * fI[q]
                             : 1.0 + c1 * thI[q] * (gam[q] * am + gmq * apm) + c2 * (am - apm) * fI[q];
        cc[q] = j == L - 1 ? 0.0 : -c1 * gam[q] * ap * thIp - c2 * ap * fIp;
      } else {
        a[q] = j == 1 ? 0.0 : -c1 * gmq * amm * thIm + c2 * amm;
        b[q] = c.hydrostatic ? c1 * thI[q] * (gam[q] * am + gmq * apm) + c2 * (am - apm)
                             : 1.0 + c1 * thI[q] * (gam[q] * am + gmq * apm) + c2 * (am - apm);
        cc[q] = j == L - 1 ? 0.0 : -c1 * gam[q] * ap * thIp - c2 * ap;
      }
      d[q] = d0[q] - c1 * (phs[q] - phsm) - c2 * (rhsm + rhs[q]);
    }
  }

  // (1) eliminate the odd rows 1 and 3 from rows 0 and 2; row 0 also uses
  // row 3 of the lane below (a[0] = 0 in the column's first lane)
  const bool first_lane = ln.sub == 0;
  const double r1 = rcpd(b[1]), r3 = rcpd(b[3]);
  const double a3d = shfl(a[3], lm), r3d = shfl(r3, lm), c3d = shfl(cc[3], lm), d3d = shfl(d[3], lm);
  double A0, B0, C0, D0, A2, B2, C2, D2;
  {
    const double k1 = first_lane ? 0.0 : a[0] * r3d, k2 = cc[0] * r1;
    A0 = -a3d * k1;              // couples to row 2 of the lane below
    B0 = b[0] - c3d * k1 - a[1] * k2;
    C0 = -cc[1] * k2;            // couples to row 2
    D0 = d[0] - d3d * k1 - d[1] * k2;
  }
  {
    const double k1 = a[2] * r1, k2 = cc[2] * r3;
    A2 = -a[1] * k1;             // couples to row 0
    B2 = b[2] - cc[1] * k1 - a[3] * k2;
    C2 = -cc[3] * k2;            // couples to row 0 of the lane above
    D2 = d[2] - d[1] * k1 - d[3] * k2;
  }
  // (2) eliminate row 2 (the lane's own and the lane below's) from row 0
  const double R2 = rcpd(B2);
  const double A2d = shfl(A2, lm), R2d = shfl(R2, lm), C2d = shfl(C2, lm), D2d = shfl(D2, lm);
  double A, B, C, D;
  {
    const double k1 = first_lane ? 0.0 : A0 * R2d, k2 = C0 * R2;
    A = -A2d * k1;               // couples to row 0 of the lane below
    B = B0 - C2d * k1 - A2 * k2;
    C = -C2 * k2;                // couples to row 0 of the lane above
    D = D0 - D2d * k1 - D2 * k2;
  }
  // (3) cyclic reduction of the rows 0 across the column's lanes
  const int lpc = c.hlpc;
  for (int s = 1; s < lpc; s <<= 1) {
    const bool lo = ln.real_col && ln.sub >= s, hi = ln.real_col && ln.sub + s < lpc;
    const int sl = lo ? ln.lane - s : ln.lane;
    const int sh = hi ? ln.lane + s : ln.lane;
    const double rb = rcpd(B);
    const double a_l = shfl(A, sl), rb_l = shfl(rb, sl), c_l = shfl(C, sl), d_l = shfl(D, sl);
    const double a_h = shfl(A, sh), rb_h = shfl(rb, sh), c_h = shfl(C, sh), d_h = shfl(D, sh);
    const double k1 = lo ? A * rb_l : 0.0;
    const double k2 = hi ? C * rb_h : 0.0;
    const double na = lo ? -a_l * k1 : 0.0;
    const double nc = hi ? -c_h * k2 : 0.0;
    B = B - (lo ? c_l * k1 : 0.0) - (hi ? a_h * k2 : 0.0);
    D = D - (lo ? d_l * k1 : 0.0) - (hi ? d_h * k2 : 0.0);
    A = na;
    C = nc;
  }
  // (4) back substitution: row 0, then row 2 (with row 0 of the lane
  // above), then rows 1 and 3
  double x[kHq];
  x[0] = D * rcpd(B);
  const bool last_lane = ln.sub + 1 >= lpc;
  const double x4n = shfl(x[0], lp);
  const double x4 = last_lane ? 0.0 : x4n;   // interface lev0 + 4
  x[2] = (D2 - A2 * x[0] - C2 * x4) * R2;
  x[1] = (d[1] - a[1] * x[0] - cc[1] * x[2]) * r1;
  x[3] = (d[3] - a[3] * x[2] - cc[3] * x4) * r3;

  double Wn[kHq], Wp[kHq], rho_new[kHq], rth_new[kHq], p[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const int j = lev0 + q;
    Wn[q] = (j > 0 && j < L) ? x[q] : 0.0;
    Wp[q] = j + 1 < L ? (q < kHq - 1 ? x[q + 1] : x4) : 0.0;
    const double thIp = j + 1 < L ? (q < kHq - 1 ? thI[q + 1] : thI_up) : 0.0;
    const double ap = dtau * gp[q + 1], am = dtau * gm[q + 1];
    if (ANEL) {
      const double fIp = q < kHq - 1 ? fI[q + 1] : fI_up;
      rho_new[q] = rho_hat[q] - ap * fIp * Wp[q] + am * fI[q] * Wn[q];
    } else {
      rho_new[q] = rho_hat[q] - ap * Wp[q] + am * Wn[q];
    }
    rth_new[q] = rth_hat[q] - ap * thIp * Wp[q] + am * thI[q] * Wn[q];
    p[q] = c.p_ref * powd(c.Rd * rth_new[q] / c.p_ref, c.gamma);
  }
  double hs_sigma[kHq] = {0.0, 0.0, 0.0, 0.0};
  if (LAST && c.forcing != THOR_FORCING_NONE) {
    const int l0 = ln.lane - ln.sub;   // the column's first lane holds its lowest cell
    const double p0 = shfl(p[0], l0), T0 = shfl(p[0] / (rho_new[0] * c.Rd), l0);
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = min(lev0 + q, L - 1);
      p[q] = physics_p(c, f.teq, col, lev, rho_new[q], p[q], p0, T0, hs_sigma[q]);
      rth_new[q] = c.p_ref / c.Rd * powd(p[q] / c.p_ref, 1.0 / c.gamma);
    }
  }
  if (!ln.store) return;
  H psn[kHq], dn[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    psn[q] = (H)(p[q] - pt[q]);
    const double D3 = (double)drho[q] + (gp[q + 1] * Wp[q] - gm[q + 1] * Wn[q]);
    dn[q] = (H)(LAST && c.forcing == THOR_FORCING_HELD_SUAREZ ? hs_sigma[q] : D3);
  }
  if (ln.nv == kHq) {
    st4<true>(f.rho + idx, kHq, rho_new);
    st4<true>(f.rth + idx, kHq, rth_new);
    st4<true>(f.W + idx, kHq, Wn);
    st4<true>(f.ps + idx, kHq, psn);
    st4<true>(f.D + idx, kHq, dn);
  } else {
    st4<false>(f.rho + idx, ln.nv, rho_new);
    st4<false>(f.rth + idx, ln.nv, rth_new);
    st4<false>(f.W + idx, ln.nv, Wn);
    st4<false>(f.ps + idx, ln.nv, psn);
    st4<false>(f.D + idx, ln.nv, dn);
  }
}

// Held-Suarez boundary-layer friction (Eq. im_eq_v with K_v of Eq. im_eq_fv)
// after the last phase V of a large step, with sigma of the dynamics output
// left in D by that kernel.  Other forcings: nothing.
template <typename H>
__device__ __forceinline__ void b_friction(const Fields<H> &f, const Consts &c, const HLane &ln) {
  if (!ln.store || c.forcing != THOR_FORCING_HELD_SUAREZ) return;
  const size_t idx = (size_t)ln.col * c.S + ln.lev0;
  H sg[kHq], mx[kHq], my[kHq], mz[kHq];
  ld4<true>(f.D + idx, kHq, sg);
  ld4<true>(f.Mx + idx, kHq, mx);
  ld4<true>(f.My + idx, kHq, my);
  ld4<true>(f.Mz + idx, kHq, mz);
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const double sigma = (double)sg[q];
    const double kv = c.hs_kf * fmax(0.0, (sigma - c.hs_sb) / (1.0 - c.hs_sb));
    const double den = 1.0 + kv * c.dt;
    mx[q] = (H)((double)mx[q] / den);
    my[q] = (H)((double)my[q] / den);
    mz[q] = (H)((double)mz[q] / den);
  }
  // levels from L up are left as they are
  if (ln.nv == kHq) {
    st4<true>(f.Mx + idx, kHq, mx);
    st4<true>(f.My + idx, kHq, my);
    st4<true>(f.Mz + idx, kHq, mz);
  } else {
    st4<false>(f.Mx + idx, ln.nv, mx);
    st4<false>(f.My + idx, ln.nv, my);
    st4<false>(f.Mz + idx, ln.nv, mz);
  }
}

// ---------------------------------------------------------------------------
// Slow terms of one RK stage at the previous stage state: advection of the
// full Cartesian momentum, Coriolis, projections (Eqs. mom, proj_h, proj_r),
// and the linearisation coefficients theta_L and gamma p / (rho theta).
// ---------------------------------------------------------------------------
template <typename H, bool VEC, bool SHALLOW, int ORD>
__device__ __forceinline__ void slow_cells(const Fields<H> &f, const Consts &c, const HLane &ln, int from_t) {
  const int L = c.L, col = ln.col, nv = ln.nv, lev0 = ln.lev0;
  const int lane = threadIdx.x & 63;
  const int lm = lane > 0 ? lane - 1 : 0;
  const int lp = lane < 63 ? lane + 1 : 63;
  const size_t idx = (size_t)col * c.S + lev0;
  const double *rho = from_t ? f.rho_t : f.rho;
  const double *rth = from_t ? f.rth_t : f.rth;
  const double *W = from_t ? f.W_t : f.W;
  const H *Mx = from_t ? f.Mx_t : f.Mx;
  const H *My = from_t ? f.My_t : f.My;
  const H *Mz = from_t ? f.Mz_t : f.Mz;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dc = f.dc + (size_t)col * 21;
  const H *rh = f.rhat + (size_t)col * 3;
  const H rx = rh[0], ry = rh[1], rz = rh[2];

  // own column: full momentum m = M + Wbar rhat and velocity m / rho (in the
  // shallow form the horizontal momentum M and velocity M / rho, with the
  // vertical velocity w = Wbar / rho advected as a scalar in Ar)
  double Wk[kHq], rho0[kHq];
  H fx[kHq], fy[kHq], fz[kHq], vx0[kHq], vy0[kHq], vz0[kHq];
  H Ax[kHq], Ay[kHq], Az[kHq];
  H w0[kHq], Ar[kHq];
  {
    ld4<VEC>(W + idx, nv, Wk);
    if (lev0 == 0) Wk[0] = 0.0;
    const double Wn = shfl(Wk[0], lp);   // interface lev0 + kHq: first value of the next lane
    double Wwin[10];
    if (ORD == 3) level_window(Wk, lev0, L, lm, lp, Wwin);
    ld4<VEC>(rho + idx, nv, rho0);
    H mx0[kHq], my0[kHq], mz0[kHq];
    ld4<VEC>(Mx + idx, nv, mx0);
    ld4<VEC>(My + idx, nv, my0);
    ld4<VEC>(Mz + idx, nv, mz0);
    const H d0x = dc[0], d0y = dc[1], d0z = dc[2];
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const double up = lev0 + q == L - 1 ? 0.0 : (q + 1 < kHq ? Wk[q + 1] : Wn);
      const H wbar = ORD == 3 ? (H)cubic_i2c(Wwin + q + 1, lev0 + q, L) : (H)(0.5 * (Wk[q] + up));
      if (SHALLOW) {
        fx[q] = mx0[q];
        fy[q] = my0[q];
        fz[q] = mz0[q];
      } else {
        fx[q] = mx0[q] + wbar * rx;
        fy[q] = my0[q] + wbar * ry;
        fz[q] = mz0[q] + wbar * rz;
      }
      const H irho0 = (H)1 / (H)rho0[q];
      vx0[q] = fx[q] * irho0;
      vy0[q] = fy[q] * irho0;
      vz0[q] = fz[q] * irho0;
      // horizontal flux divergence of v_q M: own-column term
      const H t = d0x * mx0[q] + d0y * my0[q] + d0z * mz0[q];
      Ax[q] = vx0[q] * t;
      Ay[q] = vy0[q] * t;
      Az[q] = vz0[q] * t;
      if (SHALLOW) {
        w0[q] = wbar * irho0;
        Ar[q] = w0[q] * t;
      }
    }
  }
#pragma unroll SLOW_NU
  for (int j = 0; j < 6; ++j) {
    const size_t nj = (size_t)nb[j] * c.S + lev0;
    double wn[kHq], rj[kHq];
    H mxj[kHq], myj[kHq], mzj[kHq];
    ld4<VEC>(W + nj, nv, wn);
    if (lev0 == 0) wn[0] = 0.0;
    const double wnn = shfl(wn[0], lp);
    double wwin[10];
    if (ORD == 3) level_window(wn, lev0, L, lm, lp, wwin);
    ld4<VEC>(rho + nj, nv, rj);
    ld4<VEC>(Mx + nj, nv, mxj);
    ld4<VEC>(My + nj, nv, myj);
    ld4<VEC>(Mz + nj, nv, mzj);
    const H *rn = f.rhat + (size_t)nb[j] * 3;
    const H rnx = rn[0], rny = rn[1], rnz = rn[2];
    const H cx = dc[3 * (j + 1)], cy = dc[3 * (j + 1) + 1], cz = dc[3 * (j + 1) + 2];
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const double up = lev0 + q == L - 1 ? 0.0 : (q + 1 < kHq ? wn[q + 1] : wnn);
      const H wb = ORD == 3 ? (H)cubic_i2c(wwin + q + 1, lev0 + q, L) : (H)(0.5 * (wn[q] + up));
      const H t = (cx * mxj[q] + cy * myj[q] + cz * mzj[q]) / (H)rj[q];
      if (SHALLOW) {
        Ax[q] += mxj[q] * t;
        Ay[q] += myj[q] * t;
        Az[q] += mzj[q] * t;
        Ar[q] += wb * t;
      } else {
        Ax[q] += (mxj[q] + wb * rnx) * t;
        Ay[q] += (myj[q] + wb * rny) * t;
        Az[q] += (mzj[q] + wb * rnz) * t;
      }
    }
  }
  // vertical flux divergence: r^2 W v_q at the interfaces
  H Fx[kHq], Fy[kHq], Fz[kHq], Fr[kHq];
  if (ORD == 3) {
    // r^2 W times the cubic interface value of v_q (and of w)
    H xw[10], yw[10], zw[10], ww[10];
    level_window(vx0, lev0, L, lm, lp, xw);
    level_window(vy0, lev0, L, lm, lp, yw);
    level_window(vz0, lev0, L, lm, lp, zw);
    if (SHALLOW) level_window(w0, lev0, L, lm, lp, ww);
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const H rI = (H)radius_i(c, lev);
      const H w2 = (H)Wk[q] * rI * rI;
      Fx[q] = lev == 0 ? (H)0 : w2 * cubic_c2i(xw + q, lev, L);
      Fy[q] = lev == 0 ? (H)0 : w2 * cubic_c2i(yw + q, lev, L);
      Fz[q] = lev == 0 ? (H)0 : w2 * cubic_c2i(zw + q, lev, L);
      if (SHALLOW) Fr[q] = lev == 0 ? (H)0 : w2 * cubic_c2i(ww + q, lev, L);
    }
  } else {
    const H vxm = shfl(vx0[kHq - 1], lm), vym = shfl(vy0[kHq - 1], lm), vzm = shfl(vz0[kHq - 1], lm);
    const H wm = SHALLOW ? shfl(w0[kHq - 1], lm) : (H)0;
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const H rI = (H)radius_i(c, lev);
      const H w2 = (H)Wk[q] * rI * rI * (H)0.5;
      const H px = q ? vx0[q - 1] : vxm, py = q ? vy0[q - 1] : vym, pz = q ? vz0[q - 1] : vzm;
      Fx[q] = lev == 0 ? (H)0 : w2 * (px + vx0[q]);
      Fy[q] = lev == 0 ? (H)0 : w2 * (py + vy0[q]);
      Fz[q] = lev == 0 ? (H)0 : w2 * (pz + vz0[q]);
      if (SHALLOW) Fr[q] = lev == 0 ? (H)0 : w2 * ((q ? w0[q - 1] : wm) + w0[q]);
    }
  }
  H acr[kHq];
  {
    const H nx = shfl(Fx[0], lp), ny = shfl(Fy[0], lp), nz = shfl(Fz[0], lp);
    const H nr = SHALLOW ? shfl(Fr[0], lp) : (H)0;
    const H om2 = (H)(2.0 * c.omega);
    const H idz = (H)(1.0 / c.dz);
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const H irc = (H)1 / (H)radius_c(c, lev);
      H Fx1 = q + 1 < kHq ? Fx[q + 1] : nx, Fy1 = q + 1 < kHq ? Fy[q + 1] : ny,
        Fz1 = q + 1 < kHq ? Fz[q + 1] : nz;
      if (lev == L - 1) Fx1 = Fy1 = Fz1 = 0;
      Ax[q] *= irc;
      Ay[q] *= irc;
      Az[q] *= irc;
      const H s = irc * irc * idz;
      Ax[q] += (Fx1 - Fx[q]) * s;
      Ay[q] += (Fy1 - Fy[q]) * s;
      Az[q] += (Fz1 - Fz[q]) * s;
      if (SHALLOW) {
        // traditional approximation: 2 Omega sin(lat) rhat x M, horizontal;
        // the horizontal equations take the projection of A here and the
        // vertical one the scalar advection of w
        const H fc = om2 * rz;
        Ax[q] += fc * (ry * fz[q] - rz * fy[q]);
        Ay[q] += fc * (rz * fx[q] - rx * fz[q]);
        Az[q] += fc * (rx * fy[q] - ry * fx[q]);
        const H ah = Ax[q] * rx + Ay[q] * ry + Az[q] * rz;
        Ax[q] -= ah * rx;
        Ay[q] -= ah * ry;
        Az[q] -= ah * rz;
        H Fr1 = q + 1 < kHq ? Fr[q + 1] : nr;
        if (lev == L - 1) Fr1 = 0;
        acr[q] = Ar[q] * irc + (Fr1 - Fr[q]) * s;
      } else {
        // Coriolis 2 Omega zhat x m
        Ax[q] -= om2 * fy[q];
        Ay[q] += om2 * fx[q];
        acr[q] = Ax[q] * rx + Ay[q] * ry + Az[q] * rz;
      }
    }
  }
  const H acr_m = shfl(acr[kHq - 1], lm);
  H aw[10];
  if (ORD == 3) level_window(acr, lev0, L, lm, lp, aw);
  if (!ln.store) return;
  H smx[kHq], smy[kHq], smz[kHq], thl[kHq], gam[kHq];
  double sw[kHq], fw[kHq], rth0[kHq], pt[kHq];
  H ps[kHq];
  ld4<VEC>(f.FMx + idx, nv, smx);
  ld4<VEC>(f.FMy + idx, nv, smy);
  ld4<VEC>(f.FMz + idx, nv, smz);
  ld4<VEC>(f.FW + idx, nv, fw);
  ld4<VEC>(rth + idx, nv, rth0);
  ld4<VEC>(f.p_t + idx, nv, pt);
  if (!from_t) ld4<VEC>(f.ps + idx, nv, ps);
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    if (SHALLOW) {   // A is horizontal already
      smx[q] -= Ax[q];
      smy[q] -= Ay[q];
      smz[q] -= Az[q];
    } else {
      smx[q] -= Ax[q] - acr[q] * rx;
      smy[q] -= Ay[q] - acr[q] * ry;
      smz[q] -= Az[q] - acr[q] * rz;
    }
    const H am = q ? acr[q - 1] : acr_m;
    if (ORD == 3)
      sw[q] = lev0 + q == 0 ? 0.0 : fw[q] - (double)cubic_c2i(aw + q, lev0 + q, L);
    else
      sw[q] = lev0 + q == 0 ? 0.0 : fw[q] - 0.5 * ((double)am + (double)acr[q]);
    // linearisation coefficients
    const double p0 = pt[q] + (from_t ? 0.0 : (double)ps[q]);
    thl[q] = (H)(rth0[q] / rho0[q]);
    gam[q] = (H)(c.gamma * p0 / rth0[q]);
  }
  st4<VEC>(f.SMx + idx, nv, smx);
  st4<VEC>(f.SMy + idx, nv, smy);
  st4<VEC>(f.SMz + idx, nv, smz);
  st4<VEC>(f.SW + idx, nv, sw);
  st4<VEC>(f.thL + idx, nv, thl);
  st4<VEC>(f.Gam + idx, nv, gam);
}

template <typename H, bool SHALLOW = false, int ORD = 1>
__device__ __forceinline__ void b_slow(const Fields<H> &f, const Consts &c, const HLane &ln, int from_t) {
  slow_cells<H, true, SHALLOW, ORD>(f, c, ln, from_t);   // rows of stride S: whole groups of kHq
}

// ---------------------------------------------------------------------------
// Per large step: keep Phi[t], diagnose p[t], T, v and w (pointwise), then
// two Laplacian passes for the hyperdiffusion (Eqs. diff_rho ... diff_p),
// grad p[t], the [t] vertical imbalance and the divergence-damping terms of
// Phi[t].
// ---------------------------------------------------------------------------
// Density at the interfaces lev0 .. lev0 + kHq - 1 of a lane's levels (the
// mean of the two neighbouring centres, or the cubic interpolation): the
// interface density of the hyperdiffusion of rho v_r.  Every lane calls it.
template <bool VEC>
__device__ __forceinline__ void interface_rho(const Consts &c, const double rho[kHq], int lev0, int lm, int lp,
                                              double rhoI[kHq]) {
  if (c.vorder == 3) {
    double win[10];
    level_window(rho, lev0, c.L, lm, lp, win);
#pragma unroll
    for (int q = 0; q < kHq; ++q) rhoI[q] = cubic_c2i(win + q, lev0 + q, c.L);
  } else {
    const double rho_m = shfl(rho[kHq - 1], lm);
#pragma unroll
    for (int q = 0; q < kHq; ++q) rhoI[q] = 0.5 * ((q ? rho[q - 1] : rho_m) + rho[q]);
  }
}

template <typename H, bool VEC>
__device__ __forceinline__ void large0_cells(const Fields<H> &f, const Consts &c, const HLane &ln) {
  const int lev0 = ln.lev0, nv = ln.nv;
  const size_t idx = (size_t)ln.col * c.S + lev0;
  const int lane = threadIdx.x & 63;
  const int lm = lane > 0 ? lane - 1 : 0;
  const int lp = lane < 63 ? lane + 1 : 63;
  double rho[kHq], rth[kHq], W[kHq];
  ld4<VEC>(f.rho_t + idx, nv, rho);
  ld4<VEC>(f.rth_t + idx, nv, rth);
  ld4<VEC>(f.W_t + idx, nv, W);
  double rhoI[kHq];   // rho at interfaces lev0 .. lev0 + 3
  interface_rho<VEC>(c, rho, lev0, lm, lp, rhoI);
  if (!ln.store) return;
  double p[kHq], wI[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    p[q] = c.p_ref * powd(c.Rd * rth[q] / c.p_ref, c.gamma);
    wI[q] = lev0 + q == 0 ? 0.0 : W[q] / rhoI[q];
  }
  st4<VEC>(f.p_t + idx, nv, p);
  st4<VEC>(f.wI + idx, nv, wI);
}

// The velocity M / rho and temperature p / (rho Rd) of kHq cells, the
// Laplacian inputs of the momentum and pressure hyperdiffusion, formed where
// they are gathered (every cell forms them the same way, so a neighbour's
// value equals its own).
template <typename H>
__device__ __forceinline__ void vel_temp(const Consts &c, const double rho[kHq], const double p[kHq], const H mx[kHq],
                                         const H my[kHq], const H mz[kHq], double vx[kHq], double vy[kHq],
                                         double vz[kHq], double T[kHq]) {
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const double irho = 1.0 / rho[q];
    T[q] = p[q] * irho / c.Rd;
    vx[q] = (double)mx[q] * irho;
    vy[q] = (double)my[q] * irho;
    vz[q] = (double)mz[q] * irho;
  }
}

// Anelastic switch only (Sec. 3 anelastic approximation): the mass flux is
// rho_r v with v the momentum over rho[t]; its factors rho_r / rho[t] at the
// centres and the ratio of the two-point means at the interior interfaces
// are frozen for the large step (interface 0 only meets W = 0).
template <typename H, bool VEC>
__device__ __forceinline__ void anel_cells(const Fields<H> &f, const Consts &c, const HLane &ln) {
  const int lev0 = ln.lev0, nv = ln.nv;
  const size_t idx = (size_t)ln.col * c.S + lev0;
  const int lane = threadIdx.x & 63;
  const int lm = lane > 0 ? lane - 1 : 0;
  const double rho_m = shfl(f.rho_t[idx + kHq - 1], lm);   // every lane shuffles
  if (!ln.store) return;
  double rho[kHq], rr[kHq], fi[kHq];
  H fc[kHq];
  ld4<VEC>(f.rho_t + idx, nv, rho);
  ld4<VEC>(f.rref + lev0, nv, rr);
  const double rr_m = lev0 ? f.rref[lev0 - 1] : 0.0;
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    fc[q] = (H)(rr[q] / rho[q]);
    const double rhoI = 0.5 * ((q ? rho[q - 1] : rho_m) + rho[q]);
    fi[q] = lev0 + q == 0 ? 1.0 : 0.5 * ((q ? rr[q - 1] : rr_m) + rr[q]) / rhoI;
  }
  st4<VEC>(f.fC + idx, nv, fc);
  st4<VEC>(f.fI + idx, nv, fi);
}

// sum_j l_j (s_j - s_0) at kHq consecutive levels: the Laplacian without
// its 1/r^2.
template <bool VEC, typename T, typename H>
__device__ __forceinline__ void lap4(const T *s, const int nb[6], const H *lc, int S, int lev0, int nv, size_t idx,
                                     T out[kHq]) {
  T s0[kHq];
  ld4<VEC>(s + idx, nv, s0);
#pragma unroll
  for (int q = 0; q < kHq; ++q) out[q] = 0;
#pragma unroll 2
  for (int j = 0; j < 6; ++j) {
    T sj[kHq];
    ld4<VEC>(s + (size_t)nb[j] * S + lev0, nv, sj);
    const T w = (T)lc[j];
#pragma unroll
    for (int q = 0; q < kHq; ++q) out[q] += w * (sj[q] - s0[q]);
  }
}

// Per large step, first pass: the inner Laplacians of the hyperdiffusion
// (rho; rho Kd lap of vx, vy, vz, T; rho_I Kd lap of w at the interfaces)
// and the 3D momentum divergence of Phi[t] (the second pass forms -grad
// p[t] and the [t] imbalance next to the hyperdiffusion it adds to them).
// One neighbour-major pass loads the rows of rho, p, Mx, My, Mz and w_I of
// neighbour j together and forms the neighbour's velocity and temperature
// from them (rather than reading fields the previous kernel stored); every
// sum takes its j-th term, so each adds its terms in the same order as a
// field-by-field pass.
template <typename H, bool VEC>
__device__ __forceinline__ void large1_cells(const Fields<H> &f, const Consts &c, const HLane &ln) {
  const int L = c.L, lev0 = ln.lev0, nv = ln.nv, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev0;
  const int lane = threadIdx.x & 63;
  const int lm = lane > 0 ? lane - 1 : 0;
  const int lp = lane < 63 ? lane + 1 : 63;
  double rho[kHq], p[kHq], W[kHq];
  ld4<VEC>(f.rho_t + idx, nv, rho);
  ld4<VEC>(f.p_t + idx, nv, p);
  ld4<VEC>(f.W_t + idx, nv, W);
  const double W_n = shfl(W[0], lp);
  double rhoI[kHq];   // rho at interfaces lev0 .. lev0 + 3
  interface_rho<VEC>(c, rho, lev0, lm, lp, rhoI);
  if (!ln.store) return;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dch = f.dc + (size_t)col * 21;
  const H *lch = f.lc + (size_t)col * 6;
  const double Kd = c.Kd;
  double irc2[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const double rC = radius_c(c, lev0 + q);
    irc2[q] = 1.0 / (rC * rC);
  }
  // Laplacian fields: rho, vx, vy, vz, T, w (rho is rho[] itself)
  double s0[6][kHq], lap[6][kHq];
  H dm[kHq];
  {
    H mx[kHq], my[kHq], mz[kHq];
    ld4<VEC>(f.Mx_t + idx, nv, mx);
    ld4<VEC>(f.My_t + idx, nv, my);
    ld4<VEC>(f.Mz_t + idx, nv, mz);
#pragma unroll
    for (int q = 0; q < kHq; ++q) dm[q] = dch[0] * mx[q] + dch[1] * my[q] + dch[2] * mz[q];
    vel_temp<H>(c, rho, p, mx, my, mz, s0[1], s0[2], s0[3], s0[4]);
  }
#pragma unroll
  for (int q = 0; q < kHq; ++q) s0[0][q] = rho[q];
  ld4<VEC>(f.wI + idx, nv, s0[5]);
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int q = 0; q < kHq; ++q) lap[k][q] = 0;
#pragma unroll 1
  for (int j = 0; j < 6; ++j) {
    const size_t nj = (size_t)nb[j] * c.S + lev0;
    double sj[6][kHq], pj[kHq];
    H mx[kHq], my[kHq], mz[kHq];
    ld4<VEC>(f.rho_t + nj, nv, sj[0]);
    ld4<VEC>(f.p_t + nj, nv, pj);
    ld4<VEC>(f.Mx_t + nj, nv, mx);
    ld4<VEC>(f.My_t + nj, nv, my);
    ld4<VEC>(f.Mz_t + nj, nv, mz);
    ld4<VEC>(f.wI + nj, nv, sj[5]);
    vel_temp<H>(c, sj[0], pj, mx, my, mz, sj[1], sj[2], sj[3], sj[4]);
    const double w = (double)lch[j];
    const H hx = dch[3 * (j + 1)], hy = dch[3 * (j + 1) + 1], hz = dch[3 * (j + 1) + 2];
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int q = 0; q < kHq; ++q) lap[k][q] += w * (sj[k][q] - s0[k][q]);
#pragma unroll
    for (int q = 0; q < kHq; ++q) dm[q] += hx * mx[q] + hy * my[q] + hz * mz[q];
  }
  {
    double l[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) l[q] = irc2[q] * lap[0][q];
    st4<VEC>(f.Xrho + idx, nv, l);
  }
  double *vdst[4] = {f.Xvx, f.Xvy, f.Xvz, f.XT};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double l[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) l[q] = rho[q] * Kd * irc2[q] * lap[k + 1][q];
    st4<VEC>(vdst[k] + idx, nv, l);
  }
  {
    double l[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const double rI = radius_i(c, lev);
      l[q] = lev == 0 ? 0.0 : rhoI[q] * Kd / (rI * rI) * lap[5][q];
    }
    st4<VEC>(f.Xw + idx, nv, l);
  }
  // 3D momentum divergence of Phi[t]
  {
    H Dt[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const double rC = radius_c(c, lev), rI = radius_i(c, lev);
      const double irc = 1.0 / rC;
      const double W1 = lev == L - 1 ? 0.0 : (q + 1 < kHq ? W[q + 1] : W_n);
      const double Wl = lev == 0 ? 0.0 : W[q];
      const double rI1 = rI + c.rdz;
      Dt[q] = (H)((double)dm[q] * irc + (rI1 * rI1 * W1 - rI * rI * Wl) * (irc * irc / c.dz));
    }
    st4<VEC>(f.Dt + idx, nv, Dt);
  }
}

template <typename H, bool VEC>
__device__ __forceinline__ void large2_cells(const Fields<H> &f, const Consts &c, const HLane &ln) {
  const int lev0 = ln.lev0, nv = ln.nv, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev0;
  const int lane = threadIdx.x & 63;
  const int lm = lane > 0 ? lane - 1 : 0;
  // p[t] and rho[t] of the level below the lane's first (every lane shuffles)
  const double p_m = shfl(f.p_t[idx + kHq - 1], lm), rho_m = shfl(f.rho_t[idx + kHq - 1], lm);
  if (!ln.store) return;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *lch = f.lc + (size_t)col * 6;
  double irc2[kHq];
#pragma unroll
  for (int q = 0; q < kHq; ++q) {
    const double rC = radius_c(c, lev0 + q);
    irc2[q] = 1.0 / (rC * rC);
  }
  {
    double l[kHq];
    lap4<VEC>(f.Xrho, nb, lch, c.S, lev0, nv, idx, l);
    H h[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) h[q] = (H)(-c.Kd * irc2[q] * l[q]);
    st4<VEC>(f.Hrho + idx, nv, h);
  }
  {
    const H *rh = f.rhat + (size_t)col * 3;
    const double rx = rh[0], ry = rh[1], rz = rh[2];
    // -grad p[t] (in double: full pressure), projected, in the horizontal
    // precision; the momentum hyperdiffusion is added to it below
    H fx[kHq], fy[kHq], fz[kHq];
    {
      const H *dch = f.dc + (size_t)col * 21;
      double p[kHq], gx[kHq], gy[kHq], gz[kHq];
      ld4<VEC>(f.p_t + idx, nv, p);
#pragma unroll
      for (int q = 0; q < kHq; ++q) gx[q] = gy[q] = gz[q] = 0;
#pragma unroll 2
      for (int j = 0; j < 6; ++j) {
        double pj[kHq];
        ld4<VEC>(f.p_t + (size_t)nb[j] * c.S + lev0, nv, pj);
        const double cx = dch[3 * (j + 1)], cy = dch[3 * (j + 1) + 1], cz = dch[3 * (j + 1) + 2];
#pragma unroll
        for (int q = 0; q < kHq; ++q) {
          const double dp = pj[q] - p[q];
          gx[q] += cx * dp;
          gy[q] += cy * dp;
          gz[q] += cz * dp;
        }
      }
#pragma unroll
      for (int q = 0; q < kHq; ++q) {
        const double irc = 1.0 / radius_c(c, lev0 + q);
        const double x = gx[q] * irc, y = gy[q] * irc, z = gz[q] * irc;
        const double gr = x * rx + y * ry + z * rz;
        fx[q] = (H)(-(x - gr * rx));
        fy[q] = (H)(-(y - gr * ry));
        fz[q] = (H)(-(z - gr * rz));
      }
    }
    double hx[kHq], hy[kHq], hz[kHq];
    lap4<VEC>(f.Xvx, nb, lch, c.S, lev0, nv, idx, hx);
    lap4<VEC>(f.Xvy, nb, lch, c.S, lev0, nv, idx, hy);
    lap4<VEC>(f.Xvz, nb, lch, c.S, lev0, nv, idx, hz);
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const double x = -irc2[q] * hx[q], y = -irc2[q] * hy[q], z = -irc2[q] * hz[q];
      const double hr = x * rx + y * ry + z * rz;
      fx[q] = (H)((double)fx[q] + (x - hr * rx));
      fy[q] = (H)((double)fy[q] + (y - hr * ry));
      fz[q] = (H)((double)fz[q] + (z - hr * rz));
    }
    st4<VEC>(f.FMx + idx, nv, fx);
    st4<VEC>(f.FMy + idx, nv, fy);
    st4<VEC>(f.FMz + idx, nv, fz);
  }
  {
    // the [t] vertical imbalance at interface lev plus the hyperdiffusion
    // of rho v_r
    double l[kHq], p[kHq], rho[kHq], fw[kHq];
    lap4<VEC>(f.Xw, nb, lch, c.S, lev0, nv, idx, l);
    ld4<VEC>(f.p_t + idx, nv, p);
    ld4<VEC>(f.rho_t + idx, nv, rho);
#pragma unroll
    for (int q = 0; q < kHq; ++q) {
      const int lev = lev0 + q;
      const double pm = q ? p[q - 1] : p_m, rm = q ? rho[q - 1] : rho_m;
      fw[q] = lev == 0 ? 0.0 : -(p[q] - pm) / c.dz - 0.5 * c.grav * (rm + rho[q]);
      const double rI = radius_i(c, lev);
      if (lev > 0) fw[q] += -l[q] / (rI * rI);
    }
    st4<VEC>(f.FW + idx, nv, fw);
  }
  {
    double l[kHq], rth[kHq], p[kHq];
    lap4<VEC>(f.XT, nb, lch, c.S, lev0, nv, idx, l);
    ld4<VEC>(f.rth_t + idx, nv, rth);
    ld4<VEC>(f.p_t + idx, nv, p);
    H h[kHq];
#pragma unroll
    for (int q = 0; q < kHq; ++q) h[q] = (H)(rth[q] / (c.gamma * p[q]) * (-c.Rd * irc2[q] * l[q]));
    st4<VEC>(f.Hrth + idx, nv, h);
  }
}

#define THOR_HBODY(NAME)                                                                       \
  template <typename H>                                                                      \
  __device__ __forceinline__ void b_##NAME(const Fields<H> &f, const Consts &c, const HLane &ln) { \
    NAME##_cells<H, true>(f, c, ln);   /* rows of stride S: whole groups of kHq */            \
  }
THOR_HBODY(large0)
THOR_HBODY(anel)
THOR_HBODY(large1)
THOR_HBODY(large2)
#undef THOR_HBODY

// Diagnostic field into f.diag (FP64, canonical layout [col][lev]).
template <typename H>
__device__ __forceinline__ void b_diag(const Fields<H> &f, const Consts &c, const Lane &ln, int field) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  const double W = lev == 0 ? 0.0 : f.W_t[idx];
  double W1 = shfl(W, lp);
  if (lev == L - 1) W1 = 0.0;
  if (!ln.store) return;
  const double rho = f.rho_t[idx];
  double out = 0.0;
  const H *rh = f.rhat + (size_t)col * 3;
  const double x = rh[0], y = rh[1], z = rh[2];
  if (field == THOR_F_T || field == THOR_F_P) {
    const double p = c.p_ref * powd(c.Rd * f.rth_t[idx] / c.p_ref, c.gamma);
    out = field == THOR_F_P ? p : p / (rho * c.Rd);
  } else if (field == THOR_F_U || field == THOR_F_V) {
    const double lam = (sqrt(x * x + y * y) < 1e-12) ? 0.0 : atan2(y, x);
    const double phi = asin(fmin(1.0, fmax(-1.0, z)));
    const double vx = (double)f.Mx_t[idx] / rho, vy = (double)f.My_t[idx] / rho, vz = (double)f.Mz_t[idx] / rho;
    if (field == THOR_F_U) out = -sin(lam) * vx + cos(lam) * vy;
    else out = -sin(phi) * cos(lam) * vx - sin(phi) * sin(lam) * vy + cos(phi) * vz;
  } else if (field == THOR_F_W) {
    out = 0.5 * (W + W1) / rho;
  } else if (field == THOR_F_RHO) {
    out = rho;
  } else if (field == THOR_F_RHOTHETA) {
    out = f.rth_t[idx];
  } else if (field == THOR_F_MX) {
    out = (double)f.Mx_t[idx];
  } else if (field == THOR_F_MY) {
    out = (double)f.My_t[idx];
  } else if (field == THOR_F_MZ) {
    out = (double)f.Mz_t[idx];
  } else {
    out = W;
  }
  f.diag[(size_t)col * L + lev] = out;
}

// Mass partial sums and a non-finite count per block (fixed reduction order).
template <typename H>
__global__ __launch_bounds__(256) void k_mass(Fields<H> f, Consts c) {
  __shared__ double sm[4][2];
  const Lane ln = map_lane(c, xcd_block());
  const int lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev;
  double m = 0.0, bad = 0.0;
  if (ln.store) {
    const double rC = radius_c(c, lev);
    const double rho = f.rho_t[idx];
    m = rho * f.area[col] * rC * rC * c.dz;
    const double chk = rho + f.rth_t[idx] + f.W_t[idx] + (double)f.Mx_t[idx] + (double)f.My_t[idx] +
                       (double)f.Mz_t[idx];
    bad = isfinite(chk) ? 0.0 : 1.0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    m += __shfl_down(m, o, 64);
    bad += __shfl_down(bad, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w][0] = m;
    sm[w][1] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b2 = 0.0;
    for (int i = 0; i < 4; ++i) {
      a += sm[i][0];
      b2 += sm[i][1];
    }
    f.partial[2 * blockIdx.x] = a;
    f.partial[2 * blockIdx.x + 1] = b2;
  }
}

// Total energy and mass partial sums per workgroup of one state, FP64, in a
// fixed reduction order.  which = 0: the large-step state Phi[t]; 1: the
// small-step state.  Per cell: internal energy Cv p / Rd, kinetic energy
// (|M|^2 + W_c^2) / (2 rho) with W_c the mean of the cell's two interface
// momenta (zero at the ground and the lid), potential energy rho g z; times
// the volume A_c r^2 dz.  out[2 b] = energy, out[2 b + 1] = mass.
template <typename H>
__global__ __launch_bounds__(256) void k_energy(Fields<H> f, Consts c, int which, double *out) {
  __shared__ double sm[4][2];
  const Lane ln = map_lane(c, xcd_block());
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * c.S + lev;
  const double *rho_a = which ? f.rho : f.rho_t;
  const double *rth_a = which ? f.rth : f.rth_t;
  const double *W_a = which ? f.W : f.W_t;
  const H *Mx = which ? f.Mx : f.Mx_t;
  const H *My = which ? f.My : f.My_t;
  const H *Mz = which ? f.Mz : f.Mz_t;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  const double W = lev == 0 ? 0.0 : W_a[idx];
  double W1 = shfl(W, lp);
  if (lev == L - 1) W1 = 0.0;
  double e = 0.0, m = 0.0;
  if (ln.store) {
    const double rC = radius_c(c, lev);
    const double vol = f.area[col] * rC * rC * c.dz;
    const double rho = rho_a[idx];
    const double p = c.p_ref * powd(c.Rd * rth_a[idx] / c.p_ref, c.gamma);
    const double mx = (double)Mx[idx], my = (double)My[idx], mz = (double)Mz[idx];
    const double wc = 0.5 * (W + W1);
    const double ke = 0.5 * (mx * mx + my * my + mz * mz + wc * wc) / rho;
    e = (c.Cv / c.Rd * p + ke + rho * c.grav * ((lev + 0.5) * c.dz)) * vol;
    m = rho * vol;
  }
  for (int o = 32; o > 0; o >>= 1) {
    e += __shfl_down(e, o, 64);
    m += __shfl_down(m, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w][0] = e;
    sm[w][1] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b2 = 0.0;
    for (int i = 0; i < 4; ++i) {
      a += sm[i][0];
      b2 += sm[i][1];
    }
    out[2 * blockIdx.x] = a;
    out[2 * blockIdx.x + 1] = b2;
  }
}

// One workgroup of 256: the totals of the partial sums of the step's start
// (pa) and of the dynamics output (pb), each in a fixed order, and the
// energy fixer's temperature increment dT = (E_a - E_b) / (Cv M_b) into *dT.
__global__ __launch_bounds__(256) void k_efix(const double *pa, const double *pb, int nb, double cv, double *dT) {
  __shared__ double sm[3][256];
  double ea = 0.0, eb = 0.0, mb = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    ea += pa[2 * i];
    eb += pb[2 * i];
    mb += pb[2 * i + 1];
  }
  sm[0][threadIdx.x] = ea;
  sm[1][threadIdx.x] = eb;
  sm[2][threadIdx.x] = mb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dT = (sm[0][0] - sm[1][0]) / (cv * sm[2][0]);
}

// Energy fixer and physics on the dynamics output: T += dT at every cell
// (at fixed density), then the physics of the configured forcing; for
// Held-Suarez, sigma of the fixed state goes to D for the friction kernel.
template <typename H>
__global__ __launch_bounds__(256) void k_fixphys(Fields<H> f, Consts c, const double *dT) {
  const Lane ln = map_lane(c, xcd_block());
  const size_t idx = (size_t)ln.col * c.S + ln.lev;
  const double rho = f.rho[idx];
  const double p0 = c.p_ref * powd(c.Rd * f.rth[idx] / c.p_ref, c.gamma);
  double p = rho * c.Rd * (p0 / (rho * c.Rd) + *dT);
  double sigma = 0.0;
  const int l0 = ln.lane - ln.lev;   // the column's lowest cell
  const double pl0 = shfl(p, l0), Tl0 = shfl(p / (rho * c.Rd), l0);
  p = physics_p(c, f.teq, ln.col, ln.lev, rho, p, pl0, Tl0, sigma);
  if (!ln.store) return;
  f.rth[idx] = c.p_ref / c.Rd * powd(p / c.p_ref, 1.0 / c.gamma);
  if (c.forcing == THOR_FORCING_HELD_SUAREZ) f.D[idx] = (H)sigma;
}

// Prognostic fields from a staged FP64 blob (checkpoint import; canonical
// [col][lev] layout).
template <typename H>
__device__ __forceinline__ void b_import(const Fields<H> &f, const Consts &c, const Lane &ln, const double *blob) {
  if (!ln.store) return;
  const size_t NL = (size_t)c.N * c.L;
  const size_t bi = (size_t)ln.col * c.L + ln.lev;
  const size_t idx = (size_t)ln.col * c.S + ln.lev;
  f.rho_t[idx] = blob[bi];
  f.Mx_t[idx] = (H)blob[NL + bi];
  f.My_t[idx] = (H)blob[2 * NL + bi];
  f.Mz_t[idx] = (H)blob[3 * NL + bi];
  f.rth_t[idx] = blob[4 * NL + bi];
  f.W_t[idx] = ln.lev == 0 ? 0.0 : blob[5 * NL + bi];
}

// OCC: minimum wavefronts per SIMD the register allocation must allow
// (caps VGPRs at 512 / OCC), chosen per kernel so that the gathers keep
// enough wavefronts in flight without spilling.
//
// k_NAME: one planet; kb_NAME: an ensemble, where logical workgroup b runs
// local workgroup tiles[b].y of planet tiles[b].x (x < 0: padding).  Both call
// the same body, so a planet computes bit-identical results either way.
#define THOR_KERNEL(NAME, OCC, MAP, PARAMS, ARGS)                                              \
  template <typename H>                                                                   \
  __global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(OCC)))       \
  void k_##NAME(Fields<H> f, Consts c PARAMS) {                                           \
    b_##NAME(f, c, MAP(c, xcd_block()) ARGS);                                        \
  }                                                                                       \
  template <typename H>                                                                   \
  __global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(OCC)))       \
  void kb_##NAME(const Planet<H> *P, const int2 *tiles, int parity PARAMS) {             \
    const int2 t = tiles[xcd_block()];                                                    \
    if (t.x < 0) return;                                                                  \
    const Fields<H> &f = P[t.x].f[parity];                                                \
    const Consts &c = P[t.x].c;                                                           \
    b_##NAME(f, c, MAP(c, t.y) ARGS);                                                \
  }
#define COMMA ,
THOR_KERNEL(slow, sizeof(H) == 8 ? 2 : 4, map_hlane, COMMA int from_t, COMMA from_t)
THOR_KERNEL(large0, 4, map_hlane, , )
THOR_KERNEL(anel, 8, map_hlane, , )
THOR_KERNEL(large1, sizeof(H) == 8 ? LARGE1_OCC_D : LARGE1_OCC_F, map_hlane, , )
THOR_KERNEL(large2, 4, map_hlane, , )
THOR_KERNEL(diag, 8, map_lane, COMMA int field, COMMA field)
THOR_KERNEL(import, 8, map_lane, COMMA const double *blob, COMMA blob)
THOR_KERNEL(friction, 8, map_hlane, , )
template <typename H>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? HMOM_OCC_D : HMOM_OCC_F, sizeof(H) == 8 ? HMOM_OCC_D : HMOM_OCC_F)))
void k_hmom(Fields<H> f, Consts c, int div, int first) {
  b_hmom<H, true>(f, c, map_hlane(c, xcd_block()), c.dt / div, first);
}
template <typename H>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? HMOM_OCC_D : HMOM_OCC_F, sizeof(H) == 8 ? HMOM_OCC_D : HMOM_OCC_F)))
void kb_hmom(const Planet<H> *P, const int2 *tiles, int parity, int div, int first) {
  const int2 t = tiles[xcd_block()];
  if (t.x < 0) return;
  const Fields<H> &f = P[t.x].f[parity];
  const Consts &c = P[t.x].c;
  b_hmom<H, false>(f, c, map_hlane(c, t.y), c.dt / div, first);
}
// slow terms of the shallow-atmosphere form and of the cubic vertical
// interpolation (single states only)
template <typename H, bool SHALLOW, int ORD>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? (SHALLOW && ORD == 3 ? 1 : 2) : (SHALLOW && ORD == 3 ? 2 : 3))))
void k_slow_var(Fields<H> f, Consts c, int from_t) {
  b_slow<H, SHALLOW, ORD>(f, c, map_hlane(c, xcd_block()), from_t);
}
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? 4 : (LAST ? 5 : 6))))
void k_vert(Fields<H> f, Consts c, int div, int first) {
  b_vert<H, LAST>(f, c, map_lane(c, xcd_block()), c.dt / div, first);
}
// phase V with two levels per lane (single states, 32 < L <= 64)
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? 2 : 3)))
void k_vert2(Fields<H> f, Consts c, int div, int first) {
  b_vert2<H, LAST>(f, c, map_lane2(c, xcd_block()), c.dt / div, first);
}
// phase V on the gather mapping (kHq levels per lane)
template <typename H, bool LAST, bool ANEL = false>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(VERT4_OCC)))
void k_vert4(Fields<H> f, Consts c, int div, int first) {
  b_vert4<H, LAST, ANEL>(f, c, map_vlane(c, xcd_block()), c.dt / div, first);
}
// phase V with the cubic interface theta (single states only)
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(sizeof(H) == 8 ? 3 : 4)))
void k_vert3(Fields<H> f, Consts c, int div, int first) {
  b_vert<H, LAST, 3>(f, c, map_lane(c, xcd_block()), c.dt / div, first);
}
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(VERT4_OCC)))
void kb_vert(const Planet<H> *P, const int2 *tiles, int parity, int div, int first) {
  const int2 t = tiles[xcd_block()];
  if (t.x < 0) return;
  const Fields<H> &f = P[t.x].f[parity];
  const Consts &c = P[t.x].c;
  b_vert4<H, LAST>(f, c, map_vlane(c, t.y), c.dt / div, first);
}
#undef COMMA
#undef THOR_KERNEL

}  // namespace

// One dispatch; with events (timing) they are recorded by the dispatch
// itself, at the kernel's start and end.
template <typename K, typename... Args>
void dispatch(K kernel, dim3 g, dim3 b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, g, b, 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, g, b, 0, s, args...);
}

template <typename H>
void launch_hmom(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, hipStream_t s, hipEvent_t ev0,
                 hipEvent_t ev1) {
  dispatch(k_hmom<H>, dim3(n_blocks_h(c, wpb)), dim3(64 * wpb), s, ev0, ev1, f, c, div, (int)first);
}
template <typename H>
void launch_vert(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, bool last, hipStream_t s,
                 hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 g(c.vnl == 4 ? n_blocks_h(c, wpb) : c.vnl == 2 ? n_blocks_for(c.N, c.vcpw, wpb) : n_blocks(c, wpb)),
      b(64 * wpb);
  const bool fr = last && c.forcing == THOR_FORCING_HELD_SUAREZ;
  hipEvent_t e1 = fr ? nullptr : ev1;   // with the friction kernel, the family ends with it
  if (last) {
    if (c.anelastic)
      dispatch(k_vert4<H, true, true>, g, b, s, ev0, e1, f, c, div, (int)first);
    else if (c.vnl == 4)
      dispatch(k_vert4<H, true>, g, b, s, ev0, e1, f, c, div, (int)first);
    else if (c.vnl == 2)
      dispatch(k_vert2<H, true>, g, b, s, ev0, e1, f, c, div, (int)first);
    else if (c.vorder == 3)
      dispatch(k_vert3<H, true>, g, b, s, ev0, e1, f, c, div, (int)first);
    else
      dispatch(k_vert<H, true>, g, b, s, ev0, e1, f, c, div, (int)first);
    if (fr) dispatch(k_friction<H>, dim3(n_blocks_h(c, 4)), dim3(256), s, nullptr, ev1, f, c);
  } else {
    if (c.anelastic)
      dispatch(k_vert4<H, false, true>, g, b, s, ev0, ev1, f, c, div, (int)first);
    else if (c.vnl == 4)
      dispatch(k_vert4<H, false>, g, b, s, ev0, ev1, f, c, div, (int)first);
    else if (c.vnl == 2)
      dispatch(k_vert2<H, false>, g, b, s, ev0, ev1, f, c, div, (int)first);
    else if (c.vorder == 3)
      dispatch(k_vert3<H, false>, g, b, s, ev0, ev1, f, c, div, (int)first);
    else
      dispatch(k_vert<H, false>, g, b, s, ev0, ev1, f, c, div, (int)first);
  }
}
template <typename H>
void launch_slow(const Fields<H> &f, const Consts &c, int wpb, bool from_t, hipStream_t s, hipEvent_t ev0,
                 hipEvent_t ev1) {
  const dim3 g(n_blocks_h(c, wpb)), b(64 * wpb);
  if (c.vorder == 3 && c.shallow)
    dispatch(k_slow_var<H, true, 3>, g, b, s, ev0, ev1, f, c, (int)from_t);
  else if (c.vorder == 3)
    dispatch(k_slow_var<H, false, 3>, g, b, s, ev0, ev1, f, c, (int)from_t);
  else if (c.shallow)
    dispatch(k_slow_var<H, true, 1>, g, b, s, ev0, ev1, f, c, (int)from_t);
  else
    dispatch(k_slow<H>, g, b, s, ev0, ev1, f, c, (int)from_t);
}
template <typename H>
void launch_large(const Fields<H> &f, const Consts &c, int wpb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 g(n_blocks_h(c, wpb)), b(64 * wpb);
  dispatch(k_large0<H>, g, b, s, ev0, nullptr, f, c);
  if (c.anelastic) dispatch(k_anel<H>, g, b, s, nullptr, nullptr, f, c);
  dispatch(k_large1<H>, g, b, s, nullptr, nullptr, f, c);
  dispatch(k_large2<H>, g, b, s, nullptr, ev1, f, c);
}
template <typename H>
void launch_diag_field(const Fields<H> &f, const Consts &c, int field, hipStream_t s) {
  hipLaunchKernelGGL(k_diag<H>, dim3(n_blocks(c, 4)), dim3(256), 0, s, f, c, field);
}
template <typename H>
void launch_mass(const Fields<H> &f, const Consts &c, hipStream_t s, int *nblocks_out) {
  *nblocks_out = n_blocks(c, 4);
  hipLaunchKernelGGL(k_mass<H>, dim3(n_blocks(c, 4)), dim3(256), 0, s, f, c);
}
template <typename H>
void launch_energy(const Fields<H> &f, const Consts &c, int which, double *out, hipStream_t s, int *nblocks_out) {
  *nblocks_out = n_blocks(c, 4);
  hipLaunchKernelGGL(k_energy<H>, dim3(n_blocks(c, 4)), dim3(256), 0, s, f, c, which, out);
}
template <typename H>
void launch_fixer(const Fields<H> &f, const Consts &c, hipStream_t s) {
  const int nb = n_blocks(c, 4);
  double *pa = f.epart, *pb = f.epart + 2 * (size_t)nb, *dT = f.epart + 4 * (size_t)nb;
  hipLaunchKernelGGL(k_energy<H>, dim3(nb), dim3(256), 0, s, f, c, 1, pb);
  hipLaunchKernelGGL(k_efix, dim3(1), dim3(256), 0, s, pa, pb, nb, c.Cv, dT);
  hipLaunchKernelGGL(k_fixphys<H>, dim3(nb), dim3(256), 0, s, f, c, (const double *)dT);
  if (c.forcing == THOR_FORCING_HELD_SUAREZ)
    hipLaunchKernelGGL(k_friction<H>, dim3(n_blocks_h(c, 4)), dim3(256), 0, s, f, c);
}
template <typename H>
void launch_to_state(const Fields<H> &f, const Consts &c, const double *blob, hipStream_t s) {
  hipLaunchKernelGGL(k_import<H>, dim3(n_blocks(c, 4)), dim3(256), 0, s, f, c, blob);
}

// Ensemble launchers: `tiles` holds n_tiles (multiple of kXcds) entries for
// workgroups of `wpb` wavefronts.
template <typename H>
void launch_batch(const Planet<H> *P, const int2 *tiles, int n_tiles, int wpb, int parity, BatchOp op,
                  int arg0, int arg1, hipStream_t s) {
  const dim3 g(n_tiles), b(64 * wpb);
  switch (op) {
    case BatchOp::Large:
      hipLaunchKernelGGL(kb_large0<H>, g, b, 0, s, P, tiles, parity);
      hipLaunchKernelGGL(kb_large1<H>, g, b, 0, s, P, tiles, parity);
      hipLaunchKernelGGL(kb_large2<H>, g, b, 0, s, P, tiles, parity);
      break;
    case BatchOp::Slow:
      hipLaunchKernelGGL(kb_slow<H>, g, b, 0, s, P, tiles, parity, arg0);
      break;
    case BatchOp::Hmom:
      hipLaunchKernelGGL(kb_hmom<H>, g, b, 0, s, P, tiles, parity, arg0, arg1);
      break;
    case BatchOp::Vert:
      hipLaunchKernelGGL((kb_vert<H, false>), g, b, 0, s, P, tiles, parity, arg0, arg1);
      break;
    case BatchOp::VertLast:
      hipLaunchKernelGGL((kb_vert<H, true>), g, b, 0, s, P, tiles, parity, arg0, arg1);
      // the friction of Held-Suarez members (a no-op for the others), same tiles
      hipLaunchKernelGGL(kb_friction<H>, g, b, 0, s, P, tiles, parity);
      break;
  }
}

#define THOR_INSTANTIATE(H)                                                                          \
  template void launch_hmom<H>(const Fields<H> &, const Consts &, int, int, bool, hipStream_t, hipEvent_t,   \
                               hipEvent_t);                                                          \
  template void launch_vert<H>(const Fields<H> &, const Consts &, int, int, bool, bool, hipStream_t,        \
                               hipEvent_t, hipEvent_t);                                              \
  template void launch_slow<H>(const Fields<H> &, const Consts &, int, bool, hipStream_t, hipEvent_t,       \
                               hipEvent_t);                                                          \
  template void launch_large<H>(const Fields<H> &, const Consts &, int, hipStream_t, hipEvent_t, hipEvent_t); \
  template void launch_diag_field<H>(const Fields<H> &, const Consts &, int, hipStream_t);           \
  template void launch_mass<H>(const Fields<H> &, const Consts &, hipStream_t, int *);               \
  template void launch_to_state<H>(const Fields<H> &, const Consts &, const double *, hipStream_t);  \
  template void launch_energy<H>(const Fields<H> &, const Consts &, int, double *, hipStream_t, int *); \
  template void launch_fixer<H>(const Fields<H> &, const Consts &, hipStream_t);                     \
  template void launch_batch<H>(const Planet<H> *, const int2 *, int, int, int, BatchOp, int, int,  \
                                hipStream_t);

THOR_INSTANTIATE(double)
THOR_INSTANTIATE(float)

}  // namespace thor
