// HIP kernels of the HEVI dynamical-core step for gfx950 (MI355X).
//
// Paper: Mendonca et al. 2016 (arXiv:1607.05535), Sec. 2-5.
//
// Work mapping (all kernels): a 256-thread block is 4 wavefronts; wavefront
// w covers columns [w * cpw, w * cpw + cpw) with lane = (col - w cpw) * L + lev.
// Column data is contiguous in memory, so every neighbour gather is one
// coalesced run of L values per column, and the lanes of one column can
// exchange vertical neighbours with cross-lane shuffles.  The vertical
// implicit system of a column is solved entirely in registers by cyclic
// reduction across those lanes (ceil(log2 L) shuffle rounds), which is an
// exact direct solver of the same tridiagonal the Thomas algorithm solves.
//
// Horizontal stencils use folded coefficients built on the host:
//   div F = (1/r) sum_{j=0..6} c_j . F_j                   (Eqs. flx_div, int_grid, div_gauss)
//   grad s = (1/r) sum_{j=1..6} c_j (s_j - s_0)            (Eq. grad; the curvature term
//                                                           cancels the constant part)
//   lap s = (1/r^2) sum_{j=1..6} l_j (s_j - s_0)           (Sec. 4 triangle-gradient form)
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "kernels.h"

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
  return (H)(c.p_ref * pow(c.Rd * rth / c.p_ref, c.gamma));
}

__device__ __forceinline__ double radius_c(const Consts &c, int lev) { return c.radius + (lev + 0.5) * c.dz; }
__device__ __forceinline__ double radius_i(const Consts &c, int lev) { return c.radius + lev * c.dz; }

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

// (1/r) sum_j c_j (s_j - s_0): Eq. grad with folded coefficients.
template <typename H>
__device__ __forceinline__ void grad_at(const H *s, const int nb[6], const H *dc, int L, int lev,
                                        size_t idx, H ir, H &gx, H &gy, H &gz) {
  H s0 = s[idx];
  H x = 0, y = 0, z = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    H d = s[(size_t)nb[j] * L + lev] - s0;
    x += dc[3 * (j + 1) + 0] * d;
    y += dc[3 * (j + 1) + 1] * d;
    z += dc[3 * (j + 1) + 2] * d;
  }
  gx = x * ir;
  gy = y * ir;
  gz = z * ir;
}

// sum_j l_j (s_j - s_0): the Laplacian without its 1/r^2.
template <typename T, typename H>
__device__ __forceinline__ T lap_at(const T *s, const int nb[6], const H *lc, int L, int lev, size_t idx) {
  T s0 = s[idx];
  T acc = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) acc += (T)lc[j] * (s[(size_t)nb[j] * L + lev] - s0);
  return acc;
}

// ---------------------------------------------------------------------------
// Acoustic phase H: explicit horizontal momentum (Eq. mom2) with the
// deviation-pressure gradient, slow forcing and divergence damping, then the
// horizontal projection (Eq. proj_h).
// ---------------------------------------------------------------------------
template <typename H>
__device__ __forceinline__ void b_hmom(const Fields<H> &f, const Consts &c, const Lane &ln, double dtau, int first) {
  if (!ln.store) return;
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dc = f.dc + (size_t)col * 21;
  const H r = (H)radius_c(c, lev);
  const H ir = (H)1 / r;
  H gx = 0, gy = 0, gz = 0;
  if (!first) grad_at(f.ps, nb, dc, L, lev, idx, ir, gx, gy, gz);
  H ddx = 0, ddy = 0, ddz = 0;
  if (c.div_damp) {
    // -Kd lap(grad D) over the two-ring, D of the current small-step state
    const H *D = first ? f.Dt : f.D;
    const int32_t *di = f.ddi + (size_t)col * kRing2;
    const H *dw = f.ddw + (size_t)col * kRing2 * 3;
    const H d0 = D[idx];
#pragma unroll 6
    for (int m = 0; m < kRing2; ++m) {
      const int cm = di[m] < 0 ? col : di[m];
      const H dd = D[(size_t)cm * L + lev] - d0;
      ddx += dw[3 * m] * dd;
      ddy += dw[3 * m + 1] * dd;
      ddz += dw[3 * m + 2] * dd;
    }
    const H s = (H)(-c.Kd) * ir * ir * ir;
    ddx *= s;
    ddy *= s;
    ddz *= s;
  }
  const H *Mx = first ? f.Mx_t : f.Mx;
  const H *My = first ? f.My_t : f.My;
  const H *Mz = first ? f.Mz_t : f.Mz;
  const H dt = (H)dtau;
  H mx = Mx[idx] + dt * (-gx + f.SMx[idx] + ddx);
  H my = My[idx] + dt * (-gy + f.SMy[idx] + ddy);
  H mz = Mz[idx] + dt * (-gz + f.SMz[idx] + ddz);
  const H *rh = f.rhat + (size_t)col * 3;
  const H rx = rh[0], ry = rh[1], rz = rh[2];
  const H mr = mx * rx + my * ry + mz * rz;
  f.Mx[idx] = mx - mr * rx;
  f.My[idx] = my - mr * ry;
  f.Mz[idx] = mz - mr * rz;
}

// ---------------------------------------------------------------------------
// Acoustic phase V: horizontal mass and theta fluxes of the new momentum,
// then the HEVI vertical-momentum tridiagonal (Eqs. dens2, momr2, pt2
// combined), its solution, and the density / rho-theta updates with the new
// W; pressure from the nonlinear equation of state (Eq. theta_to_p).
// ---------------------------------------------------------------------------
template <typename H, bool LAST>
__device__ __forceinline__ void b_vert(const Fields<H> &f, const Consts &c, const Lane &ln, double dtau, int first) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
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
      size_t nj = (size_t)nb[j] * L + lev;
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
  const double Hrth = f.Hrth[idx];
  const double rho_hat = rho0 + dtau * (-Drho + f.Hrho[idx]);
  const double rth_hat = rth0 + dtau * (-Dth + Hrth);
  const double phs = ps_in + dtau * gam * (-Dth + Hrth);   // p-hat minus p[t]
  const double rhs = rho_hat - f.rho_t[idx];              // rho-hat minus rho[t]

  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  const double thI = 0.5 * (shfl(thC, lm) + thC);   // theta at interface lev
  const double thI_m = shfl(thI, lm);
  const double thI_p = shfl(thI, lp);
  const double gam_m = shfl(gam, lm);
  const double phs_m = shfl(phs, lm);
  const double rhs_m = shfl(rhs, lm);

  const double dz = c.dz;
  const double rI = radius_i(c, lev), rI1 = rI + dz, rIm = rI - dz;
  const double rC = radius_c(c, lev), rCm = rC - dz;
  const double ap = dtau * rI1 * rI1 / (rC * rC * dz);     // alpha+ of cell lev
  const double am = dtau * rI * rI / (rC * rC * dz);       // alpha- of cell lev
  const double ap_m = dtau * rI * rI / (rCm * rCm * dz);   // alpha+ of cell lev-1
  const double am_m = dtau * rIm * rIm / (rCm * rCm * dz); // alpha- of cell lev-1
  const double c1 = dtau / dz, c2 = 0.5 * c.grav * dtau;

  double a = 0.0, b = 1.0, cc = 0.0, d = 0.0;
  if (ln.real_col && lev > 0) {
    a = lev == 1 ? 0.0 : -c1 * gam_m * am_m * thI_m + c2 * am_m;
    b = 1.0 + c1 * thI * (gam * am + gam_m * ap_m) + c2 * (am - ap_m);
    cc = lev == L - 1 ? 0.0 : -c1 * gam * ap * thI_p - c2 * ap;
    d = Wj + dtau * f.SW[idx] - c1 * (phs - phs_m) - c2 * (rhs_m + rhs);
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
  double p = c.p_ref * pow(c.Rd * rth_new / c.p_ref, c.gamma);
  if (LAST && c.forcing == THOR_FORCING_NEWTONIAN) {
    // physics after the dynamics (Eq. im_eq_t, K_T = 1/tau) at fixed density
    const double kt = c.dt / c.tau;
    const double T = p / (rho_new * c.Rd);
    const double Tn = (T + kt * f.teq[col]) / (1.0 + kt);
    p = rho_new * c.Rd * Tn;
    rth_new = c.p_ref / c.Rd * pow(p / c.p_ref, 1.0 / c.gamma);
  }
  const double D3 = Drho + (rI1 * rI1 * Wp - rI * rI * Wn) / (rC * rC * dz);
  if (ln.store) {
    f.rho[idx] = rho_new;
    f.rth[idx] = rth_new;
    f.W[idx] = Wn;
    f.ps[idx] = (H)(p - pt);
    f.D[idx] = (H)D3;
  }
}

// ---------------------------------------------------------------------------
// Slow terms of one RK stage at the previous stage state: advection of the
// full Cartesian momentum, Coriolis, projections (Eqs. mom, proj_h, proj_r),
// and the linearisation coefficients theta_L and gamma p / (rho theta).
// ---------------------------------------------------------------------------
template <typename H>
__device__ __forceinline__ void b_slow(const Fields<H> &f, const Consts &c, const Lane &ln, int from_t) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
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

  // own column: full momentum m = M + Wbar rhat and velocity m / rho
  const double Wk = lev == 0 ? 0.0 : W[idx];
  double Wk1 = shfl(Wk, lp);
  if (lev == L - 1) Wk1 = 0.0;
  const H wbar = (H)(0.5 * (Wk + Wk1));
  const H rho0 = (H)rho[idx];
  const H mx0 = Mx[idx], my0 = My[idx], mz0 = Mz[idx];
  const H fx = mx0 + wbar * rx, fy = my0 + wbar * ry, fz = mz0 + wbar * rz;
  const H irho0 = (H)1 / rho0;
  const H vx0 = fx * irho0, vy0 = fy * irho0, vz0 = fz * irho0;
  // horizontal flux divergence of v_q M
  H Ax, Ay, Az;
  {
    H t = dc[0] * mx0 + dc[1] * my0 + dc[2] * mz0;
    Ax = vx0 * t;
    Ay = vy0 * t;
    Az = vz0 * t;
  }
#pragma unroll 2
  for (int j = 0; j < 6; ++j) {
    const size_t nj = (size_t)nb[j] * L + lev;
    const double wn = lev == 0 ? 0.0 : W[nj];
    double wn1 = shfl(wn, lp);
    if (lev == L - 1) wn1 = 0.0;
    const H wb = (H)(0.5 * (wn + wn1));
    const H *rn = f.rhat + (size_t)nb[j] * 3;
    const H mxj = Mx[nj], myj = My[nj], mzj = Mz[nj];
    const H t = (dc[3 * (j + 1)] * mxj + dc[3 * (j + 1) + 1] * myj + dc[3 * (j + 1) + 2] * mzj) /
                (H)rho[nj];
    Ax += (mxj + wb * rn[0]) * t;
    Ay += (myj + wb * rn[1]) * t;
    Az += (mzj + wb * rn[2]) * t;
  }
  const H rC = (H)radius_c(c, lev);
  Ax /= rC;
  Ay /= rC;
  Az /= rC;
  // vertical flux divergence: r^2 W v_q at the interfaces
  {
    const H rI = (H)radius_i(c, lev);
    const H w2 = (H)Wk * rI * rI * (H)0.5;
    const H vxm = shfl(vx0, lm), vym = shfl(vy0, lm), vzm = shfl(vz0, lm);
    const H Fx = lev == 0 ? (H)0 : w2 * (vxm + vx0);
    const H Fy = lev == 0 ? (H)0 : w2 * (vym + vy0);
    const H Fz = lev == 0 ? (H)0 : w2 * (vzm + vz0);
    H Fx1 = shfl(Fx, lp), Fy1 = shfl(Fy, lp), Fz1 = shfl(Fz, lp);
    if (lev == L - 1) Fx1 = Fy1 = Fz1 = 0;
    const H s = (H)1 / (rC * rC * (H)c.dz);
    Ax += (Fx1 - Fx) * s;
    Ay += (Fy1 - Fy) * s;
    Az += (Fz1 - Fz) * s;
  }
  // Coriolis 2 Omega zhat x m
  const H om2 = (H)(2.0 * c.omega);
  const H ACx = Ax - om2 * fy, ACy = Ay + om2 * fx, ACz = Az;
  const H acr = ACx * rx + ACy * ry + ACz * rz;
  const H acr_m = shfl(acr, lm);
  // linearisation coefficients
  const double rth0 = rth[idx];
  const double p0 = f.p_t[idx] + (from_t ? 0.0 : (double)f.ps[idx]);
  if (ln.store) {
    f.SMx[idx] = f.FMx[idx] - (ACx - acr * rx);
    f.SMy[idx] = f.FMy[idx] - (ACy - acr * ry);
    f.SMz[idx] = f.FMz[idx] - (ACz - acr * rz);
    f.SW[idx] = lev == 0 ? 0.0 : f.FW[idx] - 0.5 * ((double)acr_m + (double)acr);
    f.thL[idx] = (H)(rth0 / (double)rho[idx]);
    f.Gam[idx] = (H)(c.gamma * p0 / rth0);
  }
}

// ---------------------------------------------------------------------------
// Per large step: keep Phi[t], diagnose p[t], T, v and w (pointwise), then
// two Laplacian passes for the hyperdiffusion (Eqs. diff_rho ... diff_p),
// grad p[t], the [t] vertical imbalance and the divergence-damping terms of
// Phi[t].
// ---------------------------------------------------------------------------
template <typename H>
__device__ __forceinline__ void b_large0(const Fields<H> &f, const Consts &c, const Lane &ln) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const double rho = f.rho_t[idx], rth = f.rth_t[idx];
  const double W = lev == 0 ? 0.0 : f.W_t[idx];
  const double rho_m = shfl(rho, lm);
  const double p = c.p_ref * pow(c.Rd * rth / c.p_ref, c.gamma);
  if (!ln.store) return;
  const double irho = 1.0 / rho;
  f.p_t[idx] = p;
  f.T[idx] = p * irho / c.Rd;
  f.vx[idx] = (double)f.Mx_t[idx] * irho;
  f.vy[idx] = (double)f.My_t[idx] * irho;
  f.vz[idx] = (double)f.Mz_t[idx] * irho;
  f.wI[idx] = lev == 0 ? 0.0 : W / (0.5 * (rho_m + rho));
}

template <typename H>
__device__ __forceinline__ void b_large1(const Fields<H> &f, const Consts &c, const Lane &ln) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *dch = f.dc + (size_t)col * 21;
  const H *lch = f.lc + (size_t)col * 6;
  const double rho = f.rho_t[idx];
  const double rho_m = shfl(rho, lm);
  const double p = f.p_t[idx];
  const double p_m = shfl(p, lm);
  const double W = f.W_t[idx];
  double W1 = shfl(W, lp);
  if (lev == L - 1) W1 = 0.0;
  if (!ln.store) return;
  const double rC = radius_c(c, lev), rI = radius_i(c, lev);
  const double Kd = c.Kd;
  const double irc2 = 1.0 / (rC * rC);
  f.Xrho[idx] = irc2 * lap_at(f.rho_t, nb, lch, L, lev, idx);
  f.Xvx[idx] = rho * Kd * irc2 * lap_at(f.vx, nb, lch, L, lev, idx);
  f.Xvy[idx] = rho * Kd * irc2 * lap_at(f.vy, nb, lch, L, lev, idx);
  f.Xvz[idx] = rho * Kd * irc2 * lap_at(f.vz, nb, lch, L, lev, idx);
  f.XT[idx] = rho * Kd * irc2 * lap_at(f.T, nb, lch, L, lev, idx);
  f.Xw[idx] = lev == 0 ? 0.0
                       : 0.5 * (rho_m + rho) * Kd / (rI * rI) * lap_at(f.wI, nb, lch, L, lev, idx);
  // grad p[t] (in double: full pressure), projected
  double gx = 0, gy = 0, gz = 0;
  {
    const double *pp = f.p_t;
    for (int j = 0; j < 6; ++j) {
      double dp = pp[(size_t)nb[j] * L + lev] - p;
      gx += (double)dch[3 * (j + 1)] * dp;
      gy += (double)dch[3 * (j + 1) + 1] * dp;
      gz += (double)dch[3 * (j + 1) + 2] * dp;
    }
    gx /= rC;
    gy /= rC;
    gz /= rC;
  }
  const H *rh = f.rhat + (size_t)col * 3;
  const double rx = rh[0], ry = rh[1], rz = rh[2];
  const double gr = gx * rx + gy * ry + gz * rz;
  f.FMx[idx] = (H)(-(gx - gr * rx));
  f.FMy[idx] = (H)(-(gy - gr * ry));
  f.FMz[idx] = (H)(-(gz - gr * rz));
  // 3D momentum divergence of Phi[t]
  H dm = dch[0] * f.Mx_t[idx] + dch[1] * f.My_t[idx] + dch[2] * f.Mz_t[idx];
  for (int j = 0; j < 6; ++j) {
    size_t nj = (size_t)nb[j] * L + lev;
    dm += dch[3 * (j + 1)] * f.Mx_t[nj] + dch[3 * (j + 1) + 1] * f.My_t[nj] +
          dch[3 * (j + 1) + 2] * f.Mz_t[nj];
  }
  const double Wl = lev == 0 ? 0.0 : W;
  f.Dt[idx] = (H)((double)dm / rC + ((rI + c.dz) * (rI + c.dz) * W1 - rI * rI * Wl) / (rC * rC * c.dz));
  // [t] vertical imbalance at interface lev
  f.FW[idx] = lev == 0 ? 0.0 : -(p - p_m) / c.dz - 0.5 * c.grav * (rho_m + rho);
}

template <typename H>
__device__ __forceinline__ void b_large2(const Fields<H> &f, const Consts &c, const Lane &ln) {
  if (!ln.store) return;
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
  int nb[6];
  load_nbr(f.nbr, col, nb);
  const H *lch = f.lc + (size_t)col * 6;
  const double rC = radius_c(c, lev), rI = radius_i(c, lev);
  const double irc2 = 1.0 / (rC * rC);
  f.Hrho[idx] = -c.Kd * irc2 * lap_at(f.Xrho, nb, lch, L, lev, idx);
  double hx = -irc2 * lap_at(f.Xvx, nb, lch, L, lev, idx);
  double hy = -irc2 * lap_at(f.Xvy, nb, lch, L, lev, idx);
  double hz = -irc2 * lap_at(f.Xvz, nb, lch, L, lev, idx);
  const H *rh = f.rhat + (size_t)col * 3;
  const double rx = rh[0], ry = rh[1], rz = rh[2];
  const double hr = hx * rx + hy * ry + hz * rz;
  f.FMx[idx] = (H)((double)f.FMx[idx] + (hx - hr * rx));
  f.FMy[idx] = (H)((double)f.FMy[idx] + (hy - hr * ry));
  f.FMz[idx] = (H)((double)f.FMz[idx] + (hz - hr * rz));
  if (lev > 0) f.FW[idx] += -lap_at(f.Xw, nb, lch, L, lev, idx) / (rI * rI);
  const double rth = f.rth_t[idx], p = f.p_t[idx];
  f.Hrth[idx] = rth / (c.gamma * p) * (-c.Rd * irc2 * lap_at(f.XT, nb, lch, L, lev, idx));
}

// Diagnostic field into f.diag (FP64, canonical layout).
template <typename H>
__device__ __forceinline__ void b_diag(const Fields<H> &f, const Consts &c, const Lane &ln, int field) {
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
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
    const double p = c.p_ref * pow(c.Rd * f.rth_t[idx] / c.p_ref, c.gamma);
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
  f.diag[idx] = out;
}

// Mass partial sums and a non-finite count per block (fixed reduction order).
template <typename H>
__global__ __launch_bounds__(256) void k_mass(Fields<H> f, Consts c) {
  __shared__ double sm[4][2];
  const Lane ln = map_lane(c, xcd_block());
  const int L = c.L, lev = ln.lev, col = ln.col;
  const size_t idx = (size_t)col * L + lev;
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

// Prognostic fields from a staged FP64 blob (checkpoint import).
template <typename H>
__device__ __forceinline__ void b_import(const Fields<H> &f, const Consts &c, const Lane &ln, const double *blob) {
  if (!ln.store) return;
  const size_t NL = (size_t)c.N * c.L;
  const size_t idx = (size_t)ln.col * c.L + ln.lev;
  f.rho_t[idx] = blob[idx];
  f.Mx_t[idx] = (H)blob[NL + idx];
  f.My_t[idx] = (H)blob[2 * NL + idx];
  f.Mz_t[idx] = (H)blob[3 * NL + idx];
  f.rth_t[idx] = blob[4 * NL + idx];
  f.W_t[idx] = ln.lev == 0 ? 0.0 : blob[5 * NL + idx];
}

// OCC: minimum wavefronts per SIMD the register allocation must allow
// (caps VGPRs at 512 / OCC), chosen per kernel so that the gathers keep
// enough wavefronts in flight without spilling.
//
// k_NAME: one planet; kb_NAME: an ensemble, where logical workgroup b runs
// local workgroup tiles[b].y of planet tiles[b].x (x < 0: padding).  Both call
// the same body, so a planet computes bit-identical results either way.
#define THOR_KERNEL(NAME, OCC, PARAMS, ARGS)                                              \
  template <typename H>                                                                   \
  __global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(OCC)))       \
  void k_##NAME(Fields<H> f, Consts c PARAMS) {                                           \
    b_##NAME(f, c, map_lane(c, xcd_block()) ARGS);                                        \
  }                                                                                       \
  template <typename H>                                                                   \
  __global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(OCC)))       \
  void kb_##NAME(const Planet<H> *P, const int2 *tiles, int parity PARAMS) {             \
    const int2 t = tiles[xcd_block()];                                                    \
    if (t.x < 0) return;                                                                  \
    const Fields<H> &f = P[t.x].f[parity];                                                \
    const Consts &c = P[t.x].c;                                                           \
    b_##NAME(f, c, map_lane(c, t.y) ARGS);                                                \
  }
#define COMMA ,
THOR_KERNEL(hmom, 6, COMMA int div COMMA int first, COMMA c.dt / div COMMA first)
THOR_KERNEL(slow, 4, COMMA int from_t, COMMA from_t)
THOR_KERNEL(large0, 8, , )
THOR_KERNEL(large1, 4, , )
THOR_KERNEL(large2, 5, , )
THOR_KERNEL(diag, 8, COMMA int field, COMMA field)
THOR_KERNEL(import, 8, COMMA const double *blob, COMMA blob)
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_vert(Fields<H> f, Consts c, int div, int first) {
  b_vert<H, LAST>(f, c, map_lane(c, xcd_block()), c.dt / div, first);
}
template <typename H, bool LAST>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4)))
void kb_vert(const Planet<H> *P, const int2 *tiles, int parity, int div, int first) {
  const int2 t = tiles[xcd_block()];
  if (t.x < 0) return;
  const Fields<H> &f = P[t.x].f[parity];
  const Consts &c = P[t.x].c;
  b_vert<H, LAST>(f, c, map_lane(c, t.y), c.dt / div, first);
}
#undef COMMA
#undef THOR_KERNEL

}  // namespace

template <typename H>
void launch_hmom(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, hipStream_t s) {
  hipLaunchKernelGGL(k_hmom<H>, dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c, div, (int)first);
}
template <typename H>
void launch_vert(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, bool last,
                 hipStream_t s) {
  if (last)
    hipLaunchKernelGGL((k_vert<H, true>), dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c, div, (int)first);
  else
    hipLaunchKernelGGL((k_vert<H, false>), dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c, div, (int)first);
}
template <typename H>
void launch_slow(const Fields<H> &f, const Consts &c, int wpb, bool from_t, hipStream_t s) {
  hipLaunchKernelGGL(k_slow<H>, dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c, (int)from_t);
}
template <typename H>
void launch_large(const Fields<H> &f, const Consts &c, int wpb, hipStream_t s) {
  hipLaunchKernelGGL(k_large0<H>, dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c);
  hipLaunchKernelGGL(k_large1<H>, dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c);
  hipLaunchKernelGGL(k_large2<H>, dim3(n_blocks(c, wpb)), dim3(64 * wpb), 0, s, f, c);
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
      break;
  }
}

#define THOR_INSTANTIATE(H)                                                                          \
  template void launch_hmom<H>(const Fields<H> &, const Consts &, int, int, bool, hipStream_t);      \
  template void launch_vert<H>(const Fields<H> &, const Consts &, int, int, bool, bool, hipStream_t); \
  template void launch_slow<H>(const Fields<H> &, const Consts &, int, bool, hipStream_t);           \
  template void launch_large<H>(const Fields<H> &, const Consts &, int, hipStream_t);                \
  template void launch_diag_field<H>(const Fields<H> &, const Consts &, int, hipStream_t);           \
  template void launch_mass<H>(const Fields<H> &, const Consts &, hipStream_t, int *);               \
  template void launch_to_state<H>(const Fields<H> &, const Consts &, const double *, hipStream_t);  \
  template void launch_batch<H>(const Planet<H> *, const int2 *, int, int, int, BatchOp, int, int,  \
                                hipStream_t);

THOR_INSTANTIATE(double)
THOR_INSTANTIATE(float)

}  // namespace thor
