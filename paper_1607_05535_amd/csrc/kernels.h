// Device data layout and kernel launchers of the HEVI step (gfx950).
//
// Every field is stored [col][lev] with the levels of one column contiguous.
// Interface fields (W) use the same layout: slot j holds interface j
// (0 = ground, always 0); the lid value (j = L) is 0 and not stored.
// Launch geometry: see n_blocks (lanes = levels, cpw columns per wavefront)
// and n_blocks_h (kHq levels per lane, hcpw columns per wavefront).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/thor.h"

namespace thor {

// Horizontal-field storage/arithmetic type: double (FP64 path) or float
// (mixed-precision form).  Vertical solve, reference state and prognostic
// density / rho-theta / W stay double in both.
template <typename H>
struct Fields {
  // geometry (per column)
  const int32_t *nbr;     // [N][6], -1 pad
  const H *dc;            // [N][21] divergence/gradient coefficient vectors
  const H *lc;            // [N][6]  Laplacian neighbour weights
  const H *rhat;          // [N][3]
  const int32_t *ddi;     // [N][18] two-ring columns (-1 pad)
  const H *ddw;           // [N][18][3] lap(grad .) weights
  const double *area;     // [N]
  const double *teq;      // [N] Newtonian T_eq; cos(lon - lon_ss) cos(lat) (hot Jupiter); sin(lat) (Held-Suarez)

  // current small-step state
  double *rho, *rth, *W;  // [N][L]
  H *Mx, *My, *Mz;        // [N][L]
  H *ps;                  // p* = p - p[t]
  // large-step copies Phi[t]
  double *rho_t, *rth_t, *W_t, *p_t;
  H *Mx_t, *My_t, *Mz_t;
  // large-step forcing (frozen over the step)
  H *FMx, *FMy, *FMz;     // proj_h(-grad p[t]) + hyperdiffusion of momentum
  double *FW;             // [t] vertical imbalance + hyperdiffusion of W
  H *Hrho, *Hrth;         // hyperdiffusion of rho and rho theta (horizontal stencils)
  // stage forcing
  H *SMx, *SMy, *SMz;
  double *SW;
  H *thL, *Gam;           // linearisation theta and gamma p / rho theta
  // divergence damping
  H *D;                   // 3D divergence of the small-step state
  H *Dt;                  // and of Phi[t]
  // large-step temporaries
  double *wI;             // w at the interfaces (W / rho_I) of Phi[t]
  double *Xrho, *Xvx, *Xvy, *Xvz, *Xw, *XT;
  // diagnostics
  double *diag;           // [N][L]
  double *partial;        // per-block partial sums
  double *epart;          // energy fixer: partial sums of the step's start and of
                          // the dynamics output, then the temperature increment
  // anelastic switch only (null otherwise): the reference column rho_r [S]
  // (padding levels repeat the top level) and, frozen per large step,
  // rho_r / rho[t] at the centres and the ratio of the two-point means at
  // interface slot j (slot 0, the ground, holds 1)
  const double *rref;
  H *fC;                  // [N][L]
  double *fI;             // [N][L]
};

struct Consts {
  int N, L, cpw;          // columns, levels, columns per wavefront
  int S;                  // row stride of the per-cell state arrays (L rounded up to a multiple of 4)
  int hlpc, hcpw;         // phase-M mapping: lanes per column, columns per wavefront
  double radius, omega, grav, Rd, Cp, Cv, gamma, p_ref;
  double dz, Kd;
  double rdz;             // radial spacing of the levels: dz, or 0 (shallow atmosphere)
  double dt;
  int div_damp;
  int energy_fixer;       // 1: uniform internal-energy fixer after the dynamics
  int hydrostatic;        // 1: no vertical acceleration in the acoustic substeps
  int shallow;            // 1: shallow atmosphere (r = radius), traditional Coriolis
  int vorder;             // order of the vertical Lagrange interpolation (1 or 3)
  int anelastic;          // 1: reference-density mass flux (needs vorder 1 and vnl 4)
  int vnl, vlpc, vcpw;    // phase V: levels per lane (1 or 2); with 2, lanes per column and columns per wavefront
  int forcing;
  double tau;
  // hot-Jupiter benchmark forcing (Eqs. teq-hj, btrop, tvert)
  double hj_Tsurf, hj_dTep, hj_lapse, hj_zstrat, hj_dTstrat, hj_sstrat;
  // Held-Suarez forcing (Eqs. im_eq_v, im_eq_fv; Sec. 7.1 T_eq, K_T)
  double hs_kf, hs_ka, hs_ks, hs_sb, hs_dTy, hs_dthz, hs_pstar, hs_Ttop, hs_Tmin;
};

// Workgroups have 1, 2, 4 or 8 wavefronts (tuned per kernel family).
constexpr int kMaxBlock = 512;
constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, one L2 each

// Launched workgroups of `wpb` wavefronts (a multiple of kXcds; surplus
// workgroups store nothing).
inline int n_blocks_for(long n_col, int cols_per_wave, int wpb) {
  long waves = (n_col + cols_per_wave - 1) / cols_per_wave;
  long wg = (waves + wpb - 1) / wpb;
  return (int)((wg + kXcds - 1) / kXcds * kXcds);
}
inline int n_blocks(const Consts &c, int wpb) { return n_blocks_for(c.N, c.cpw, wpb); }

// Kernels dominated by horizontal gathers (acoustic phase M, slow terms) use
// a second mapping: each lane owns kHq consecutive levels of one column,
// hlpc = ceil(L / kHq) lanes per column and hcpw = floor(64 / hlpc) columns
// per wavefront.  Per-column stencil weights are then loaded once per kHq
// cells, rows move in 16-byte loads, and a vertical neighbour is a register
// or, across a lane boundary, one shuffle.
constexpr int kHq = 4;
inline int n_blocks_h(const Consts &c, int wpb) { return n_blocks_for(c.N, c.hcpw, wpb); }

// Launchers.  `wpb` = wavefronts per workgroup (tuned per kernel family).
// The prognostic state between large steps lives in the *_t buffers; a large
// step reads them as Phi[t] and leaves its result in the unsuffixed buffers,
// after which the host swaps the two buffer sets.
// Acoustic substeps take dtau = dt / div (div = 3 in stage 1, n otherwise);
// first = first substep of an RK stage (restart from Phi[t], p* = 0);
// last = final substep of the large step (the physics is applied there).
// ev0 / ev1 (timing, may be null): events recorded by the dispatch itself
// when the family's first kernel starts and its last kernel ends.
template <typename H>
void launch_hmom(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, hipStream_t s,
                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename H>
void launch_vert(const Fields<H> &f, const Consts &c, int wpb, int div, bool first, bool last,
                 hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename H>
void launch_slow(const Fields<H> &f, const Consts &c, int wpb, bool from_t, hipStream_t s,
                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename H>
void launch_large(const Fields<H> &f, const Consts &c, int wpb, hipStream_t s, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);
template <typename H>
void launch_diag_field(const Fields<H> &f, const Consts &c, int field, hipStream_t s);
template <typename H>
void launch_mass(const Fields<H> &f, const Consts &c, hipStream_t s, int *nblocks_out);
template <typename H>
void launch_to_state(const Fields<H> &f, const Consts &c, const double *blob, hipStream_t s);
// Total energy and mass partial sums of the state Phi[t] (which = 0) or of
// the small-step state (which = 1) into out[2 b], out[2 b + 1].
template <typename H>
void launch_energy(const Fields<H> &f, const Consts &c, int which, double *out, hipStream_t s, int *nblocks_out);
// Partial sums (one per workgroup) of the absolute axial angular momentum of
// the state Phi[t] (postproc.hip).
template <typename H>
void launch_angmom(const Fields<H> &f, const Consts &c, double *out, hipStream_t s, int *nblocks_out);
// The energy fixer after the dynamics of a large step (the start's partial
// sums already in f.epart), followed by the physics: replaces the physics of
// the last phase V, which then runs with last = false.
template <typename H>
void launch_fixer(const Fields<H> &f, const Consts &c, hipStream_t s);

// One member of an ensemble as the device sees it.
template <typename H>
struct Planet {
  Fields<H> f[2];   // the two buffer-set orders (see thor_state)
  Consts c;
};

enum class BatchOp { Large, Slow, Hmom, Vert, VertLast };

// Every member of an ensemble in one launch per phase.  arg0/arg1: Slow:
// from_t; Hmom/Vert: div, first.
template <typename H>
void launch_batch(const Planet<H> *P, const int2 *tiles, int n_tiles, int wpb, int parity, BatchOp op,
                  int arg0, int arg1, hipStream_t s);

}  // namespace thor
