// Device data layout and kernel launchers of the HEVI step (gfx950).
//
// Every field is stored [col][lev] with the levels of one column contiguous.
// A wavefront of 64 lanes covers cpw = floor(64 / L) whole columns, lane =
// col_in_wave * L + lev, so a neighbour gather reads one contiguous run of
// L values and the vertical solve of a column stays inside one wavefront.
// Interface fields (W) use the same layout: slot j holds interface j
// (0 = ground, always 0); the lid value (j = L) is 0 and not stored.
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
  const double *area;     // [N]
  const double *teq;      // [N] Newtonian target temperature

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
  double *Hrho, *Hrth;    // hyperdiffusion of rho and rho theta
  // stage forcing
  H *SMx, *SMy, *SMz;
  double *SW;
  H *thL, *Gam;           // linearisation theta and gamma p / rho theta
  // divergence damping
  H *D, *Gx, *Gy, *Gz;    // 3D divergence of the small-step state and its gradient
  H *Dt, *GDx, *GDy, *GDz;
  // large-step temporaries
  double *T, *vx, *vy, *vz, *wI;
  double *Xrho, *Xvx, *Xvy, *Xvz, *Xw, *XT;
  // diagnostics
  double *diag;           // [N][L]
  double *partial;        // per-block partial sums
};

struct Consts {
  int N, L, cpw;          // columns, levels, columns per wavefront
  double radius, omega, grav, Rd, Cp, Cv, gamma, p_ref;
  double dz, Kd;
  double dt;
  int div_damp;
  int forcing;
  double tau;
};

// Launch shape shared by all kernels: 256 threads (4 wavefronts).
constexpr int kBlock = 256;

inline int n_blocks(const Consts &c) {
  long waves = (c.N + c.cpw - 1) / c.cpw;
  return (int)((waves + 3) / 4);
}

// Per-substep launchers.  first = the first substep of an RK stage (the
// small-step state restarts from Phi[t], p* = 0).
template <typename H>
void launch_hmom(const Fields<H> &f, const Consts &c, double dtau, bool first, hipStream_t s);
template <typename H>
void launch_vert(const Fields<H> &f, const Consts &c, double dtau, bool first, hipStream_t s);
template <typename H>
void launch_graddiv(const Fields<H> &f, const Consts &c, hipStream_t s);
// Per stage.
template <typename H>
void launch_slow(const Fields<H> &f, const Consts &c, bool from_t, hipStream_t s);
// Per large step.
template <typename H>
void launch_large(const Fields<H> &f, const Consts &c, hipStream_t s);
template <typename H>
void launch_newton(const Fields<H> &f, const Consts &c, hipStream_t s);
// Diagnostics.
template <typename H>
void launch_diag_field(const Fields<H> &f, const Consts &c, int field, hipStream_t s);
template <typename H>
void launch_mass(const Fields<H> &f, const Consts &c, hipStream_t s, int *nblocks_out);
template <typename H>
void launch_to_state(const Fields<H> &f, const Consts &c, const double *blob, hipStream_t s);

}  // namespace thor
