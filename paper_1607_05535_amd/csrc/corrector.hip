// Learned per-column corrector around the HEVI step: restriction of a fine
// state onto a coarse grid, per-cell (T, u, v, w, p) extraction, network
// inputs (a column and its 5-6 neighbours), training batches from stored
// coarse/fine pairs, and the bounded application of the predicted
// correction to a coarse state.
//
// Network input of column c: x[(s * 5 + f) * L + k], s = 0 the column, s = 1..6
// its neighbours (a pentagon repeats itself in slot 6), f over (T, u, v, w, p),
// k over levels, each normalised by a mean and spread per (field, level).  Output:
// y[f * L + k], the normalised correction of field f at level k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "powd.h"
#include "state.h"

namespace thor {
namespace {

constexpr int kF = 5;   // T, u, v, w, p

struct CLane {
  int lane, lev, col;
  bool store;
};

// Same wavefront mapping as the dynamics: floor(64 / L) columns per
// wavefront, lanes = levels.
__device__ __forceinline__ CLane clane(int N, int L) {
  CLane r;
  r.lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int cpw = 64 / L;
  const int cw = r.lane / L;
  r.lev = r.lane - cw * L;
  const int col = wave * cpw + cw;
  r.store = cw < cpw && col < N;
  r.col = col < N ? col : N - 1;
  return r;
}

inline unsigned cblocks(int N, int L) {
  const int cpw = 64 / L;
  const long waves = (N + cpw - 1) / cpw;
  return (unsigned)((waves + 3) / 4);
}

__device__ __forceinline__ void east_north(double x, double y, double z, double e[3], double n[3]) {
  const double lam = sqrt(x * x + y * y) < 1e-12 ? 0.0 : atan2(y, x);
  const double phi = asin(fmin(1.0, fmax(-1.0, z)));
  e[0] = -sin(lam);
  e[1] = cos(lam);
  e[2] = 0.0;
  n[0] = -sin(phi) * cos(lam);
  n[1] = -sin(phi) * sin(lam);
  n[2] = cos(phi);
}

// (T, u, v, w, p) of every cell of the state (FP32, [f][col][lev]).
template <typename H>
__global__ __launch_bounds__(256) void k_fields(Fields<H> f, Consts c, float *out) {
  const CLane ln = clane(c.N, c.L);
  const int L = c.L;
  const size_t idx = (size_t)ln.col * c.S + ln.lev;   // state (row stride S)
  const size_t oi = (size_t)ln.col * L + ln.lev;      // output, [f][col][lev]
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  const double W = ln.lev == 0 ? 0.0 : f.W_t[idx];
  double W1 = __shfl(W, lp, 64);
  if (ln.lev == L - 1) W1 = 0.0;
  if (!ln.store) return;
  const double rho = f.rho_t[idx];
  const double p = c.p_ref * powd(c.Rd * f.rth_t[idx] / c.p_ref, c.gamma);
  const H *rh = f.rhat + (size_t)ln.col * 3;
  double e[3], n[3];
  east_north(rh[0], rh[1], rh[2], e, n);
  const double vx = (double)f.Mx_t[idx] / rho, vy = (double)f.My_t[idx] / rho, vz = (double)f.Mz_t[idx] / rho;
  const size_t NL = (size_t)c.N * L;
  out[oi] = (float)(p / (rho * c.Rd));
  out[NL + oi] = (float)(e[0] * vx + e[1] * vy + e[2] * vz);
  out[2 * NL + oi] = (float)(n[0] * vx + n[1] * vy + n[2] * vz);
  out[3 * NL + oi] = (float)(0.5 * (W + W1) / rho);
  out[4 * NL + oi] = (float)p;
}

// Coarse state from a fine one: area-weighted T and p, mass-weighted
// velocity (Cartesian, projected on the coarse tangent plane), over the fine
// columns listed for each coarse column.  Writes the coarse *_t buffers.
template <typename H>
__global__ __launch_bounds__(256) void k_restrict(Fields<H> ff, Consts cf, Fields<H> fc, Consts cc,
                                                  const int32_t *off, const int32_t *list) {
  const CLane ln = clane(cc.N, cc.L);
  const int L = cc.L;
  const int lp = ln.lane < 63 ? ln.lane + 1 : 63;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  double sA = 0, sT = 0, sp = 0, sM = 0, smx = 0, smy = 0, smz = 0, smw = 0;
  const int a = off[ln.col], b = off[ln.col + 1];
  for (int i = a; i < b; ++i) {
    const int fcol = list[i];
    const size_t fi = (size_t)fcol * cf.S + ln.lev;
    const double W = ln.lev == 0 ? 0.0 : ff.W_t[fi];
    double W1 = __shfl(W, lp, 64);
    if (ln.lev == L - 1) W1 = 0.0;
    const double A = ff.area[fcol];
    const double rho = ff.rho_t[fi];
    const double p = cf.p_ref * powd(cf.Rd * ff.rth_t[fi] / cf.p_ref, cf.gamma);
    sA += A;
    sT += A * p / (rho * cf.Rd);
    sp += A * p;
    sM += A * rho;
    smx += A * (double)ff.Mx_t[fi];
    smy += A * (double)ff.My_t[fi];
    smz += A * (double)ff.Mz_t[fi];
    smw += A * 0.5 * (W + W1);
  }
  const double T = sT / sA, p = sp / sA;
  const double rho = p / (cc.Rd * T);
  const H *rh = fc.rhat + (size_t)ln.col * 3;
  const double rx = rh[0], ry = rh[1], rz = rh[2];
  double vx = smx / sM, vy = smy / sM, vz = smz / sM;
  const double vr = vx * rx + vy * ry + vz * rz;
  vx -= vr * rx;
  vy -= vr * ry;
  vz -= vr * rz;
  const double mw = rho * (smw / sM);   // rho w at the centre
  const double mw_m = __shfl(mw, lm, 64);
  if (!ln.store) return;
  const size_t ci = (size_t)ln.col * cc.S + ln.lev;
  fc.rho_t[ci] = rho;
  fc.rth_t[ci] = cc.p_ref / cc.Rd * powd(p / cc.p_ref, 1.0 / cc.gamma);
  fc.Mx_t[ci] = (H)(rho * vx);
  fc.My_t[ci] = (H)(rho * vy);
  fc.Mz_t[ci] = (H)(rho * vz);
  fc.W_t[ci] = ln.lev == 0 ? 0.0 : 0.5 * (mw_m + mw);
}

__device__ __forceinline__ int slot_col(const int32_t *nbr, int col, int s) {
  if (s == 0) return col;
  const int v = nbr[(size_t)col * 6 + s - 1];
  return v < 0 ? col : v;
}

// Network inputs of every column from a fields array [f][col][lev].
__global__ void k_features(const float *F, const int32_t *nbr, const float *norm, __bf16 *X, int N, int L) {
  const size_t n_in = (size_t)7 * kF * L;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)N * n_in) return;
  const int col = (int)(i / n_in);
  const int r = (int)(i % n_in);
  const int s = r / (kF * L), f = (r / L) % kF, k = r % L;
  const int src = slot_col(nbr, col, s);
  const float v = F[((size_t)f * N + src) * L + k];
  const int q = f * L + k;
  X[i] = (__bf16)((v - norm[q]) / norm[kF * L + q]);
}

// Training batch: row b is column cols[b] of pair pairs[b]; inputs from the
// coarse fields, targets = normalised (fine - coarse).
__global__ void k_batch(const float *C, const float *Fn, size_t pair_stride, const int32_t *pairs,
                        const int32_t *cols, const int32_t *nbr, const float *norm, __bf16 *X, float *T, int B,
                        int N, int L) {
  const size_t n_in = (size_t)7 * kF * L, n_out = (size_t)kF * L;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)B * (n_in + n_out)) return;
  const int b = (int)(i / (n_in + n_out));
  const int r = (int)(i % (n_in + n_out));
  const size_t base = (size_t)pairs[b] * pair_stride;
  const int col = cols[b];
  if (r < (int)n_in) {
    const int s = r / (kF * L), f = (r / L) % kF, k = r % L;
    const int src = slot_col(nbr, col, s);
    const float v = C[base + ((size_t)f * N + src) * L + k];
    const int q = f * L + k;
    X[(size_t)b * n_in + r] = (__bf16)((v - norm[q]) / norm[kF * L + q]);
  } else {
    const int q = r - (int)n_in, f = q / L, k = q % L;
    const size_t j = base + ((size_t)f * N + col) * L + k;
    T[(size_t)b * n_out + q] = ((Fn[j] - C[j]) - norm[2 * kF * L + q]) / norm[3 * kF * L + q];
  }
}

// Bounded correction of the state's *_t buffers from network outputs Y
// [col][f * L + k]: a column whose largest |y| exceeds `bound`, that has a
// non-finite output, or whose corrected temperature or pressure would not
// stay positive is left unchanged.  Otherwise the cell is rebuilt the way a restriction builds it:
// density from the corrected p and T through the gas law, rho theta from the
// corrected p, horizontal momentum from the corrected velocity at the new
// density, and interface vertical momentum rescaled to the new interface
// density plus the centre increments rho' dw averaged onto the interface.
template <typename H>
__global__ __launch_bounds__(256) void k_apply(Fields<H> f, Consts c, const float *Y, const float *norm, float bound,
                                               int *applied) {
  const CLane ln = clane(c.N, c.L);
  const int L = c.L;
  const int k = ln.lev;
  const int lm = ln.lane > 0 ? ln.lane - 1 : 0;
  const size_t idx = (size_t)ln.col * c.S + k;
  const float *y = Y + (size_t)ln.col * kF * L;
  const float yT = y[k], yu = y[L + k], yv = y[2 * L + k], yw = y[3 * L + k], yp = y[4 * L + k];
  float m = fmaxf(fmaxf(fabsf(yT), fabsf(yu)), fmaxf(fmaxf(fabsf(yv), fabsf(yw)), fabsf(yp)));
  // fmaxf drops a NaN operand: a non-finite output marks the column here,
  // before the reduction, as out of bound
  if (!(isfinite(yT) && isfinite(yu) && isfinite(yv) && isfinite(yw) && isfinite(yp))) m = INFINITY;
  const double rho = f.rho_t[idx];
  const double p = c.p_ref * powd(c.Rd * f.rth_t[idx] / c.p_ref, c.gamma);
  const float *mo = norm + 2 * kF * L, *so = norm + 3 * kF * L;   // output mean, spread [f][k]
  const double dT = (double)(yT * so[k] + mo[k]);
  const double du = (double)(yu * so[L + k] + mo[L + k]);
  const double dv = (double)(yv * so[2 * L + k] + mo[2 * L + k]);
  const double dw = (double)(yw * so[3 * L + k] + mo[3 * L + k]);
  const double dp = (double)(yp * so[4 * L + k] + mo[4 * L + k]);
  const double p1 = p + dp, T1 = p / (rho * c.Rd) + dT;
  if (!(p1 > 0.0 && T1 > 0.0)) m = INFINITY;
  // largest |y| over the column's lanes
  const int cpw = 64 / L, cw = ln.lane / L;
  for (int s = 1; s < 64; s <<= 1) {
    const float o = __shfl_xor(m, s, 64);
    const int other = (ln.lane ^ s) / L;
    if (other == cw && (ln.lane ^ s) < cpw * L) m = fmaxf(m, o);
  }
  const bool ok = m <= bound && m < INFINITY;
  const double rho1 = ok ? p1 / (c.Rd * T1) : rho;
  const double rdw = rho1 * dw;
  const double rdw_m = __shfl(rdw, lm, 64);
  const double rho_m = __shfl(rho, lm, 64), rho1_m = __shfl(rho1, lm, 64);
  if (!ln.store) return;
  if (k == 0 && applied) applied[ln.col] = ok ? 1 : 0;
  if (!ok) return;
  const H *rh = f.rhat + (size_t)ln.col * 3;
  double e[3], n[3];
  east_north(rh[0], rh[1], rh[2], e, n);
  const double r = rho1 / rho;
  f.Mx_t[idx] = (H)(r * (double)f.Mx_t[idx] + rho1 * (du * e[0] + dv * n[0]));
  f.My_t[idx] = (H)(r * (double)f.My_t[idx] + rho1 * (du * e[1] + dv * n[1]));
  f.Mz_t[idx] = (H)(r * (double)f.Mz_t[idx] + rho1 * (du * e[2] + dv * n[2]));
  if (k > 0) f.W_t[idx] = f.W_t[idx] * (rho1_m + rho1) / (rho_m + rho) + 0.5 * (rdw_m + rdw);
  f.rho_t[idx] = rho1;
  f.rth_t[idx] = c.p_ref / c.Rd * powd(p1 / c.p_ref, 1.0 / c.gamma);
}

// Per (field, level) sum and sum of squares over n arrays [f][col][lev] (or
// of the differences Fn - C when Fn is given).  Workgroup (chunk, f, a) runs
// over a range of columns with thread t on level t % L (L divides 256).
__global__ __launch_bounds__(256) void k_stats(const float *C, const float *Fn, size_t stride, int N, int L,
                                               double *partial, int chunks) {
  __shared__ double s1[256], s2[256];
  const int chunk = blockIdx.x, f = blockIdx.y, a = blockIdx.z;
  const int per = (N + chunks - 1) / chunks;
  const int lo = chunk * per, hi = min(N, lo + per);
  const int k = threadIdx.x % L, c0 = threadIdx.x / L, cstep = 256 / L;
  double x1 = 0, x2 = 0;
  for (int col = lo + c0; col < hi; col += cstep) {
    const size_t j = (size_t)a * stride + ((size_t)f * N + col) * L + k;
    const double v = Fn ? (double)Fn[j] - (double)C[j] : (double)C[j];
    x1 += v;
    x2 += v * v;
  }
  s1[threadIdx.x] = x1;
  s2[threadIdx.x] = x2;
  __syncthreads();
  if ((int)threadIdx.x < L) {
    double t1 = 0, t2 = 0;
    for (int i = threadIdx.x; i < 256; i += L) {
      t1 += s1[i];
      t2 += s2[i];
    }
    const size_t o = ((((size_t)a * kF + f) * chunks + chunk) * L + threadIdx.x) * 2;
    partial[o] = t1;
    partial[o + 1] = t2;
  }
}

bool ok_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

// Running sums of the allocation-free statistics: adds a group of arrays'
// partial sums (k_stats layout, group-local array index) to sums[f][k][2]
// in the order the host reduction of thor_field_stats uses (array, then
// chunk), starting from zero for the first group.
__global__ __launch_bounds__(256) void k_stats_accumulate(const double *partial, int n_group, int chunks, int L,
                                                          double *sums, int first) {
  for (int q = threadIdx.x; q < kF * L; q += blockDim.x) {
    const int f = q / L, k = q % L;
    double s1 = first ? 0.0 : sums[2 * q], s2 = first ? 0.0 : sums[2 * q + 1];
    for (int a = 0; a < n_group; ++a)
      for (int ch = 0; ch < chunks; ++ch) {
        const size_t o = ((((size_t)a * kF + f) * chunks + ch) * L + k) * 2;
        s1 += partial[o];
        s2 += partial[o + 1];
      }
    sums[2 * q] = s1;
    sums[2 * q + 1] = s2;
  }
}

// Means and spreads [mean f k][spread f k] from the running sums.
__global__ __launch_bounds__(256) void k_stats_finish(const double *sums, int L, double n, double *out) {
  for (int q = threadIdx.x; q < kF * L; q += blockDim.x) {
    const double mu = sums[2 * q] / n;
    out[q] = mu;
    out[kF * L + q] = sqrt(fmax(sums[2 * q + 1] / n - mu * mu, 0.0));
  }
}

// Library-owned scratch of the allocation-free statistics: running sums
// (2 kF 256 doubles), the result (2 kF 256), then the partial sums of as
// many arrays as fit (320 n_lev doubles each).  One copy per GPU, kept until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStatsScratch = 131072;   // doubles: 1 MiB
constexpr size_t kStatsHead = 2 * 2 * kF * 256;
static __device__ __align__(256) double stats_scratch[kStatsScratch];

std::mutex g_stats_mu;
double *g_stats_ptr[64] = {};

// Device address of stats_scratch on the current device (looked up once per
// device), or nullptr with the error set.
double *stats_scratch_ptr() {
  int dev = 0;
  if (!ok_hip(hipGetDevice(&dev), "thor_field_stats_noalloc: current device")) return nullptr;
  if (dev < 0 || dev >= 64) { set_error("thor_field_stats_noalloc: device index above 63"); return nullptr; }
  std::lock_guard<std::mutex> lock(g_stats_mu);
  if (!g_stats_ptr[dev]) {
    void *p = nullptr;
    if (!ok_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(stats_scratch)), "thor_field_stats_noalloc: scratch address"))
      return nullptr;
    g_stats_ptr[dev] = static_cast<double *>(p);
  }
  return g_stats_ptr[dev];
}

}  // namespace
}  // namespace thor

using namespace thor;

struct thor_restriction {
  int n_fine = 0, n_coarse = 0;
  std::vector<int32_t> coarse_of_fine;
  int32_t *off = nullptr, *list = nullptr;   // device CSR (caller's buffer)
};

struct thor_corrector {
  thor_state *s = nullptr;
  thor_mlp *net = nullptr;
  float bound = 5.f;
  float *norm = nullptr;     // device [4][5][L]: input mean, spread; target mean, spread
  float *F = nullptr;        // device fields [5][N][L]
  __bf16 *X = nullptr;       // device inputs [N][35 L]
  float *Y = nullptr;        // device outputs [N][5 L]
  int *applied = nullptr;    // device [N]
};

extern "C" {

int thor_restriction_bytes(const thor_grid *fine, const thor_grid *coarse, size_t *bytes) {
  clear_error();
  if (!fine || !coarse || !bytes) { set_error("thor_restriction_bytes: NULL argument"); return THOR_EINVAL; }
  *bytes = ((size_t)(coarse->g.n + 1) * 4 + 255) / 256 * 256 + ((size_t)fine->g.n * 4 + 255) / 256 * 256;
  return THOR_OK;
}

int thor_restriction_build(const thor_grid *fine, const thor_grid *coarse, void *dev_buf, size_t dev_bytes,
                           void *hip_stream, thor_restriction **out) {
  clear_error();
  if (!fine || !coarse || !out) { set_error("thor_restriction_build: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  size_t need = 0;
  thor_restriction_bytes(fine, coarse, &need);
  if (dev_buf && dev_bytes < need) { set_error("thor_restriction_build: dev_bytes too small"); return THOR_ENOMEM; }
  if (((uintptr_t)dev_buf & 255) != 0) { set_error("thor_restriction_build: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  const Grid &F = fine->g, &C = coarse->g;
  if (F.glevel < C.glevel) { set_error("thor_restriction_build: fine grid is coarser"); return THOR_EINVAL; }
  thor_restriction *r = new (std::nothrow) thor_restriction;
  if (!r) { set_error("thor_restriction_build: out of host memory"); return THOR_ENOMEM; }
  r->n_fine = (int)F.n;
  r->n_coarse = (int)C.n;
  r->coarse_of_fine.assign(F.n, 0);
  auto dotp = [](const Vec3 &a, const Vec3 &b) { return a.x * b.x + a.y * b.y + a.z * b.z; };
  // Nearest coarse point (largest dot product, ties to the lower id) by a
  // greedy walk over the coarse neighbour graph from the previous answer,
  // finished with a check of the two-ring around the walk's end.
  int cur = 0;
  for (int64_t i = 0; i < F.n; ++i) {
    const Vec3 p = F.pos[i];
    auto better = [&](int a, int b) {   // is a strictly better than b
      const double da = dotp(p, C.pos[a]), db = dotp(p, C.pos[b]);
      return da > db || (da == db && a < b);
    };
    for (bool moved = true; moved;) {
      moved = false;
      for (int k = 0; k < 6; ++k) {
        const int nbk = C.nbr[(size_t)cur * 6 + k];
        if (nbk >= 0 && better(nbk, cur)) {
          cur = nbk;
          moved = true;
        }
      }
    }
    int best = cur;
    for (int k = 0; k < 6; ++k) {
      const int a = C.nbr[(size_t)cur * 6 + k];
      if (a < 0) continue;
      if (better(a, best)) best = a;
      for (int q = 0; q < 6; ++q) {
        const int b2 = C.nbr[(size_t)a * 6 + q];
        if (b2 >= 0 && better(b2, best)) best = b2;
      }
    }
    cur = best;
    r->coarse_of_fine[i] = best;
  }
  std::vector<int32_t> off(C.n + 1, 0), list(F.n);
  for (int64_t i = 0; i < F.n; ++i) off[r->coarse_of_fine[i] + 1]++;
  for (int64_t c = 0; c < C.n; ++c) off[c + 1] += off[c];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (int64_t i = 0; i < F.n; ++i) list[fill[r->coarse_of_fine[i]]++] = (int32_t)i;
  for (int64_t c = 0; c < C.n; ++c)
    if (off[c + 1] == off[c]) {
      delete r;
      set_error("thor_restriction_build: a coarse column received no fine column");
      return THOR_EINVAL;
    }
  if (!dev_buf) {   // host-only map (export works, thor_restrict does not)
    *out = r;
    return THOR_OK;
  }
  char *base = (char *)dev_buf;
  r->off = (int32_t *)base;
  r->list = (int32_t *)(base + ((size_t)(C.n + 1) * 4 + 255) / 256 * 256);
  hipStream_t st = (hipStream_t)hip_stream;
  if (!ok_hip(hipMemcpyAsync(r->off, off.data(), off.size() * 4, hipMemcpyHostToDevice, st), "copy off") ||
      !ok_hip(hipMemcpyAsync(r->list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st), "copy list") ||
      !ok_hip(hipStreamSynchronize(st), "restriction synchronize")) {
    delete r;
    return THOR_EHIP;
  }
  *out = r;
  return THOR_OK;
}

int thor_restriction_export(const thor_restriction *r, int32_t *coarse_of_fine) {
  clear_error();
  if (!r || !coarse_of_fine) { set_error("thor_restriction_export: NULL argument"); return THOR_EINVAL; }
  std::copy(r->coarse_of_fine.begin(), r->coarse_of_fine.end(), coarse_of_fine);
  return THOR_OK;
}

void thor_restriction_free(thor_restriction *r) { delete r; }

int thor_restrict(thor_state *fine, thor_state *coarse, const thor_restriction *r) {
  clear_error();
  if (!fine || !coarse || !r) { set_error("thor_restrict: NULL argument"); return THOR_EINVAL; }
  if (!r->off) { set_error("thor_restrict: the restriction was built without device memory"); return THOR_EINVAL; }
  if (fine->c.N != r->n_fine || coarse->c.N != r->n_coarse || fine->c.L != coarse->c.L ||
      fine->precision != coarse->precision || fine->c.dz != coarse->c.dz) {
    set_error("thor_restrict: states do not match the restriction (grids, levels, precision)");
    return THOR_EINVAL;
  }
  if (!ok_hip(hipStreamSynchronize(fine->stream), "restrict synchronize")) return THOR_EHIP;
  const unsigned nbk = cblocks(coarse->c.N, coarse->c.L);
  if (coarse->precision == THOR_MIXED)
    hipLaunchKernelGGL(k_restrict<float>, dim3(nbk), dim3(256), 0, coarse->stream, fine->f32[fine->parity], fine->c,
                       coarse->f32[coarse->parity], coarse->c, r->off, r->list);
  else
    hipLaunchKernelGGL(k_restrict<double>, dim3(nbk), dim3(256), 0, coarse->stream, fine->f64[fine->parity], fine->c,
                       coarse->f64[coarse->parity], coarse->c, r->off, r->list);
  return ok_hip(hipGetLastError(), "restrict launch") ? THOR_OK : THOR_EHIP;
}

int thor_state_fields32(thor_state *s, float *dev_out) {
  clear_error();
  if (!s || !dev_out) { set_error("thor_state_fields32: NULL argument"); return THOR_EINVAL; }
  const unsigned nbk = cblocks(s->c.N, s->c.L);
  if (s->precision == THOR_MIXED)
    hipLaunchKernelGGL(k_fields<float>, dim3(nbk), dim3(256), 0, s->stream, s->f32[s->parity], s->c, dev_out);
  else
    hipLaunchKernelGGL(k_fields<double>, dim3(nbk), dim3(256), 0, s->stream, s->f64[s->parity], s->c, dev_out);
  return ok_hip(hipGetLastError(), "fields launch") ? THOR_OK : THOR_EHIP;
}

int thor_field_stats(const float *C, const float *Fn, int n_arrays, size_t stride, int n_col, int n_lev,
                     void *dev_scratch, size_t scratch_bytes, void *hip_stream, double *mean_std_host) {
  clear_error();
  if (!C || !dev_scratch || !mean_std_host || n_arrays < 1 || n_col < 1 || n_lev < 1 || 256 % n_lev) {
    set_error("thor_field_stats: bad argument (n_lev must divide 256)");
    return THOR_EINVAL;
  }
  const int chunks = 32;
  const size_t np = (size_t)n_arrays * kF * chunks * n_lev * 2;
  if (scratch_bytes < np * sizeof(double)) { set_error("thor_field_stats: scratch too small"); return THOR_ENOMEM; }
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_stats, dim3(chunks, kF, n_arrays), dim3(256), 0, st, C, Fn, stride, n_col, n_lev,
                     (double *)dev_scratch, chunks);
  std::vector<double> part(np);
  if (!ok_hip(hipMemcpyAsync(part.data(), dev_scratch, np * sizeof(double), hipMemcpyDeviceToHost, st), "copy stats") ||
      !ok_hip(hipStreamSynchronize(st), "stats synchronize"))
    return THOR_EHIP;
  const int L = n_lev;
  for (int f = 0; f < kF; ++f)
    for (int k = 0; k < L; ++k) {
      double s1 = 0, s2 = 0;
      for (int a = 0; a < n_arrays; ++a)
        for (int ch = 0; ch < chunks; ++ch) {
          const size_t o = ((((size_t)a * kF + f) * chunks + ch) * L + k) * 2;
          s1 += part[o];
          s2 += part[o + 1];
        }
      const double n = (double)n_arrays * n_col;
      const double mu = s1 / n;
      mean_std_host[f * L + k] = mu;
      mean_std_host[kF * L + f * L + k] = std::sqrt(std::max(s2 / n - mu * mu, 0.0));
    }
  return THOR_OK;
}

int thor_field_stats_noalloc(const float *C, const float *Fn, int n_arrays, size_t stride, int n_col, int n_lev,
                             void *hip_stream, double *mean_std_host) {
  clear_error();
  if (!C || !mean_std_host || n_arrays < 1 || n_col < 1 || n_lev < 1 || 256 % n_lev) {
    set_error("thor_field_stats_noalloc: bad argument (n_lev must divide 256)");
    return THOR_EINVAL;
  }
  const int chunks = 32;
  const size_t per_array = (size_t)kF * chunks * n_lev * 2;
  const size_t cap = (kStatsScratch - kStatsHead) / per_array;   // arrays per group
  if (cap < 1) {
    set_error("thor_field_stats_noalloc: one array's partial sums exceed the 1 MiB scratch");
    return THOR_ENOMEM;
  }
  double *scr = stats_scratch_ptr();
  if (!scr) return THOR_EHIP;
  double *sums = scr, *result = scr + 2 * kF * 256, *partial = scr + kStatsHead;
  hipStream_t st = (hipStream_t)hip_stream;
  for (int a0 = 0; a0 < n_arrays; a0 += (int)cap) {
    const int ng = (int)std::min<size_t>(cap, (size_t)(n_arrays - a0));
    const float *Cg = C + (size_t)a0 * stride;
    const float *Fg = Fn ? Fn + (size_t)a0 * stride : nullptr;
    hipLaunchKernelGGL(k_stats, dim3(chunks, kF, ng), dim3(256), 0, st, Cg, Fg, stride, n_col, n_lev, partial, chunks);
    hipLaunchKernelGGL(k_stats_accumulate, dim3(1), dim3(256), 0, st, (const double *)partial, ng, chunks, n_lev, sums,
                       (int)(a0 == 0));
  }
  hipLaunchKernelGGL(k_stats_finish, dim3(1), dim3(256), 0, st, (const double *)sums, n_lev,
                     (double)n_arrays * n_col, result);
  if (!ok_hip(hipGetLastError(), "thor_field_stats_noalloc: launch") ||
      !ok_hip(hipMemcpyAsync(mean_std_host, result, (size_t)2 * kF * n_lev * sizeof(double), hipMemcpyDeviceToHost,
                             st),
              "thor_field_stats_noalloc: copy") ||
      !ok_hip(hipStreamSynchronize(st), "thor_field_stats_noalloc: synchronize"))
    return THOR_EHIP;
  return THOR_OK;
}

int thor_corrector_bytes(const thor_state *s, size_t *bytes) {
  clear_error();
  if (!s || !bytes) { set_error("thor_corrector_bytes: NULL argument"); return THOR_EINVAL; }
  const size_t N = s->c.N, L = s->c.L;
  auto a = [](size_t x) { return (x + 255) / 256 * 256; };
  *bytes = a(4 * kF * L * 4) + a(kF * N * L * 4) + a(N * 7 * kF * L * 2) + a(N * kF * L * 4) + a(N * 4);
  return THOR_OK;
}

int thor_corrector_init(thor_state *s, thor_mlp *net, const float *norm_host, float bound, void *dev_buf,
                        size_t dev_bytes, thor_corrector **out) {
  clear_error();
  if (!s || !net || !norm_host || !dev_buf || !out) { set_error("thor_corrector_init: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  if ((7 * kF * s->c.L) % 32) { set_error("thor_corrector_init: n_lev must be a multiple of 32"); return THOR_EINVAL; }
  int n_in = 0, n_out = 0, max_batch = 0;
  mlp_shape_of(net, &n_in, &n_out, &max_batch);
  if (n_in != 7 * kF * s->c.L || n_out != kF * s->c.L || max_batch < s->c.N) {
    set_error("thor_corrector_init: the network needs 35 n_lev inputs, 5 n_lev outputs and max_batch >= n_col");
    return THOR_EINVAL;
  }
  if (((uintptr_t)dev_buf & 255) != 0) { set_error("thor_corrector_init: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  size_t need = 0;
  thor_corrector_bytes(s, &need);
  if (dev_bytes < need) { set_error("thor_corrector_init: dev_bytes too small"); return THOR_ENOMEM; }
  for (size_t q = 0; q < (size_t)kF * s->c.L; ++q)
    if (!(norm_host[kF * s->c.L + q] > 0) || !(norm_host[3 * kF * s->c.L + q] > 0)) {
      set_error("thor_corrector_init: spreads must be positive");
      return THOR_EINVAL;
    }
  thor_corrector *c = new (std::nothrow) thor_corrector;
  if (!c) { set_error("thor_corrector_init: out of host memory"); return THOR_ENOMEM; }
  const size_t N = s->c.N, L = s->c.L;
  auto a = [](size_t x) { return (x + 255) / 256 * 256; };
  char *base = (char *)dev_buf;
  c->norm = (float *)base;
  base += a(4 * kF * L * 4);
  c->F = (float *)base;
  base += a(kF * N * L * 4);
  c->X = (__bf16 *)base;
  base += a(N * 7 * kF * L * 2);
  c->Y = (float *)base;
  base += a(N * kF * L * 4);
  c->applied = (int *)base;
  c->s = s;
  c->net = net;
  c->bound = bound;
  if (!ok_hip(hipMemcpyAsync(c->norm, norm_host, 4 * kF * L * 4, hipMemcpyHostToDevice, s->stream), "copy norm") ||
      !ok_hip(hipStreamSynchronize(s->stream), "corrector synchronize")) {
    delete c;
    return THOR_EHIP;
  }
  *out = c;
  return THOR_OK;
}

int thor_corrector_batch(thor_corrector *c, const float *coarse_fields, const float *fine_fields,
                         size_t pair_stride, const int32_t *pairs, const int32_t *cols, int B, void *x_bf16,
                         float *target) {
  clear_error();
  if (!c || !coarse_fields || !fine_fields || !pairs || !cols || !x_bf16 || !target || B < 1) {
    set_error("thor_corrector_batch: bad argument");
    return THOR_EINVAL;
  }
  const int N = c->s->c.N, L = c->s->c.L;
  const size_t total = (size_t)B * (7 * kF + kF) * L;
  const int32_t *nbr = c->s->precision == THOR_MIXED ? c->s->f32[0].nbr : c->s->f64[0].nbr;
  hipLaunchKernelGGL(k_batch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->s->stream, coarse_fields,
                     fine_fields, pair_stride, pairs, cols, nbr, c->norm, (__bf16 *)x_bf16, target, B, N, L);
  return ok_hip(hipGetLastError(), "batch launch") ? THOR_OK : THOR_EHIP;
}

int thor_corrector_apply(thor_corrector *c, int *n_applied) {
  clear_error();
  if (!c) { set_error("thor_corrector_apply: NULL argument"); return THOR_EINVAL; }
  thor_state *s = c->s;
  const int N = s->c.N, L = s->c.L;
  int rc = thor_state_fields32(s, c->F);
  if (rc != THOR_OK) return rc;
  const int32_t *nbr = s->precision == THOR_MIXED ? s->f32[0].nbr : s->f64[0].nbr;
  const size_t total = (size_t)N * 7 * kF * L;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s->stream, c->F, nbr, c->norm,
                     c->X, N, L);
  rc = thor_mlp_forward(c->net, c->X, N, c->Y);
  if (rc != THOR_OK) return rc;
  const unsigned nbk = cblocks(N, L);
  if (s->precision == THOR_MIXED)
    hipLaunchKernelGGL(k_apply<float>, dim3(nbk), dim3(256), 0, s->stream, s->f32[s->parity], s->c, c->Y, c->norm,
                       c->bound, c->applied);
  else
    hipLaunchKernelGGL(k_apply<double>, dim3(nbk), dim3(256), 0, s->stream, s->f64[s->parity], s->c, c->Y, c->norm,
                       c->bound, c->applied);
  if (!ok_hip(hipGetLastError(), "apply launch")) return THOR_EHIP;
  if (n_applied) {
    std::vector<int> a(N);
    if (!ok_hip(hipMemcpyAsync(a.data(), c->applied, (size_t)N * 4, hipMemcpyDeviceToHost, s->stream), "copy applied") ||
        !ok_hip(hipStreamSynchronize(s->stream), "apply synchronize"))
      return THOR_EHIP;
    int k = 0;
    for (int v : a) k += v;
    *n_applied = k;
  }
  return THOR_OK;
}

void thor_corrector_free(thor_corrector *c) { delete c; }

}  // extern "C"
