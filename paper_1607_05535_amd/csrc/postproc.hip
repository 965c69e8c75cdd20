// Post-processing on pressure levels (the results of Sec. 7 are shown on
// pressure levels): per snapshot, every column's u, v, T and theta are
// interpolated linearly in pressure to the requested levels; latitude-band
// zonal means (area-weighted over the columns that have a value), the eddy
// fluxes [u'v'] and [v'T'] (eddies = deviations from the zonal mean) and the
// valid area fraction are added to running time sums; the result divides
// the sums by the number of snapshots with a value and adds the mass
// streamfunction Psi = 2 pi A cos(lat) / g * int_0^p [v] dp.  Beside them,
// the grid-imprinting map of the Held-Suarez results: per column, the time
// sum of w* = w - {w} in the first model layer, {w} the area-weighted mean
// of w over the column's latitude band.
//
// Readings: a level outside a column's [top-cell, bottom-cell] pressure
// range has no value in that column; band b covers latitudes
// [-90 + 180 b / n, -90 + 180 (b + 1) / n) degrees (the north pole in the
// last band); Psi uses the trapezoid rule with [v](p = 0) = [v](first level);
// the imprinting bracket is a zonal deviation followed by a time mean (a
// deviation from the time mean alone would average to zero).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "powd.h"
#include "state.h"

namespace thor {
namespace {

constexpr int kZq = 4;          // interpolated quantities: u, v, T, theta
constexpr int kZslot = kZq + 1; // + valid flag
constexpr int kZthreads = 256;  // threads of a band's reduction

bool zok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

// Per column (lanes = levels, floor(64 / L) columns per wavefront): p, T,
// u, v, theta of every level, then for each pressure level the interval of
// the lowest-index level pair whose pressures bracket it; the column's
// values there go to Z[col][j][0..3] and Z[col][j][4] = 1 (0 if none).
// Zw[col] = w at the centre of the first layer (half the momentum of the
// first interior interface over rho; the ground interface carries none).
template <typename H>
__global__ __launch_bounds__(256) void k_zinterp(Fields<H> f, Consts c, const double *plev, int np, double *Z,
                                                 double *Zw) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int L = c.L, cpw = 64 / L;
  const int cw = lane / L, lev = lane - cw * L;
  const bool real = cw < cpw;
  int col = wave * cpw + cw;
  const bool store = real && col < c.N;
  if (col >= c.N) col = c.N - 1;
  const size_t idx = (size_t)col * c.S + lev;   // state row stride
  const double rho = f.rho_t[idx], rth = f.rth_t[idx];
  const double p = c.p_ref * powd(c.Rd * rth / c.p_ref, c.gamma);
  const H *rh = f.rhat + (size_t)col * 3;
  const double x = rh[0], y = rh[1], z = rh[2];
  const double lam = sqrt(x * x + y * y) < 1e-12 ? 0.0 : atan2(y, x);
  const double phi = asin(fmin(1.0, fmax(-1.0, z)));
  const double vx = (double)f.Mx_t[idx] / rho, vy = (double)f.My_t[idx] / rho, vz = (double)f.Mz_t[idx] / rho;
  double q[kZq];
  q[0] = -sin(lam) * vx + cos(lam) * vy;
  q[1] = -sin(phi) * cos(lam) * vx - sin(phi) * sin(lam) * vy + cos(phi) * vz;
  q[2] = p / (rho * c.Rd);
  q[3] = rth / rho;
  const int lp = lane < 63 ? lane + 1 : 63;
  const double p_up = __shfl(p, lp, 64);
  const double Wl = lev == 0 ? 0.0 : (double)f.W_t[idx];
  const double W_up = __shfl(Wl, lp, 64);
  if (store && lev == 0) Zw[col] = L > 1 ? 0.5 * W_up / rho : 0.0;
  double q_up[kZq];
#pragma unroll
  for (int k = 0; k < kZq; ++k) q_up[k] = __shfl(q[k], lp, 64);
  const int first = cw * L;   // first lane of the column (in range for every lane)
  const unsigned long long colmask = (L == 64 ? ~0ull : ((1ull << L) - 1)) << (real ? first : 0);
  for (int j = 0; j < np; ++j) {
    const double pj = plev[j];
    // interval (lev, lev + 1): lo = p_up < hi = p
    const bool hit = real && lev + 1 < L && p_up <= pj && pj <= p;
    const unsigned long long m = __ballot(hit) & colmask;
    const int src = m ? __builtin_ctzll(m) : lane;
    const double w = (pj - p_up) / (p - p_up);
    double v[kZq];
#pragma unroll
    for (int k = 0; k < kZq; ++k) v[k] = q_up[k] + w * (q[k] - q_up[k]);
    double o[kZq];
#pragma unroll
    for (int k = 0; k < kZq; ++k) o[k] = __shfl(v[k], src, 64);
    if (store && lev == 0) {
      double *out = Z + ((size_t)col * np + j) * kZslot;
#pragma unroll
      for (int k = 0; k < kZq; ++k) out[k] = m ? o[k] : 0.0;
      out[kZq] = m ? 1.0 : 0.0;
    }
  }
}

// Fixed-order sum of one value per thread over the workgroup.
__device__ __forceinline__ double block_sum(double v, double *sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = kZthreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

// Band b, pressure level j (one workgroup each): area-weighted means of the
// band's columns that have a value (thread t takes columns t, t + 256, ... of
// the band's list), then the eddy products; added to the time sums
// S[b][j][0..6] = u, v, T, theta, [u'v'], [v'T'], valid fraction and to the
// snapshot count S[b][j][7].
__global__ __launch_bounds__(kZthreads) void k_zreduce(const double *Z, int np, const int32_t *off,
                                                       const int32_t *cols, const double *area, double *S) {
  __shared__ double sm[kZthreads];
  const int b = blockIdx.x, j = blockIdx.y;
  const int a0 = off[b], a1 = off[b + 1];
  double Aband = 0.0, sA = 0, su = 0, sv = 0, sT = 0, sth = 0;
  for (int i = a0 + threadIdx.x; i < a1; i += kZthreads) {
    const int col = cols[i];
    const double *z = Z + ((size_t)col * np + j) * kZslot;
    const double A0 = area[col], A = A0 * z[kZq];
    Aband += A0;
    sA += A;
    su += A * z[0];
    sv += A * z[1];
    sT += A * z[2];
    sth += A * z[3];
  }
  sA = block_sum(sA, sm);
  if (sA == 0.0) return;   // uniform across the workgroup
  Aband = block_sum(Aband, sm);
  const double mu = block_sum(su, sm) / sA, mv = block_sum(sv, sm) / sA;
  const double mT = block_sum(sT, sm) / sA, mth = block_sum(sth, sm) / sA;
  double euv = 0, evT = 0;
  for (int i = a0 + threadIdx.x; i < a1; i += kZthreads) {
    const int col = cols[i];
    const double *z = Z + ((size_t)col * np + j) * kZslot;
    const double A = area[col] * z[kZq];
    euv += A * (z[0] - mu) * (z[1] - mv);
    evT += A * (z[1] - mv) * (z[2] - mT);
  }
  euv = block_sum(euv, sm) / sA;
  evT = block_sum(evT, sm) / sA;
  if (threadIdx.x == 0) {
    double *o = S + ((size_t)b * np + j) * 8;
    o[0] += mu;
    o[1] += mv;
    o[2] += mT;
    o[3] += mth;
    o[4] += euv;
    o[5] += evT;
    o[6] += sA / Aband;
    o[7] += 1.0;
  }
}

// Band b (one workgroup): area-weighted mean of the first-layer w over all
// of the band's columns, then each column's deviation from it added to the
// time sum Wsum[col].
__global__ __launch_bounds__(kZthreads) void k_zimprint(const double *Zw, const int32_t *off, const int32_t *cols,
                                                        const double *area, double *Wsum) {
  __shared__ double sm[kZthreads];
  const int b = blockIdx.x;
  const int a0 = off[b], a1 = off[b + 1];
  double sA = 0, sw = 0;
  for (int i = a0 + threadIdx.x; i < a1; i += kZthreads) {
    const int col = cols[i];
    sA += area[col];
    sw += area[col] * Zw[col];
  }
  sA = block_sum(sA, sm);
  if (sA == 0.0) return;   // empty band, uniform across the workgroup
  const double mw = block_sum(sw, sm) / sA;
  for (int i = a0 + threadIdx.x; i < a1; i += kZthreads) {
    const int col = cols[i];
    Wsum[col] += Zw[col] - mw;
  }
}

__global__ void k_zzero(double *S, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) S[i] = 0.0;
}

size_t a256z(size_t x) { return (x + 255) & ~(size_t)255; }

// Partial sums per workgroup (4 wavefronts, lanes = levels) of the absolute
// angular momentum about the rotation axis of the state between large steps:
// per cell (R x rho v)_z with R = r_C rhat, plus rho Omega r_C^2 cos^2(lat),
// times the volume A_c r_C^2 dz; fixed reduction order.
template <typename H>
__global__ __launch_bounds__(256) void k_angmom(Fields<H> f, Consts c, double *out) {
  __shared__ double sm[4];
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int L = c.L, cpw = 64 / L;
  const int cw = lane / L, lev = lane - cw * L;
  const int col = wave * cpw + cw;
  double v = 0.0;
  if (cw < cpw && col < c.N) {
    const size_t idx = (size_t)col * c.S + lev;
    const double rC = c.radius + (lev + 0.5) * c.rdz;
    const H *rh = f.rhat + (size_t)col * 3;
    const double x = rh[0], y = rh[1];
    const double rel = rC * (x * (double)f.My_t[idx] - y * (double)f.Mx_t[idx]);
    const double plan = f.rho_t[idx] * c.omega * rC * rC * (x * x + y * y);
    v = (rel + plan) * f.area[col] * rC * rC * c.dz;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
}

}  // namespace

template <typename H>
void launch_angmom(const Fields<H> &f, const Consts &c, double *out, hipStream_t s, int *nblocks_out) {
  const long waves = (c.N + 64 / c.L - 1) / (64 / c.L);
  const int nb = (int)((waves + 3) / 4);
  *nblocks_out = nb;
  hipLaunchKernelGGL(k_angmom<H>, dim3(nb), dim3(256), 0, s, f, c, out);
}
template void launch_angmom<double>(const Fields<double> &, const Consts &, double *, hipStream_t, int *);
template void launch_angmom<float>(const Fields<float> &, const Consts &, double *, hipStream_t, int *);

}  // namespace thor

using namespace thor;

struct thor_zonal {
  thor_state *s = nullptr;
  int nb = 0, np = 0;
  std::vector<double> plev_h;
  double radius = 0, gravity = 0;
  double *plev = nullptr, *Z = nullptr, *S = nullptr, *area = nullptr, *Zw = nullptr, *Wsum = nullptr;
  int32_t *off = nullptr, *cols = nullptr;
  int snapshots = 0;
};

namespace {

size_t zonal_layout(thor_zonal *z, size_t N, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *p = base ? base + off : nullptr;
    off += a256z(bytes);
    return p;
  };
  z->plev = (double *)take(z->np * sizeof(double));
  z->Z = (double *)take(N * z->np * kZslot * sizeof(double));
  z->S = (double *)take((size_t)z->nb * z->np * 8 * sizeof(double));
  z->area = (double *)take(N * sizeof(double));
  z->off = (int32_t *)take((z->nb + 1) * sizeof(int32_t));
  z->cols = (int32_t *)take(N * sizeof(int32_t));
  z->Zw = (double *)take(N * sizeof(double));
  z->Wsum = (double *)take(N * sizeof(double));
  return off;
}

bool zonal_args(const thor_state *s, int n_bands, const double *plev, int n_plev) {
  if (!s || !plev) { set_error("thor_zonal: NULL argument"); return false; }
  if (n_bands < 1 || n_bands > 4096 || n_plev < 1 || n_plev > 1024) {
    set_error("thor_zonal: need 1..4096 bands and 1..1024 pressure levels");
    return false;
  }
  for (int j = 0; j < n_plev; ++j)
    if (!(plev[j] > 0) || (j > 0 && !(plev[j] > plev[j - 1]))) {
      set_error("thor_zonal: pressure levels must be positive and strictly ascending");
      return false;
    }
  return true;
}

}  // namespace

extern "C" {

int thor_zonal_bytes(const thor_state *s, int n_bands, const double *plev, int n_plev, size_t *bytes) {
  clear_error();
  if (!bytes || !zonal_args(s, n_bands, plev, n_plev)) {
    if (!bytes) set_error("thor_zonal_bytes: NULL argument");
    return THOR_EINVAL;
  }
  thor_zonal z;
  z.nb = n_bands;
  z.np = n_plev;
  *bytes = zonal_layout(&z, (size_t)s->n_col, nullptr);
  return THOR_OK;
}

int thor_zonal_init(thor_state *s, const thor_grid *g, double radius, double gravity, int n_bands,
                    const double *plev, int n_plev, void *dev_buf, size_t dev_bytes, thor_zonal **out) {
  clear_error();
  if (!out || !g || !dev_buf) { set_error("thor_zonal_init: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  if (!zonal_args(s, n_bands, plev, n_plev)) return THOR_EINVAL;
  if (g->g.n != s->n_col) { set_error("thor_zonal_init: grid does not match the state"); return THOR_EINVAL; }
  if (!(radius > 0 && gravity > 0)) { set_error("thor_zonal_init: radius and gravity must be positive"); return THOR_EINVAL; }
  if (((uintptr_t)dev_buf & 255) != 0) { set_error("thor_zonal_init: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  thor_zonal *z = new (std::nothrow) thor_zonal;
  if (!z) { set_error("thor_zonal_init: out of host memory"); return THOR_ENOMEM; }
  z->s = s;
  z->nb = n_bands;
  z->np = n_plev;
  z->plev_h.assign(plev, plev + n_plev);
  z->radius = radius;
  z->gravity = gravity;
  const size_t N = (size_t)s->n_col;
  if (dev_bytes < zonal_layout(z, N, nullptr)) {
    delete z;
    set_error("thor_zonal_init: dev_bytes smaller than thor_zonal_bytes");
    return THOR_ENOMEM;
  }
  zonal_layout(z, N, (char *)dev_buf);
  // latitude bands, columns in increasing id within a band
  std::vector<int32_t> off(n_bands + 1, 0), cols(N);
  std::vector<int> band(N);
  for (size_t i = 0; i < N; ++i) {
    const double lat = std::asin(std::fmin(1.0, std::fmax(-1.0, g->g.pos[i].z)));
    int b = (int)std::floor((lat + M_PI / 2) / M_PI * n_bands);
    band[i] = std::min(std::max(b, 0), n_bands - 1);
    off[band[i] + 1] += 1;
  }
  for (int b = 0; b < n_bands; ++b) off[b + 1] += off[b];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  for (size_t i = 0; i < N; ++i) cols[fill[band[i]]++] = (int32_t)i;
  hipStream_t st = s->stream;
  const size_t ns = (size_t)n_bands * n_plev * 8;
  bool ok = zok(hipMemcpyAsync(z->plev, plev, n_plev * sizeof(double), hipMemcpyHostToDevice, st), "copy plev") &&
            zok(hipMemcpyAsync(z->area, g->g.area.data(), N * sizeof(double), hipMemcpyHostToDevice, st), "copy area") &&
            zok(hipMemcpyAsync(z->off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy off") &&
            zok(hipMemcpyAsync(z->cols, cols.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy cols");
  if (ok) {
    hipLaunchKernelGGL(k_zzero, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, z->S, ns);
    hipLaunchKernelGGL(k_zzero, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, z->Wsum, N);
    ok = zok(hipGetLastError(), "zero sums") && zok(hipStreamSynchronize(st), "zonal init synchronize");
  }
  if (!ok) { delete z; return THOR_EHIP; }
  *out = z;
  return THOR_OK;
}

int thor_zonal_accumulate(thor_zonal *z) {
  clear_error();
  if (!z) { set_error("thor_zonal_accumulate: NULL argument"); return THOR_EINVAL; }
  thor_state *s = z->s;
  const int L = s->c.L, cpw = 64 / L;
  const long waves = (s->c.N + cpw - 1) / cpw;
  const unsigned nbk = (unsigned)((waves + 3) / 4);
  if (s->precision == THOR_MIXED)
    hipLaunchKernelGGL(k_zinterp<float>, dim3(nbk), dim3(256), 0, s->stream, s->f32[s->parity], s->c, z->plev, z->np, z->Z,
                       z->Zw);
  else
    hipLaunchKernelGGL(k_zinterp<double>, dim3(nbk), dim3(256), 0, s->stream, s->f64[s->parity], s->c, z->plev, z->np, z->Z,
                       z->Zw);
  hipLaunchKernelGGL(k_zreduce, dim3(z->nb, z->np), dim3(kZthreads), 0, s->stream, z->Z, z->np, z->off, z->cols, z->area, z->S);
  hipLaunchKernelGGL(k_zimprint, dim3(z->nb), dim3(kZthreads), 0, s->stream, z->Zw, z->off, z->cols, z->area, z->Wsum);
  if (!zok(hipGetLastError(), "zonal accumulate")) return THOR_EHIP;
  z->snapshots += 1;
  return THOR_OK;
}

int thor_zonal_result(thor_zonal *z, double *host_out, int *n_snapshots) {
  clear_error();
  if (!z || !host_out) { set_error("thor_zonal_result: NULL argument"); return THOR_EINVAL; }
  const int nb = z->nb, np = z->np;
  std::vector<double> S((size_t)nb * np * 8);
  if (!zok(hipMemcpyAsync(S.data(), z->S, S.size() * sizeof(double), hipMemcpyDeviceToHost, z->s->stream), "copy sums") ||
      !zok(hipStreamSynchronize(z->s->stream), "zonal result synchronize"))
    return THOR_EHIP;
  for (int b = 0; b < nb; ++b) {
    const double lat = -M_PI / 2 + (b + 0.5) * M_PI / nb;
    const double fac = 2.0 * M_PI * z->radius * std::cos(lat) / z->gravity;
    double integ = 0.0, v_prev = 0.0, p_prev = 0.0;
    for (int j = 0; j < np; ++j) {
      const double *s = &S[((size_t)b * np + j) * 8];
      double *o = host_out + ((size_t)b * np + j) * THOR_ZM_COUNT;
      const double n = s[7];
      for (int k = 0; k < 7; ++k) o[k] = n > 0 ? s[k] / n : 0.0;
      const double v = o[THOR_ZM_V];
      integ = j == 0 ? v * z->plev_h[0] : integ + 0.5 * (v + v_prev) * (z->plev_h[j] - p_prev);
      o[THOR_ZM_PSI] = fac * integ;
      o[THOR_ZM_SNAPSHOTS] = n;
      v_prev = v;
      p_prev = z->plev_h[j];
    }
  }
  if (n_snapshots) *n_snapshots = z->snapshots;
  return THOR_OK;
}

int thor_zonal_imprint(thor_zonal *z, double *host_out, int *n_snapshots) {
  clear_error();
  if (!z || !host_out) { set_error("thor_zonal_imprint: NULL argument"); return THOR_EINVAL; }
  const size_t N = (size_t)z->s->n_col;
  if (!zok(hipMemcpyAsync(host_out, z->Wsum, N * sizeof(double), hipMemcpyDeviceToHost, z->s->stream), "copy imprint") ||
      !zok(hipStreamSynchronize(z->s->stream), "zonal imprint synchronize"))
    return THOR_EHIP;
  const double n = z->snapshots;
  for (size_t i = 0; i < N; ++i) host_out[i] = n > 0 ? host_out[i] / n : 0.0;
  if (n_snapshots) *n_snapshots = z->snapshots;
  return THOR_OK;
}

int thor_zonal_reset(thor_zonal *z) {
  clear_error();
  if (!z) { set_error("thor_zonal_reset: NULL argument"); return THOR_EINVAL; }
  const size_t ns = (size_t)z->nb * z->np * 8;
  const size_t N = (size_t)z->s->n_col;
  hipLaunchKernelGGL(k_zzero, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, z->s->stream, z->S, ns);
  hipLaunchKernelGGL(k_zzero, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, z->s->stream, z->Wsum, N);
  z->snapshots = 0;
  return zok(hipGetLastError(), "zonal reset") ? THOR_OK : THOR_EHIP;
}

void thor_zonal_free(thor_zonal *z) { delete z; }

}  // extern "C"

// ===========================================================================
// Measurement aid: streaming kernel with a given read/write mix.
// ===========================================================================
namespace {
struct StreamPtrs {
  const double *src[16];
  double *dst[8];
};

// NS sources unrolled (every load issued before the sum uses it), the stores
// in a loop.
template <int NS>
__global__ __launch_bounds__(256) void k_stream_mix(StreamPtrs p, int n_dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = p.src[k][i];
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) acc += v[k];
  for (int k = 0; k < n_dst; ++k) p.dst[k][i] = acc + k;
}

template <int NS>
void launch_stream_mix(int n_src, const StreamPtrs &p, int n_dst, int64_t n, unsigned blocks, hipStream_t s) {
  if (n_src == NS) hipLaunchKernelGGL(k_stream_mix<NS>, dim3(blocks), dim3(256), 0, s, p, n_dst, n);
  else if constexpr (NS > 1) launch_stream_mix<NS - 1>(n_src, p, n_dst, n, blocks, s);
}
}  // namespace

extern "C" int thor_stream_mix(const double *const *src, int n_src, double *const *dst, int n_dst, int64_t n,
                               void *hip_stream) {
  thor::clear_error();
  if (!src || !dst || n_src < 1 || n_src > 16 || n_dst < 1 || n_dst > 8 || n < 1) {
    thor::set_error("thor_stream_mix: 1..16 sources, 1..8 destinations, n >= 1");
    return THOR_EINVAL;
  }
  StreamPtrs p{};
  for (int k = 0; k < n_src; ++k) {
    if (!src[k]) { thor::set_error("thor_stream_mix: NULL source"); return THOR_EINVAL; }
    p.src[k] = src[k];
  }
  for (int k = 0; k < n_dst; ++k) {
    if (!dst[k]) { thor::set_error("thor_stream_mix: NULL destination"); return THOR_EINVAL; }
    p.dst[k] = dst[k];
  }
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) { thor::set_error("thor_stream_mix: n too large"); return THOR_EINVAL; }
  launch_stream_mix<16>(n_src, p, n_dst, n, (unsigned)blocks, (hipStream_t)hip_stream);
  if (hipGetLastError() != hipSuccess) { thor::set_error("thor_stream_mix: launch failed"); return THOR_EHIP; }
  return THOR_OK;
}
