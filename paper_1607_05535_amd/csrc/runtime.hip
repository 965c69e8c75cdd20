// Host runtime of libthor: state set-up in caller-owned device memory, the
// large-step schedule (Sec. 3: WS-RK3 stages of 1, n/2 and n acoustic
// substeps, Sec. 5 physics after the stages), HIP-graph replay of a large
// step, diagnostics, checkpoints and kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "state.h"

namespace thor {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

namespace {

// SplitMix64 output step (Steele, Lea and Flood 2014) of a counter state.
inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Assigns consecutive 256-byte aligned slices of a device buffer.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += align256(count * sizeof(T));
    return p;
  }
};

// Per-cell state arrays use the row stride S = L rounded up to a multiple of
// kHq, so that every row starts 16-byte aligned and the gather kernels load
// whole groups of kHq levels; the staging/diagnostic area keeps the
// canonical [col][lev] layout.
inline size_t row_stride(size_t L) { return (L + kHq - 1) / kHq * kHq; }

template <typename H>
void carve(Carver &cv, Fields<H> &f, size_t N, size_t L, bool anelastic) {
  const size_t NL = N * row_stride(L), NLc = N * L;
  f.nbr = cv.take<int32_t>(N * 6);
  f.dc = cv.take<H>(N * 21);
  f.lc = cv.take<H>(N * 6);
  f.rhat = cv.take<H>(N * 3);
  f.ddi = cv.take<int32_t>(N * kRing2);
  f.ddw = cv.take<H>(N * kRing2 * 3);
  f.area = cv.take<double>(N);
  f.teq = cv.take<double>(N);
  f.rho = cv.take<double>(NL);
  f.rth = cv.take<double>(NL);
  f.W = cv.take<double>(NL);
  f.Mx = cv.take<H>(NL);
  f.My = cv.take<H>(NL);
  f.Mz = cv.take<H>(NL);
  f.ps = cv.take<H>(NL);
  f.rho_t = cv.take<double>(NL);
  f.rth_t = cv.take<double>(NL);
  f.W_t = cv.take<double>(NL);
  f.p_t = cv.take<double>(NL);
  f.Mx_t = cv.take<H>(NL);
  f.My_t = cv.take<H>(NL);
  f.Mz_t = cv.take<H>(NL);
  f.FMx = cv.take<H>(NL);
  f.FMy = cv.take<H>(NL);
  f.FMz = cv.take<H>(NL);
  f.FW = cv.take<double>(NL);
  f.Hrho = cv.take<H>(NL);
  f.Hrth = cv.take<H>(NL);
  f.SMx = cv.take<H>(NL);
  f.SMy = cv.take<H>(NL);
  f.SMz = cv.take<H>(NL);
  f.SW = cv.take<double>(NL);
  f.thL = cv.take<H>(NL);
  f.Gam = cv.take<H>(NL);
  f.D = cv.take<H>(NL);
  f.Dt = cv.take<H>(NL);
  f.wI = cv.take<double>(NL);
  f.Xrho = cv.take<double>(NL);
  f.Xvx = cv.take<double>(NL);
  f.Xvy = cv.take<double>(NL);
  f.Xvz = cv.take<double>(NL);
  f.Xw = cv.take<double>(NL);
  f.XT = cv.take<double>(NL);
  // the staging/diagnostic area doubles as checkpoint staging (6 fields)
  f.diag = cv.take<double>(6 * NLc);
  f.partial = cv.take<double>(2 * ((N + 3) / 4 + 16));
  f.epart = cv.take<double>(4 * ((N + 3) / 4 + 16) + 8);
  // after everything else, so that the other arrays keep their offsets
  f.rref = anelastic ? cv.take<double>(row_stride(L)) : nullptr;
  f.fC = anelastic ? cv.take<H>(NL) : nullptr;
  f.fI = anelastic ? cv.take<double>(NL) : nullptr;
}

template <typename H>
Fields<H> swapped(const Fields<H> &a) {
  Fields<H> b = a;
  std::swap(b.rho, b.rho_t);
  std::swap(b.rth, b.rth_t);
  std::swap(b.W, b.W_t);
  std::swap(b.Mx, b.Mx_t);
  std::swap(b.My, b.My_t);
  std::swap(b.Mz, b.Mz_t);
  return b;
}

bool hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

}  // namespace
}  // namespace thor

using namespace thor;

namespace {

bool validate(const thor_planet *pl, const thor_vertical *v, const thor_numerics *num,
              const thor_forcing *fo, const thor_init *in) {
  if (!pl || !v || !num || !fo || !in) { set_error("thor_state_init: NULL argument"); return false; }
  if (!(pl->radius > 0 && pl->gravity >= 0 && pl->Rd > 0 && pl->Cp > pl->Rd && pl->p_ref > 0)) {
    set_error("thor_state_init: planet needs radius > 0, Rd > 0, Cp > Rd, p_ref > 0");
    return false;
  }
  if (v->n_lev < 1 || v->n_lev > 64 || !(v->z_top > 0)) {
    set_error("thor_state_init: n_lev must be 1..64 and z_top > 0");
    return false;
  }
  if (!(num->dt > 0) || !(num->diff_D >= 0) || (num->precision != THOR_FP64 && num->precision != THOR_MIXED) ||
      (num->div_damp != 0 && num->div_damp != 1) || (num->energy_fixer != 0 && num->energy_fixer != 1) ||
      (num->hydrostatic != 0 && num->hydrostatic != 1) || (num->shallow != 0 && num->shallow != 1) ||
      (num->lagrange_order < 0 || num->lagrange_order > 3 || num->lagrange_order == 2) ||
      (num->lagrange_order == 3 && v->n_lev < 4) || (num->anelastic != 0 && num->anelastic != 1) ||
      (num->anelastic && num->lagrange_order == 3)) {
    set_error("thor_state_init: numerics need dt > 0, diff_D >= 0, precision FP64|MIXED, div_damp 0|1, "
              "energy_fixer 0|1, hydrostatic 0|1, shallow 0|1, lagrange_order 0, 1 or 3 (3: n_lev >= 4), "
              "anelastic 0|1 (1: lagrange_order 0 or 1)");
    return false;
  }
  if (fo->kind != THOR_FORCING_NONE && fo->kind != THOR_FORCING_NEWTONIAN && fo->kind != THOR_FORCING_HOT_JUPITER &&
      fo->kind != THOR_FORCING_HELD_SUAREZ) {
    set_error("thor_state_init: unknown forcing kind");
    return false;
  }
  if (fo->kind == THOR_FORCING_HELD_SUAREZ &&
      !(fo->k_f >= 0 && fo->k_a >= 0 && fo->k_s >= 0 && fo->sigma_b >= 0 && fo->sigma_b < 1 && fo->p_star > 0 &&
        fo->T_min > 0 && fo->T_top > 0)) {
    set_error("thor_state_init: Held-Suarez forcing needs rates >= 0, 0 <= sigma_b < 1, p_star > 0, T_min, T_top > 0");
    return false;
  }
  if ((fo->kind == THOR_FORCING_NEWTONIAN || fo->kind == THOR_FORCING_HOT_JUPITER) && !(fo->tau > 0)) {
    set_error("thor_state_init: Newtonian forcing needs tau > 0");
    return false;
  }
  if (fo->kind == THOR_FORCING_HOT_JUPITER &&
      !(fo->T_mean > 0 && fo->lapse >= 0 && fo->z_strat > 0 && fo->dT_strat >= 0 && fo->sigma_strat >= 0 &&
        fo->sigma_strat < 1)) {
    set_error("thor_state_init: hot-Jupiter forcing needs T_mean > 0, lapse >= 0, z_strat > 0, dT_strat >= 0, "
              "0 <= sigma_strat < 1");
    return false;
  }
  if (!(in->T0 > 0 && in->p_surf > 0 && in->noise_amp >= 0 && in->noise_amp < in->T0)) {
    set_error("thor_state_init: init needs T0 > 0, p_surf > 0, 0 <= noise_amp < T0");
    return false;
  }
  if (in->planet_index < 0 || in->planet_index > 0xFFFFFF) {
    set_error("thor_state_init: planet_index out of range");
    return false;
  }
  double dz = v->z_top / v->n_lev;
  if (!(0.5 * pl->gravity * dz < pl->Rd * in->T0)) {
    set_error("thor_state_init: layers too thick for a discrete hydrostatic state (g dz / 2 >= Rd T0)");
    return false;
  }
  return true;
}

size_t bytes_for(int precision, size_t N, size_t L, bool anelastic) {
  Carver cv{nullptr};
  if (precision == THOR_MIXED) {
    Fields<float> f;
    carve(cv, f, N, L, anelastic);
  } else {
    Fields<double> f;
    carve(cv, f, N, L, anelastic);
  }
  return cv.off;
}

template <typename H>
int upload(thor_state *s, const Grid &G, const thor_planet *pl, const thor_vertical *v,
           const thor_forcing *fo, const thor_init *in, char *base, Fields<H> *fp) {
  Carver cv{base};
  const size_t N = G.n, L = v->n_lev, S = row_stride(L), NL = N * S;
  carve(cv, fp[0], N, L, s->c.anelastic != 0);
  // every array starts at zero (padding levels included)
  if (!hip_ok(hipMemsetAsync(base, 0, cv.off, s->stream), "clear state")) return THOR_EHIP;
  fp[1] = swapped(fp[0]);
  const Fields<H> &f = fp[0];
  const Consts &c = s->c;
  // geometry
  std::vector<H> dc(G.div_coef.begin(), G.div_coef.end());
  std::vector<H> lc(G.lap_coef.begin(), G.lap_coef.end());
  std::vector<H> rh(N * 3);
  std::vector<H> ddw(G.dd_w.begin(), G.dd_w.end());
  std::vector<double> teq(N);
  for (size_t i = 0; i < N; ++i) {
    const Vec3 p = G.pos[i];
    rh[3 * i] = (H)p.x;
    rh[3 * i + 1] = (H)p.y;
    rh[3 * i + 2] = (H)p.z;
    double lam = std::sqrt(p.x * p.x + p.y * p.y) < 1e-12 ? 0.0 : std::atan2(p.y, p.x);
    double phi = std::asin(std::fmin(1.0, std::fmax(-1.0, p.z)));
    // NEWTONIAN: T_eq itself; HOT_JUPITER: its horizontal factor cos(lon - lon_ss) cos(lat)
    // HELD_SUAREZ: sin(lat)
    teq[i] = fo->kind == THOR_FORCING_HOT_JUPITER ? std::cos(lam - fo->lon_substellar) * std::cos(phi)
             : fo->kind == THOR_FORCING_HELD_SUAREZ
                 ? std::sin(phi)
                 : fo->T_mean + 0.5 * fo->dT_daynight * std::cos(phi) * std::cos(lam - fo->lon_substellar);
  }
  // initial state: isothermal columns in discrete hydrostatic balance
  std::vector<double> rcol(L), pcol(L);
  const double RT = pl->Rd * in->T0, half = 0.5 * pl->gravity * c.dz;
  rcol[0] = in->p_surf * std::exp(-half / RT) / RT;
  for (size_t k = 1; k < L; ++k) rcol[k] = rcol[k - 1] * (RT - half) / (RT + half);
  for (size_t k = 0; k < L; ++k) pcol[k] = rcol[k] * RT;
  // anelastic reference column: the same isothermal column, padded to S
  std::vector<double> rref(S);
  for (size_t k = 0; k < S; ++k) rref[k] = rcol[k < L ? k : L - 1];
  std::vector<double> rho(NL), rth(NL), zero(NL, 0.0);
  std::vector<H> zeroH(NL, (H)0);
  const uint64_t pbase = (uint64_t)in->planet_index << 40;
  for (size_t i = 0; i < N; ++i)
    for (size_t k = 0; k < L; ++k) {
      uint64_t z = splitmix64(in->seed ^ (pbase + ((uint64_t)i << 20) + k));
      double u = (double)(z >> 11) * 0x1.0p-53;
      double T = in->T0 + in->noise_amp * (2.0 * u - 1.0);
      double p = pcol[k];
      rho[i * S + k] = p / (pl->Rd * T);
      rth[i * S + k] = pl->p_ref / pl->Rd * std::pow(p / pl->p_ref, 1.0 / c.gamma);
    }
  // padding levels repeat the top level (finite, positive density)
  for (size_t i = 0; i < N; ++i)
    for (size_t k = L; k < S; ++k) {
      rho[i * S + k] = rho[i * S + L - 1];
      rth[i * S + k] = rth[i * S + L - 1];
    }
  hipStream_t st = s->stream;
  bool ok = hip_ok(hipMemcpyAsync((void *)f.nbr, G.nbr.data(), N * 6 * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy nbr") &&
            hip_ok(hipMemcpyAsync((void *)f.dc, dc.data(), dc.size() * sizeof(H), hipMemcpyHostToDevice, st), "copy dc") &&
            hip_ok(hipMemcpyAsync((void *)f.lc, lc.data(), lc.size() * sizeof(H), hipMemcpyHostToDevice, st), "copy lc") &&
            hip_ok(hipMemcpyAsync((void *)f.rhat, rh.data(), rh.size() * sizeof(H), hipMemcpyHostToDevice, st), "copy rhat") &&
            hip_ok(hipMemcpyAsync((void *)f.ddi, G.dd_idx.data(), G.dd_idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy ddi") &&
            hip_ok(hipMemcpyAsync((void *)f.ddw, ddw.data(), ddw.size() * sizeof(H), hipMemcpyHostToDevice, st), "copy ddw") &&
            hip_ok(hipMemcpyAsync((void *)f.area, G.area.data(), N * sizeof(double), hipMemcpyHostToDevice, st), "copy area") &&
            hip_ok(hipMemcpyAsync((void *)f.teq, teq.data(), N * sizeof(double), hipMemcpyHostToDevice, st), "copy teq") &&
            hip_ok(hipMemcpyAsync(f.rho_t, rho.data(), NL * sizeof(double), hipMemcpyHostToDevice, st), "copy rho") &&
            hip_ok(hipMemcpyAsync(f.rth_t, rth.data(), NL * sizeof(double), hipMemcpyHostToDevice, st), "copy rth") &&
            hip_ok(hipMemcpyAsync(f.W_t, zero.data(), NL * sizeof(double), hipMemcpyHostToDevice, st), "copy W") &&
            hip_ok(hipMemcpyAsync(f.Mx_t, zeroH.data(), NL * sizeof(H), hipMemcpyHostToDevice, st), "copy Mx") &&
            hip_ok(hipMemcpyAsync(f.My_t, zeroH.data(), NL * sizeof(H), hipMemcpyHostToDevice, st), "copy My") &&
            hip_ok(hipMemcpyAsync(f.Mz_t, zeroH.data(), NL * sizeof(H), hipMemcpyHostToDevice, st), "copy Mz") &&
            hip_ok(hipMemcpyAsync(f.ps, zeroH.data(), NL * sizeof(H), hipMemcpyHostToDevice, st), "copy ps") &&
            (!f.rref || hip_ok(hipMemcpyAsync((void *)f.rref, rref.data(), S * sizeof(double),
                                              hipMemcpyHostToDevice, st), "copy rref")) &&
            hip_ok(hipStreamSynchronize(st), "init synchronize");
  return ok ? THOR_OK : THOR_EHIP;
}

hipEvent_t next_event(thor_state *s) {
  if (s->next_event == s->event_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->event_pool.push_back(e);
  }
  return s->event_pool[s->next_event++];
}

// Enqueue one kernel family; when timing is on, the dispatches themselves
// record a start event (first kernel) and an end event (last kernel), so the
// interval is the family's execution without event-packet overheads.
template <typename F>
void timed(thor_state *s, hipStream_t st, const char *family, F &&launch) {
  if (!s->timing) {
    launch(nullptr, nullptr);
    return;
  }
  hipEvent_t a = next_event(s), b = next_event(s);
  launch(a, b);
  s->timed.push_back({family, a, b});
}

template <typename H>
void enqueue_large_step(thor_state *s, const Fields<H> &f, int n, hipStream_t st) {
  const Consts &c = s->c;
  const int *it = s->wpb;
  if (c.energy_fixer) {   // energy of the step's start (not a timed family)
    int nb = 0;
    launch_energy(f, c, 0, f.epart, st, &nb);
  }
  timed(s, st, "large", [&](hipEvent_t a, hipEvent_t b) { launch_large(f, c, it[FAM_LARGE], st, a, b); });
  const int ns[3] = {1, n / 2, n};
  const int div[3] = {3, n, n};   // dtau = dt / div
  for (int stage = 0; stage < 3; ++stage) {
    timed(s, st, "slow", [&](hipEvent_t a, hipEvent_t b) { launch_slow(f, c, it[FAM_SLOW], stage == 0, st, a, b); });
    for (int i = 0; i < ns[stage]; ++i) {
      const bool first = i == 0, last = stage == 2 && i + 1 == ns[stage];
      timed(s, st, "hmom",
            [&](hipEvent_t a, hipEvent_t b) { launch_hmom(f, c, it[FAM_HMOM], div[stage], first, st, a, b); });
      timed(s, st, "vert", [&](hipEvent_t a, hipEvent_t b) {
        launch_vert(f, c, it[FAM_VERT], div[stage], first, last && !c.energy_fixer, st, a, b);
      });
    }
  }
  if (c.energy_fixer) launch_fixer(f, c, st);
}

void enqueue(thor_state *s, int n, int parity, hipStream_t st) {
  if (s->precision == THOR_MIXED) enqueue_large_step(s, s->f32[parity], n, st);
  else enqueue_large_step(s, s->f64[parity], n, st);
}

int graph_for(thor_state *s, int n, int parity, hipGraphExec_t *out) {
  const int key = 2 * n + parity;
  auto it = s->graphs.find(key);
  if (it != s->graphs.end()) {
    *out = it->second;
    return THOR_OK;
  }
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (!hip_ok(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed), "graph capture")) return THOR_EHIP;
  enqueue(s, n, parity, s->cap_stream);
  if (!hip_ok(hipStreamEndCapture(s->cap_stream, &g), "graph end capture")) return THOR_EHIP;
  if (!hip_ok(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate")) {
    (void)hipGraphDestroy(g);
    return THOR_EHIP;
  }
  (void)hipGraphDestroy(g);
  s->graphs[key] = ex;
  *out = ex;
  return THOR_OK;
}

void drop_graphs(thor_state *s) {
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
}

// Mean duration [ms] of one kernel family over the launches recorded while
// timing was on.
double family_mean(thor_state *s, const char *name, int *count) {
  double sum = 0.0;
  int n = 0;
  for (auto &t : s->timed)
    if (t.family == name) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) continue;
      sum += ms;
      ++n;
    }
  if (count) *count = n;
  return n ? sum / n : 0.0;
}

template <typename H>
int diag_impl(thor_state *s, const Fields<H> &f, int kind, int field, void *host_out, size_t out_bytes) {
  const Consts &c = s->c;
  const size_t NL = (size_t)c.N * c.L;
  hipStream_t st = s->stream;
  if (kind == THOR_DIAG_FIELD) {
    if (field < THOR_F_T || field > THOR_F_WI) { set_error("thor_diag: unknown field"); return THOR_EINVAL; }
    if (out_bytes < NL * sizeof(double)) { set_error("thor_diag: out_bytes too small"); return THOR_EINVAL; }
  } else if (kind == THOR_DIAG_MASS) {
    if (out_bytes < sizeof(double)) { set_error("thor_diag: out_bytes too small"); return THOR_EINVAL; }
  } else if (kind == THOR_DIAG_SCALARS) {
    if (out_bytes < sizeof(thor_scalars)) { set_error("thor_diag: out_bytes too small"); return THOR_EINVAL; }
  } else if (kind == THOR_DIAG_ENERGY || kind == THOR_DIAG_ANGULAR_MOMENTUM) {
    if (out_bytes < sizeof(double)) { set_error("thor_diag: out_bytes too small"); return THOR_EINVAL; }
  } else if (kind == THOR_DIAG_STATE_EXPORT) {
    if (out_bytes < thor_state_blob_bytes(s)) { set_error("thor_diag: out_bytes too small"); return THOR_EINVAL; }
  } else {
    set_error("thor_diag: unknown kind");
    return THOR_EINVAL;
  }
  // mass and non-finite scan
  int nb = 0;
  launch_mass(f, c, st, &nb);
  std::vector<double> part(2 * (size_t)nb);
  if (!hip_ok(hipMemcpyAsync(part.data(), f.partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy partial") ||
      !hip_ok(hipStreamSynchronize(st), "diag synchronize"))
    return THOR_EHIP;
  double mass = 0.0, bad = 0.0;
  for (int i = 0; i < nb; ++i) {
    mass += part[2 * i];
    bad += part[2 * i + 1];
  }
  auto field_to_host = [&](int fld, double *dst) -> bool {
    launch_diag_field(f, c, fld, st);
    return hip_ok(hipMemcpyAsync(dst, f.diag, NL * sizeof(double), hipMemcpyDeviceToHost, st), "copy field") &&
           hip_ok(hipStreamSynchronize(st), "diag synchronize");
  };
  if (kind == THOR_DIAG_MASS) {
    *(double *)host_out = mass;
  } else if (kind == THOR_DIAG_ENERGY) {
    int ne = 0;
    launch_energy(f, c, 0, f.partial, st, &ne);
    std::vector<double> ep(2 * (size_t)ne);
    if (!hip_ok(hipMemcpyAsync(ep.data(), f.partial, ep.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy energy") ||
        !hip_ok(hipStreamSynchronize(st), "diag synchronize"))
      return THOR_EHIP;
    double e = 0.0;
    for (int i = 0; i < ne; ++i) e += ep[2 * i];
    *(double *)host_out = e;
  } else if (kind == THOR_DIAG_ANGULAR_MOMENTUM) {
    int na = 0;
    launch_angmom(f, c, f.partial, st, &na);
    std::vector<double> ap((size_t)na);
    if (!hip_ok(hipMemcpyAsync(ap.data(), f.partial, ap.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy angular momentum") ||
        !hip_ok(hipStreamSynchronize(st), "diag synchronize"))
      return THOR_EHIP;
    double a = 0.0;
    for (int i = 0; i < na; ++i) a += ap[i];
    *(double *)host_out = a;
  } else if (kind == THOR_DIAG_FIELD) {
    if (!field_to_host(field, (double *)host_out)) return THOR_EHIP;
  } else if (kind == THOR_DIAG_SCALARS) {
    std::vector<double> a(NL), b(NL), w(NL);
    thor_scalars sc{};
    sc.mass = mass;
    if (!field_to_host(THOR_F_U, a.data()) || !field_to_host(THOR_F_V, b.data()) || !field_to_host(THOR_F_W, w.data()))
      return THOR_EHIP;
    double ms = 0, mw = 0;
    for (size_t i = 0; i < NL; ++i) {
      ms = std::fmax(ms, std::sqrt(a[i] * a[i] + b[i] * b[i] + w[i] * w[i]));
      mw = std::fmax(mw, std::fabs(w[i]));
    }
    if (!field_to_host(THOR_F_T, a.data())) return THOR_EHIP;
    double tmin = a[0], tmax = a[0];
    for (size_t i = 0; i < NL; ++i) {
      tmin = std::fmin(tmin, a[i]);
      tmax = std::fmax(tmax, a[i]);
    }
    sc.max_speed = ms;
    sc.max_w = mw;
    sc.min_T = tmin;
    sc.max_T = tmax;
    std::memcpy(host_out, &sc, sizeof(sc));
  } else {
    // checkpoint: header (magic, N, L) then rho, Mx, My, Mz, rho theta, W
    double *out = (double *)host_out;
    out[0] = 1953460050.0;  // 'THOR' tag
    out[1] = (double)c.N;
    out[2] = (double)c.L;
    out[3] = 0.0;
    const int flds[6] = {THOR_F_RHO, THOR_F_MX, THOR_F_MY, THOR_F_MZ, THOR_F_RHOTHETA, THOR_F_WI};
    for (int i = 0; i < 6; ++i)
      if (!field_to_host(flds[i], out + 4 + i * NL)) return THOR_EHIP;
  }
  if (bad > 0) {
    set_error("thor_diag: state holds non-finite values");
    return THOR_ENONFINITE;
  }
  return THOR_OK;
}

}  // namespace

extern "C" {

const char *thor_last_error(void) { return g_err.c_str(); }

int thor_state_bytes(const thor_grid *g, const thor_vertical *v, const thor_numerics *num, size_t *bytes) {
  clear_error();
  if (!g || !v || !num || !bytes) { set_error("thor_state_bytes: NULL argument"); return THOR_EINVAL; }
  if (v->n_lev < 1 || v->n_lev > 64) { set_error("thor_state_bytes: n_lev must be 1..64"); return THOR_EINVAL; }
  if (num->precision != THOR_FP64 && num->precision != THOR_MIXED) { set_error("thor_state_bytes: bad precision"); return THOR_EINVAL; }
  *bytes = bytes_for(num->precision, (size_t)g->g.n, (size_t)v->n_lev, num->anelastic == 1);
  return THOR_OK;
}

int thor_state_init(const thor_grid *g, const thor_planet *pl, const thor_vertical *v,
                    const thor_numerics *num, const thor_forcing *fo, const thor_init *in,
                    void *dev_buf, size_t dev_bytes, void *hip_stream, thor_state **out) {
  clear_error();
  if (!g || !out || !dev_buf) { set_error("thor_state_init: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  if (!validate(pl, v, num, fo, in)) return THOR_EINVAL;
  if (((uintptr_t)dev_buf & 255) != 0) { set_error("thor_state_init: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  const size_t need = bytes_for(num->precision, (size_t)g->g.n, (size_t)v->n_lev, num->anelastic == 1);
  if (dev_bytes < need) {
    set_error("thor_state_init: dev_bytes smaller than thor_state_bytes");
    return THOR_ENOMEM;
  }
  thor_state *s = new (std::nothrow) thor_state;
  if (!s) { set_error("thor_state_init: out of host memory"); return THOR_ENOMEM; }
  s->precision = num->precision;
  s->stream = (hipStream_t)hip_stream;
  s->n_col = g->g.n;
  s->n_lev = v->n_lev;
  Consts &c = s->c;
  c.N = (int)g->g.n;
  c.L = v->n_lev;
  c.S = (int)row_stride(v->n_lev);
  c.cpw = 64 / v->n_lev;
  c.hlpc = (v->n_lev + kHq - 1) / kHq;
  c.hcpw = 64 / c.hlpc;
  c.radius = pl->radius;
  c.omega = pl->omega;
  c.grav = pl->gravity;
  c.Rd = pl->Rd;
  c.Cp = pl->Cp;
  c.Cv = pl->Cp - pl->Rd;
  c.gamma = pl->Cp / c.Cv;
  c.p_ref = pl->p_ref;
  c.dz = v->z_top / v->n_lev;
  const double dbar = std::sqrt(2.0 * M_PI / 5.0) * pl->radius / std::ldexp(1.0, g->g.glevel);  // Eq. grid_qts
  c.Kd = num->diff_D * std::pow(dbar, 4) / num->dt;                                             // Eq. kd
  c.dt = num->dt;
  c.div_damp = num->div_damp;
  c.energy_fixer = num->energy_fixer;
  c.hydrostatic = num->hydrostatic;
  c.shallow = num->shallow;
  c.rdz = num->shallow ? 0.0 : c.dz;
  c.vorder = num->lagrange_order == 3 ? 3 : 1;
  c.anelastic = num->anelastic;
  // phase V: four levels per lane (the gather mapping), as in the ensemble
  // kernels, so that a planet's results equal its ensemble member's bitwise;
  // with cubic interpolation one level per lane.  thor_autotune may choose
  // another mapping.
  c.vnl = c.vorder == 1 ? 4 : 1;
  c.vlpc = (c.L + 1) / 2;
  c.vcpw = 64 / c.vlpc;
  c.forcing = fo->kind;
  c.tau = (fo->kind == THOR_FORCING_NEWTONIAN || fo->kind == THOR_FORCING_HOT_JUPITER) ? fo->tau : 1.0;
  c.hs_kf = fo->k_f;
  c.hs_ka = fo->k_a;
  c.hs_ks = fo->k_s;
  c.hs_sb = fo->sigma_b;
  c.hs_dTy = fo->dT_y;
  c.hs_dthz = fo->dtheta_z;
  c.hs_pstar = fo->p_star;
  c.hs_Ttop = fo->T_top;
  c.hs_Tmin = fo->T_min;
  c.hj_Tsurf = fo->T_mean;
  c.hj_dTep = fo->dT_daynight;
  c.hj_lapse = fo->lapse;
  c.hj_zstrat = fo->z_strat;
  c.hj_dTstrat = fo->dT_strat;
  c.hj_sstrat = fo->sigma_strat;
  if (!hip_ok(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking), "capture stream")) {
    delete s;
    return THOR_EHIP;
  }
  int rc;
  try {
    rc = s->precision == THOR_MIXED ? upload(s, g->g, pl, v, fo, in, (char *)dev_buf, s->f32)
                                    : upload(s, g->g, pl, v, fo, in, (char *)dev_buf, s->f64);
  } catch (const std::bad_alloc &) {
    set_error("thor_state_init: out of host memory");
    rc = THOR_ENOMEM;
  }
  if (rc != THOR_OK) {
    (void)hipStreamDestroy(s->cap_stream);
    delete s;
    return rc;
  }
  *out = s;
  return THOR_OK;
}

int thor_step(thor_state *s, int n_large, int n_acoustic) {
  clear_error();
  if (!s) { set_error("thor_step: NULL state"); return THOR_EINVAL; }
  if (n_large < 0) { set_error("thor_step: n_large must be >= 0"); return THOR_EINVAL; }
  if (n_acoustic < 2 || (n_acoustic & 1)) { set_error("thor_step: n_acoustic must be even and >= 2"); return THOR_EINVAL; }
  if (s->in_batch) { set_error("thor_step: this state is an ensemble member; use thor_batch_step"); return THOR_EINVAL; }
  if (n_large == 0) return THOR_OK;
  if (s->timing) {
    for (int i = 0; i < n_large; ++i) {
      enqueue(s, n_acoustic, s->parity, s->stream);
      s->parity ^= 1;
    }
    return hip_ok(hipGetLastError(), "kernel launch") ? THOR_OK : THOR_EHIP;
  }
  for (int i = 0; i < n_large; ++i) {
    hipGraphExec_t ex;
    int rc = graph_for(s, n_acoustic, s->parity, &ex);
    if (rc != THOR_OK) return rc;
    if (!hip_ok(hipGraphLaunch(ex, s->stream), "graph launch")) return THOR_EHIP;
    s->parity ^= 1;
  }
  return THOR_OK;
}

int thor_autotune(thor_state *s, int n_acoustic, int *iters_out) {
  clear_error();
  if (!s) { set_error("thor_autotune: NULL state"); return THOR_EINVAL; }
  if (n_acoustic < 2 || (n_acoustic & 1)) { set_error("thor_autotune: n_acoustic must be even and >= 2"); return THOR_EINVAL; }
  // Tune on real large steps (the kernels see the caches as in production),
  // one family at a time, then restore the state from a checkpoint.
  static const int cand[] = {1, 2, 4, 8};
  std::vector<double> blob(thor_state_blob_bytes(s) / sizeof(double));
  int rc = thor_diag(s, THOR_DIAG_STATE_EXPORT, 0, blob.data(), blob.size() * sizeof(double));
  if (rc != THOR_OK && rc != THOR_ENONFINITE) return rc;
  const int parity0 = s->parity;
  const bool timing0 = s->timing;
  // phase V may also choose its mapping: one level per lane, two (L > 32)
  // or four (the gather mapping), with linear interpolation
  // (the anelastic switch has the four-level mapping only)
  const bool two_ok = s->c.L > 32 && s->c.vorder == 1 && !s->c.anelastic;
  const bool four_ok = s->c.vorder == 1;
  const bool one_ok = !s->c.anelastic;
  for (int fam = 0; fam < FAM_COUNT; ++fam) {
    double best = 1e30;
    int best_it = s->wpb[fam], best_nl = s->c.vnl;
    for (int k = 0; k < 12; ++k) {
      const int it = cand[k & 3], nl = k < 4 ? 1 : k < 8 ? 2 : 4;
      if (nl != 1 && fam != FAM_VERT) continue;
      if ((nl == 2 && !two_ok) || (nl == 4 && !four_ok)) continue;
      if (nl == 1 && fam == FAM_VERT && !one_ok) continue;
      if (fam == FAM_VERT) s->c.vnl = nl;
      s->wpb[fam] = it;
      s->timing = true;
      s->timed.clear();
      s->next_event = 0;
      enqueue(s, n_acoustic, s->parity, s->stream);
      s->parity ^= 1;
      s->timed.clear();   // first step warms up; time the next two
      s->next_event = 0;
      for (int r = 0; r < 2; ++r) {
        enqueue(s, n_acoustic, s->parity, s->stream);
        s->parity ^= 1;
      }
      if (!hip_ok(hipStreamSynchronize(s->stream), "autotune synchronize")) return THOR_EHIP;
      int cnt = 0;
      double ms = family_mean(s, kFamily[fam], &cnt);
      if (cnt > 0 && ms < best) {
        best = ms;
        best_it = it;
        best_nl = s->c.vnl;
      }
    }
    s->wpb[fam] = best_it;
    s->c.vnl = best_nl;
  }
  s->timing = timing0;
  s->timed.clear();
  s->next_event = 0;
  drop_graphs(s);
  s->parity = parity0;
  rc = thor_state_import(s, blob.data(), blob.size() * sizeof(double));
  if (rc != THOR_OK) return rc;
  if (iters_out)
    for (int k = 0; k < FAM_COUNT; ++k) iters_out[k] = s->wpb[k];
  return THOR_OK;
}

int thor_diag(thor_state *s, int kind, int field, void *host_out, size_t out_bytes) {
  clear_error();
  if (!s || !host_out) { set_error("thor_diag: NULL argument"); return THOR_EINVAL; }
  return s->precision == THOR_MIXED ? diag_impl(s, s->f32[s->parity], kind, field, host_out, out_bytes)
                                    : diag_impl(s, s->f64[s->parity], kind, field, host_out, out_bytes);
}

size_t thor_state_blob_bytes(const thor_state *s) {
  if (!s) return 0;
  return (4 + 6 * (size_t)s->c.N * s->c.L) * sizeof(double);
}

int thor_state_import(thor_state *s, const void *blob, size_t bytes) {
  clear_error();
  if (!s || !blob) { set_error("thor_state_import: NULL argument"); return THOR_EINVAL; }
  const double *b = (const double *)blob;
  if (bytes != thor_state_blob_bytes(s) || b[0] != 1953460050.0 || b[1] != (double)s->c.N || b[2] != (double)s->c.L) {
    set_error("thor_state_import: blob does not match this state");
    return THOR_EINVAL;
  }
  const size_t NL = (size_t)s->c.N * s->c.L;
  double *stage = s->precision == THOR_MIXED ? s->f32[0].diag : s->f64[0].diag;
  if (!hip_ok(hipMemcpyAsync(stage, b + 4, 6 * NL * sizeof(double), hipMemcpyHostToDevice, s->stream), "copy blob"))
    return THOR_EHIP;
  if (s->precision == THOR_MIXED) launch_to_state(s->f32[s->parity], s->c, stage, s->stream);
  else launch_to_state(s->f64[s->parity], s->c, stage, s->stream);
  return hip_ok(hipStreamSynchronize(s->stream), "import synchronize") ? THOR_OK : THOR_EHIP;
}

int thor_set_vert_levels_per_lane(thor_state *s, int nl) {
  clear_error();
  if (!s) { set_error("thor_set_vert_levels_per_lane: NULL state"); return THOR_EINVAL; }
  if ((nl != 1 && ((nl != 2 && nl != 4) || s->c.vorder != 1 || (nl == 2 && s->c.L <= 32))) ||
      (s->c.anelastic && nl != 4)) {
    set_error("thor_set_vert_levels_per_lane: 1, 4 with linear interpolation, or 2 with 33..64 levels and linear "
              "interpolation; 4 only with the anelastic switch");
    return THOR_EINVAL;
  }
  if (!hip_ok(hipStreamSynchronize(s->stream), "vert mapping synchronize")) return THOR_EHIP;
  if (s->c.vnl != nl) {
    s->c.vnl = nl;
    drop_graphs(s);   // captured launches carry the old mapping
  }
  return THOR_OK;
}

int thor_set_timing(thor_state *s, int on) {
  clear_error();
  if (!s) { set_error("thor_set_timing: NULL state"); return THOR_EINVAL; }
  if (!hip_ok(hipStreamSynchronize(s->stream), "timing synchronize")) return THOR_EHIP;
  s->timing = on != 0;
  s->timed.clear();
  s->next_event = 0;
  return THOR_OK;
}

int thor_kernel_time(thor_state *s, const char *name, double *mean_ms, int *count) {
  clear_error();
  if (!s || !name || !mean_ms || !count) { set_error("thor_kernel_time: NULL argument"); return THOR_EINVAL; }
  bool ok = false;
  for (auto k : kFamily) ok = ok || std::strcmp(k, name) == 0;
  if (!ok) { set_error("thor_kernel_time: unknown kernel family"); return THOR_EINVAL; }
  if (!hip_ok(hipStreamSynchronize(s->stream), "timing synchronize")) return THOR_EHIP;
  *mean_ms = family_mean(s, name, count);
  return THOR_OK;
}

void thor_state_free(thor_state *s) {
  if (!s) return;
  drop_graphs(s);
  for (auto e : s->event_pool) (void)hipEventDestroy(e);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

}  // extern "C"

// ===========================================================================
// Ensembles: many planets, each its own grid level, level count and
// constants, advanced together with one launch per phase (a tile table maps
// every workgroup to a planet and a local workgroup), the whole large step
// captured in one HIP graph.
// ===========================================================================
struct thor_batch {
  int n = 0;
  int precision = THOR_FP64;
  std::vector<thor_state *> members;
  std::vector<size_t> member_bytes;
  void *tables = nullptr;          // device: Planet<H>[n], then FAM_COUNT tile tables
  size_t tile_cap = 0;             // entries reserved per tile table
  int n_tiles[FAM_COUNT] = {0, 0, 0, 0};
  int wpb[FAM_COUNT] = {4, 4, 4, 4};
  int parity = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::map<int, hipGraphExec_t> graphs;
};

namespace {

size_t batch_tile_cap(int n, const thor_grid *const *grids, const thor_vertical *v) {
  size_t cap = kXcds;
  for (int i = 0; i < n; ++i) {
    const size_t cpw = 64 / v[i].n_lev;
    cap += (grids[i]->g.n + cpw - 1) / cpw;   // one-wavefront workgroups at most
  }
  return cap;
}

template <typename H>
size_t planet_table_bytes(int n) { return align256(sizeof(Planet<H>) * n); }

template <typename H>
Planet<H> *planet_table(thor_batch *b) { return reinterpret_cast<Planet<H> *>(b->tables); }

int2 *tile_table(thor_batch *b, int fam, size_t planet_bytes) {
  char *base = reinterpret_cast<char *>(b->tables) + planet_bytes;
  return reinterpret_cast<int2 *>(base) + (size_t)fam * b->tile_cap;
}

// (planet, local workgroup) of every logical workgroup, padded with (-1, 0)
// to a multiple of kXcds; planets are laid out one after the other so each
// XCD gets a contiguous run of columns.
int upload_tiles(thor_batch *b, size_t planet_bytes) {
  for (int fam = 0; fam < FAM_COUNT; ++fam) {
    std::vector<int2> t;
    for (int i = 0; i < b->n; ++i) {
      const Consts &c = b->members[i]->c;
      const int cols = c.hcpw;   // every ensemble kernel runs on the gather mapping
      const long waves = (c.N + cols - 1) / cols;
      const long wg = (waves + b->wpb[fam] - 1) / b->wpb[fam];
      for (long k = 0; k < wg; ++k) t.push_back(make_int2(i, (int)k));
    }
    while (t.size() % kXcds) t.push_back(make_int2(-1, 0));
    if (t.size() > b->tile_cap) { set_error("thor_batch: tile table overflow"); return THOR_EINVAL; }
    b->n_tiles[fam] = (int)t.size();
    if (!hip_ok(hipMemcpyAsync(tile_table(b, fam, planet_bytes), t.data(), t.size() * sizeof(int2),
                               hipMemcpyHostToDevice, b->stream), "copy tiles"))
      return THOR_EHIP;
  }
  return hip_ok(hipStreamSynchronize(b->stream), "tiles synchronize") ? THOR_OK : THOR_EHIP;
}

template <typename H>
void enqueue_batch_step(thor_batch *b, int n, int parity, hipStream_t st) {
  const size_t pb = planet_table_bytes<H>(b->n);
  const Planet<H> *P = planet_table<H>(b);
  auto L = [&](int fam, BatchOp op, int a0, int a1) {
    launch_batch<H>(P, tile_table(b, fam, pb), b->n_tiles[fam], b->wpb[fam], parity, op, a0, a1, st);
  };
  L(FAM_LARGE, BatchOp::Large, 0, 0);
  const int ns[3] = {1, n / 2, n};
  const int div[3] = {3, n, n};
  for (int stage = 0; stage < 3; ++stage) {
    L(FAM_SLOW, BatchOp::Slow, stage == 0, 0);
    for (int i = 0; i < ns[stage]; ++i) {
      const bool first = i == 0, last = stage == 2 && i + 1 == ns[stage];
      L(FAM_HMOM, BatchOp::Hmom, div[stage], first);
      L(FAM_VERT, last ? BatchOp::VertLast : BatchOp::Vert, div[stage], first);
    }
  }
}

void batch_enqueue(thor_batch *b, int n, int parity, hipStream_t st) {
  if (b->precision == THOR_MIXED) enqueue_batch_step<float>(b, n, parity, st);
  else enqueue_batch_step<double>(b, n, parity, st);
}

void batch_flip(thor_batch *b) {
  b->parity ^= 1;
  for (auto m : b->members) m->parity = b->parity;
}

void batch_drop_graphs(thor_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

}  // namespace

extern "C" {

int thor_batch_bytes(int n, const thor_grid *const *grids, const thor_vertical *v,
                     const thor_numerics *num, size_t *bytes) {
  clear_error();
  if (n < 1 || !grids || !v || !num || !bytes) { set_error("thor_batch_bytes: bad argument"); return THOR_EINVAL; }
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) { set_error("thor_batch_bytes: NULL grid"); return THOR_EINVAL; }
    if (num[i].precision != num[0].precision) { set_error("thor_batch_bytes: mixed precisions"); return THOR_EINVAL; }
    size_t b = 0;
    int rc = thor_state_bytes(grids[i], &v[i], &num[i], &b);
    if (rc != THOR_OK) return rc;
    total += align256(b);
  }
  const size_t pb = num[0].precision == THOR_MIXED ? planet_table_bytes<float>(n) : planet_table_bytes<double>(n);
  total += pb + align256(FAM_COUNT * batch_tile_cap(n, grids, v) * sizeof(int2));
  *bytes = total;
  return THOR_OK;
}

int thor_batch_init(int n, const thor_grid *const *grids, const thor_planet *pl, const thor_vertical *v,
                    const thor_numerics *num, const thor_forcing *fo, const thor_init *in,
                    void *dev_buf, size_t dev_bytes, void *hip_stream, thor_batch **out) {
  clear_error();
  if (!out || !dev_buf || !pl || !fo || !in) { set_error("thor_batch_init: NULL argument"); return THOR_EINVAL; }
  if (((uintptr_t)dev_buf & 255) != 0) { set_error("thor_batch_init: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  *out = nullptr;
  size_t need = 0;
  int rc = thor_batch_bytes(n, grids, v, num, &need);
  if (rc != THOR_OK) return rc;
  if (dev_bytes < need) { set_error("thor_batch_init: dev_bytes smaller than thor_batch_bytes"); return THOR_ENOMEM; }
  for (int i = 0; i < n; ++i) {
    if (!validate(&pl[i], &v[i], &num[i], &fo[i], &in[i])) return THOR_EINVAL;
    if (num[i].energy_fixer || num[i].shallow || num[i].lagrange_order == 3 || num[i].anelastic) {
      set_error("thor_batch_init: the energy fixer, the shallow-atmosphere form, cubic vertical "
                "interpolation and the anelastic switch are not available in ensembles");
      return THOR_EINVAL;
    }
  }
  thor_batch *b = new (std::nothrow) thor_batch;
  if (!b) { set_error("thor_batch_init: out of host memory"); return THOR_ENOMEM; }
  b->n = n;
  b->precision = num[0].precision;
  b->stream = (hipStream_t)hip_stream;
  char *base = (char *)dev_buf;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    size_t bytes = 0;
    thor_state_bytes(grids[i], &v[i], &num[i], &bytes);
    thor_state *m = nullptr;
    rc = thor_state_init(grids[i], &pl[i], &v[i], &num[i], &fo[i], &in[i], base + off, bytes, hip_stream, &m);
    if (rc != THOR_OK) {
      thor_batch_free(b);
      return rc;
    }
    m->in_batch = true;
    b->members.push_back(m);
    off += align256(bytes);
  }
  b->tables = base + off;
  b->tile_cap = batch_tile_cap(n, grids, v);
  size_t pb;
  bool ok;
  if (b->precision == THOR_MIXED) {
    std::vector<Planet<float>> P(n);
    for (int i = 0; i < n; ++i) {
      P[i].f[0] = b->members[i]->f32[0];
      P[i].f[1] = b->members[i]->f32[1];
      P[i].c = b->members[i]->c;
    }
    pb = planet_table_bytes<float>(n);
    ok = hip_ok(hipMemcpyAsync(b->tables, P.data(), sizeof(Planet<float>) * n, hipMemcpyHostToDevice, b->stream), "copy planets");
  } else {
    std::vector<Planet<double>> P(n);
    for (int i = 0; i < n; ++i) {
      P[i].f[0] = b->members[i]->f64[0];
      P[i].f[1] = b->members[i]->f64[1];
      P[i].c = b->members[i]->c;
    }
    pb = planet_table_bytes<double>(n);
    ok = hip_ok(hipMemcpyAsync(b->tables, P.data(), sizeof(Planet<double>) * n, hipMemcpyHostToDevice, b->stream), "copy planets");
  }
  if (!ok || !hip_ok(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "capture stream")) {
    thor_batch_free(b);
    return THOR_EHIP;
  }
  rc = upload_tiles(b, pb);
  if (rc != THOR_OK) {
    thor_batch_free(b);
    return rc;
  }
  *out = b;
  return THOR_OK;
}

int thor_batch_step(thor_batch *b, int n_large, int n_acoustic) {
  clear_error();
  if (!b) { set_error("thor_batch_step: NULL batch"); return THOR_EINVAL; }
  if (n_large < 0) { set_error("thor_batch_step: n_large must be >= 0"); return THOR_EINVAL; }
  if (n_acoustic < 2 || (n_acoustic & 1)) { set_error("thor_batch_step: n_acoustic must be even and >= 2"); return THOR_EINVAL; }
  for (int i = 0; i < n_large; ++i) {
    const int key = 2 * n_acoustic + b->parity;
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      if (!hip_ok(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed), "graph capture")) return THOR_EHIP;
      batch_enqueue(b, n_acoustic, b->parity, b->cap_stream);
      if (!hip_ok(hipStreamEndCapture(b->cap_stream, &g), "graph end capture")) return THOR_EHIP;
      if (!hip_ok(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate")) {
        (void)hipGraphDestroy(g);
        return THOR_EHIP;
      }
      (void)hipGraphDestroy(g);
      it = b->graphs.emplace(key, ex).first;
    }
    if (!hip_ok(hipGraphLaunch(it->second, b->stream), "graph launch")) return THOR_EHIP;
    batch_flip(b);
  }
  return THOR_OK;
}

int thor_batch_member(thor_batch *b, int i, thor_state **out) {
  clear_error();
  if (!b || !out || i < 0 || i >= b->n) { set_error("thor_batch_member: bad argument"); return THOR_EINVAL; }
  *out = b->members[i];
  return THOR_OK;
}

int thor_batch_autotune(thor_batch *b, int n_acoustic, int *wpb_out) {
  clear_error();
  if (!b) { set_error("thor_batch_autotune: NULL batch"); return THOR_EINVAL; }
  if (n_acoustic < 2 || (n_acoustic & 1)) { set_error("thor_batch_autotune: n_acoustic must be even and >= 2"); return THOR_EINVAL; }
  static const int cand[] = {1, 2, 4, 8};
  std::vector<std::vector<double>> blobs(b->n);
  for (int i = 0; i < b->n; ++i) {
    blobs[i].resize(thor_state_blob_bytes(b->members[i]) / sizeof(double));
    int rc = thor_diag(b->members[i], THOR_DIAG_STATE_EXPORT, 0, blobs[i].data(), blobs[i].size() * sizeof(double));
    if (rc != THOR_OK && rc != THOR_ENONFINITE) return rc;
  }
  const size_t pb = b->precision == THOR_MIXED ? planet_table_bytes<float>(b->n) : planet_table_bytes<double>(b->n);
  hipEvent_t e0, e1;
  if (!hip_ok(hipEventCreate(&e0), "event") || !hip_ok(hipEventCreate(&e1), "event")) return THOR_EHIP;
  // time whole eager large steps for each candidate of one family at a time
  for (int fam = 0; fam < FAM_COUNT; ++fam) {
    double best = 1e30;
    int best_w = b->wpb[fam];
    for (int w : cand) {
      b->wpb[fam] = w;
      int rc = upload_tiles(b, pb);
      if (rc != THOR_OK) return rc;
      batch_enqueue(b, n_acoustic, b->parity, b->stream);   // warm-up
      batch_flip(b);
      (void)hipEventRecord(e0, b->stream);
      for (int r = 0; r < 2; ++r) {
        batch_enqueue(b, n_acoustic, b->parity, b->stream);
        batch_flip(b);
      }
      (void)hipEventRecord(e1, b->stream);
      if (!hip_ok(hipEventSynchronize(e1), "autotune synchronize")) return THOR_EHIP;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_w = w;
      }
    }
    b->wpb[fam] = best_w;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int rc = upload_tiles(b, pb);
  if (rc != THOR_OK) return rc;
  batch_drop_graphs(b);
  for (int i = 0; i < b->n; ++i) {
    rc = thor_state_import(b->members[i], blobs[i].data(), blobs[i].size() * sizeof(double));
    if (rc != THOR_OK) return rc;
  }
  if (wpb_out)
    for (int k = 0; k < FAM_COUNT; ++k) wpb_out[k] = b->wpb[k];
  return THOR_OK;
}

void thor_batch_free(thor_batch *b) {
  if (!b) return;
  batch_drop_graphs(b);
  for (auto m : b->members) thor_state_free(m);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
