// Per-column corrector network on gfx950: multilayer perceptron with GELU
// hidden layers, BF16 operands and FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), forward, backward and Adam on the GPU.
//
// Layout: weights W[out][in] row-major with a transposed copy WT[in][out];
// activations [batch][width] row-major with transposed copies where a
// product reduces over the batch.  Every product is C[M][N] = A[M][K] B[N][K]^T
// with both operands contiguous along K, so one GEMM kernel serves
//   forward    Z  = H_prev W^T          (A = H_prev, B = W)
//   input grad dH = dZ W                (A = dZ,     B = WT)
//   weight grad dW = dZ^T H_prev         (A = dZT,    B = H_prevT)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace thor {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // C tile per workgroup (4 wavefronts of 32 x 32)

// C = A B^T (+ bias), A [M][K], B [N][K] bf16, K % 32 == 0, C fp32 [M][ldc].
// Wavefront w of the workgroup owns rows m0 + 32 (w / 2) .. + 31 and columns
// n0 + 32 (w % 2) .. + 31 as 2 x 2 MFMA tiles of 16 x 16.  In a tile, lane l
// holds A[row l % 16][k0 + 8 (l / 16) .. + 7] and B[col l % 16][same k] and
// accumulates D[4 (l / 16) + i][l % 16], i = 0..3.
__global__ __launch_bounds__(256) void k_gemm_nt(const __bf16 *__restrict__ A, const __bf16 *__restrict__ B,
                                                 float *__restrict__ C, const float *__restrict__ bias,
                                                 int M, int N, int K, int ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * kTile + 32 * (w >> 1);
  const int n0 = blockIdx.y * kTile + 32 * (w & 1);
  const int r = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = {};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) {
      const int row = m0 + 16 * i + r;
      a[i] = row < M ? *reinterpret_cast<const bf16x8 *>(A + (size_t)row * K + k0 + kq) : zero;
      const int col = n0 + 16 * i + r;
      b[i] = col < N ? *reinterpret_cast<const bf16x8 *>(B + (size_t)col * K + k0 + kq) : zero;
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + 16 * j + r;
      if (col >= N) continue;
      const float bb = bias ? bias[col] : 0.f;
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + 16 * i + (lane >> 4) * 4 + q;
        if (row < M) C[(size_t)row * ldc + col] = acc[i][j][q] + bb;
      }
    }
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// H = g(Z) (or Z for the output layer) as bf16 in both layouts.
__global__ void k_activate(const float *Z, __bf16 *H, __bf16 *HT, int B, int N, int act) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)B * N) return;
  const int b = (int)(i / N), n = (int)(i % N);
  const float v = act ? gelu_f(Z[i]) : Z[i];
  H[i] = (__bf16)v;
  if (HT) HT[(size_t)n * B + b] = (__bf16)v;
}

// Transposed bf16 copy: XT[k][b] = X[b][k].
__global__ void k_transpose_bf16(const __bf16 *X, __bf16 *XT, int B, int K) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)B * K) return;
  const int b = (int)(i / K), k = (int)(i % K);
  XT[(size_t)k * B + b] = X[i];
}

// Output layer: dZ = 2 (Y - T) / (B N); per-workgroup partial loss sums.
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *T, float *dZ, __bf16 *dZb,
                                              __bf16 *dZT, float *partial, int B, int N) {
  __shared__ float sm[256];
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < (size_t)B * N) {
    const float d = Y[i] - T[i];
    l = d * d;
    const float g = 2.f * d / ((float)B * (float)N);
    const int b = (int)(i / N), n = (int)(i % N);
    dZ[i] = g;
    dZb[i] = (__bf16)g;
    dZT[(size_t)n * B + b] = (__bf16)g;
  }
  sm[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// Hidden layer: dZ = dH * g'(Z) in fp32 and bf16 (both layouts).
__global__ void k_act_grad(const float *dH, const float *Z, float *dZ, __bf16 *dZb, __bf16 *dZT, int B, int N) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)B * N) return;
  const float g = dH[i] * gelu_grad_f(Z[i]);
  const int b = (int)(i / N), n = (int)(i % N);
  dZ[i] = g;
  dZb[i] = (__bf16)g;
  dZT[(size_t)n * B + b] = (__bf16)g;
}

// db[n] = sum_b dZ[b][n] (fixed order).
__global__ void k_bias_grad(const float *dZ, float *db, int B, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dZ[(size_t)b * N + n];
  db[n] = s;
}

// Adam on the packed fp32 parameters.
__global__ void k_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies W[out][in] and WT[in][out] of one layer's fp32 weights.
__global__ void k_weights_bf16(const float *W, __bf16 *Wb, __bf16 *WT, int out, int in) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)out * in) return;
  const int o = (int)(i / in), k = (int)(i % in);
  Wb[i] = (__bf16)W[i];
  WT[(size_t)k * out + o] = (__bf16)W[i];
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
inline unsigned nb(size_t n, unsigned t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace thor

using namespace thor;

struct thor_mlp {
  int nl = 0;                    // layers
  std::vector<int> w;            // widths, nl + 1
  int max_batch = 0;
  size_t n_params = 0;
  std::vector<size_t> woff, boff;   // offsets of W_l, b_l in the packed arrays
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  std::vector<__bf16 *> Wb, WT;
  __bf16 *XT = nullptr;
  std::vector<float *> Z;        // pre-activations, [B][w_{l+1}]
  std::vector<__bf16 *> H, HT;   // activations of layer outputs (hidden)
  std::vector<float *> dZ;
  std::vector<__bf16 *> dZb, dZT;
  float *dH = nullptr;           // [B][max width]
  float *partial = nullptr;
  int adam_t = 0;
  hipStream_t stream = nullptr;
};

namespace {

bool mlp_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

// Sizes every device array; with base == nullptr only counts bytes.
size_t mlp_layout(thor_mlp *M, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *ptr = base ? base + off : nullptr;
    off += a256(bytes);
    return ptr;
  };
  const int B = M->max_batch, nl = M->nl;
  int wmax = 0;
  for (int x : M->w) wmax = std::max(wmax, x);
  M->p = (float *)take(M->n_params * 4);
  M->g = (float *)take(M->n_params * 4);
  M->m = (float *)take(M->n_params * 4);
  M->v = (float *)take(M->n_params * 4);
  M->Wb.assign(nl, nullptr);
  M->WT.assign(nl, nullptr);
  M->Z.assign(nl, nullptr);
  M->H.assign(nl, nullptr);
  M->HT.assign(nl, nullptr);
  M->dZ.assign(nl, nullptr);
  M->dZb.assign(nl, nullptr);
  M->dZT.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    const size_t wsz = (size_t)M->w[l] * M->w[l + 1];
    M->Wb[l] = (__bf16 *)take(wsz * 2);
    M->WT[l] = (__bf16 *)take(wsz * 2);
    M->Z[l] = (float *)take((size_t)B * M->w[l + 1] * 4);
    M->H[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
    M->HT[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
    M->dZ[l] = (float *)take((size_t)B * M->w[l + 1] * 4);
    M->dZb[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
    M->dZT[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
  }
  M->XT = (__bf16 *)take((size_t)B * M->w[0] * 2);
  M->dH = (float *)take((size_t)B * wmax * 4);
  M->partial = (float *)take((size_t)nb((size_t)B * M->w[nl]) * 4);
  return off;
}

bool mlp_shape(thor_mlp *M, int n_layers, const int *widths, int max_batch) {
  if (n_layers < 1 || n_layers > 16 || !widths || max_batch < 1) {
    set_error("thor_mlp: need 1..16 layers, widths and max_batch >= 1");
    return false;
  }
  M->nl = n_layers;
  M->w.assign(widths, widths + n_layers + 1);
  for (int x : M->w)
    if (x < 1 || x % 32) {
      set_error("thor_mlp: every width must be a positive multiple of 32");
      return false;
    }
  M->max_batch = max_batch;
  M->n_params = 0;
  M->woff.clear();
  M->boff.clear();
  for (int l = 0; l < n_layers; ++l) {
    M->woff.push_back(M->n_params);
    M->n_params += (size_t)M->w[l] * M->w[l + 1];
    M->boff.push_back(M->n_params);
    M->n_params += M->w[l + 1];
  }
  return true;
}

void refresh_bf16(thor_mlp *M) {
  for (int l = 0; l < M->nl; ++l) {
    const size_t n = (size_t)M->w[l] * M->w[l + 1];
    hipLaunchKernelGGL(k_weights_bf16, dim3(nb(n)), dim3(256), 0, M->stream, M->p + M->woff[l], M->Wb[l],
                       M->WT[l], M->w[l + 1], M->w[l]);
  }
}

void gemm(const __bf16 *A, const __bf16 *B, float *C, const float *bias, int Mr, int N, int K, int ldc,
          hipStream_t s) {
  dim3 grid((Mr + kTile - 1) / kTile, (N + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, s, A, B, C, bias, Mr, N, K, ldc);
}

void forward(thor_mlp *M, const __bf16 *X, int B, bool need_t) {
  const __bf16 *in = X;
  for (int l = 0; l < M->nl; ++l) {
    const int K = M->w[l], N = M->w[l + 1];
    gemm(in, M->Wb[l], M->Z[l], M->p + M->boff[l], B, N, K, N, M->stream);
    const bool hidden = l + 1 < M->nl;
    if (hidden) {
      hipLaunchKernelGGL(k_activate, dim3(nb((size_t)B * N)), dim3(256), 0, M->stream, M->Z[l], M->H[l],
                         need_t ? M->HT[l] : nullptr, B, N, 1);
      in = M->H[l];
    }
  }
}

// Gradients of the mean-squared loss into M->g; partial loss sums in M->partial.
void backward(thor_mlp *M, const __bf16 *X, const float *T, int B) {
  const int nl = M->nl;
  hipStream_t s = M->stream;
  hipLaunchKernelGGL(k_transpose_bf16, dim3(nb((size_t)B * M->w[0])), dim3(256), 0, s, X, M->XT, B, M->w[0]);
  const int No = M->w[nl];
  hipLaunchKernelGGL(k_loss, dim3(nb((size_t)B * No)), dim3(256), 0, s, M->Z[nl - 1], T, M->dZ[nl - 1],
                     M->dZb[nl - 1], M->dZT[nl - 1], M->partial, B, No);
  for (int l = nl - 1; l >= 0; --l) {
    const int K = M->w[l], N = M->w[l + 1];
    const __bf16 *prevT = l == 0 ? M->XT : M->HT[l - 1];
    // dW[N][K] = dZ^T H_prev
    gemm(M->dZT[l], prevT, M->g + M->woff[l], nullptr, N, K, B, K, s);
    hipLaunchKernelGGL(k_bias_grad, dim3(nb(N)), dim3(256), 0, s, M->dZ[l], M->g + M->boff[l], B, N);
    if (l > 0) {
      // dH[B][K] = dZ W, then through the activation of layer l-1
      gemm(M->dZb[l], M->WT[l], M->dH, nullptr, B, K, N, K, s);
      hipLaunchKernelGGL(k_act_grad, dim3(nb((size_t)B * K)), dim3(256), 0, s, M->dH, M->Z[l - 1], M->dZ[l - 1],
                         M->dZb[l - 1], M->dZT[l - 1], B, K);
    }
  }
}

// SplitMix64 stream and Box-Muller normals for the initial weights.
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * 0x1.0p-53; }
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(2.0 * M_PI * uniform()); }
};

}  // namespace

extern "C" {

int thor_mlp_bytes(int n_layers, const int *widths, int max_batch, size_t *bytes) {
  clear_error();
  if (!bytes) { set_error("thor_mlp_bytes: NULL argument"); return THOR_EINVAL; }
  thor_mlp M;
  if (!mlp_shape(&M, n_layers, widths, max_batch)) return THOR_EINVAL;
  *bytes = mlp_layout(&M, nullptr);
  return THOR_OK;
}

int thor_mlp_init(int n_layers, const int *widths, int max_batch, uint64_t seed, void *dev_buf,
                  size_t dev_bytes, void *hip_stream, thor_mlp **out) {
  clear_error();
  if (!out || !dev_buf) { set_error("thor_mlp_init: NULL argument"); return THOR_EINVAL; }
  *out = nullptr;
  thor_mlp *M = new (std::nothrow) thor_mlp;
  if (!M) { set_error("thor_mlp_init: out of host memory"); return THOR_ENOMEM; }
  if (!mlp_shape(M, n_layers, widths, max_batch)) { delete M; return THOR_EINVAL; }
  if (dev_bytes < mlp_layout(M, nullptr)) {
    delete M;
    set_error("thor_mlp_init: dev_bytes smaller than thor_mlp_bytes");
    return THOR_ENOMEM;
  }
  if (((uintptr_t)dev_buf & 255) != 0) { delete M; set_error("thor_mlp_init: dev_buf must be 256-byte aligned"); return THOR_EINVAL; }
  mlp_layout(M, (char *)dev_buf);
  M->stream = (hipStream_t)hip_stream;
  // He-style normal weights (std sqrt(2 / in)), zero biases; Adam moments 0
  std::vector<float> host(M->n_params, 0.f);
  Rng rng{seed};
  for (int l = 0; l < M->nl; ++l) {
    const double sd = std::sqrt(2.0 / M->w[l]);
    for (size_t i = 0; i < (size_t)M->w[l] * M->w[l + 1]; ++i) host[M->woff[l] + i] = (float)(sd * rng.normal());
  }
  std::vector<float> zeros(M->n_params, 0.f);
  bool ok = mlp_ok(hipMemcpyAsync(M->p, host.data(), M->n_params * 4, hipMemcpyHostToDevice, M->stream), "copy params") &&
            mlp_ok(hipMemcpyAsync(M->m, zeros.data(), M->n_params * 4, hipMemcpyHostToDevice, M->stream), "copy m") &&
            mlp_ok(hipMemcpyAsync(M->v, zeros.data(), M->n_params * 4, hipMemcpyHostToDevice, M->stream), "copy v");
  if (ok) refresh_bf16(M);
  ok = ok && mlp_ok(hipStreamSynchronize(M->stream), "mlp init synchronize");
  if (!ok) { delete M; return THOR_EHIP; }
  *out = M;
  return THOR_OK;
}

size_t thor_mlp_param_count(const thor_mlp *m) { return m ? m->n_params : 0; }

int thor_mlp_set_params(thor_mlp *m, const float *host) {
  clear_error();
  if (!m || !host) { set_error("thor_mlp_set_params: NULL argument"); return THOR_EINVAL; }
  if (!mlp_ok(hipMemcpyAsync(m->p, host, m->n_params * 4, hipMemcpyHostToDevice, m->stream), "copy params")) return THOR_EHIP;
  refresh_bf16(m);
  m->adam_t = 0;
  std::vector<float> zeros(m->n_params, 0.f);
  bool ok = mlp_ok(hipMemcpyAsync(m->m, zeros.data(), m->n_params * 4, hipMemcpyHostToDevice, m->stream), "zero m") &&
            mlp_ok(hipMemcpyAsync(m->v, zeros.data(), m->n_params * 4, hipMemcpyHostToDevice, m->stream), "zero v") &&
            mlp_ok(hipStreamSynchronize(m->stream), "set params synchronize");
  return ok ? THOR_OK : THOR_EHIP;
}

int thor_mlp_get_params(thor_mlp *m, float *host) {
  clear_error();
  if (!m || !host) { set_error("thor_mlp_get_params: NULL argument"); return THOR_EINVAL; }
  bool ok = mlp_ok(hipMemcpyAsync(host, m->p, m->n_params * 4, hipMemcpyDeviceToHost, m->stream), "copy params") &&
            mlp_ok(hipStreamSynchronize(m->stream), "get params synchronize");
  return ok ? THOR_OK : THOR_EHIP;
}

int thor_mlp_forward(thor_mlp *m, const void *x_bf16, int B, float *y) {
  clear_error();
  if (!m || !x_bf16 || !y) { set_error("thor_mlp_forward: NULL argument"); return THOR_EINVAL; }
  if (B < 1 || B > m->max_batch) { set_error("thor_mlp_forward: batch outside 1..max_batch"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, false);
  const int No = m->w[m->nl];
  return mlp_ok(hipMemcpyAsync(y, m->Z[m->nl - 1], (size_t)B * No * 4, hipMemcpyDeviceToDevice, m->stream), "copy y")
             ? THOR_OK : THOR_EHIP;
}

int thor_mlp_loss_grad(thor_mlp *m, const void *x_bf16, const float *t, int B, double *loss, float *grad_host) {
  clear_error();
  if (!m || !x_bf16 || !t) { set_error("thor_mlp_loss_grad: NULL argument"); return THOR_EINVAL; }
  if (B < 1 || B > m->max_batch || B % 32) { set_error("thor_mlp_loss_grad: batch must be a multiple of 32 within max_batch"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, true);
  backward(m, (const __bf16 *)x_bf16, t, B);
  const size_t np = nb((size_t)B * m->w[m->nl]);
  std::vector<float> part(np);
  if (!mlp_ok(hipMemcpyAsync(part.data(), m->partial, np * 4, hipMemcpyDeviceToHost, m->stream), "copy loss"))
    return THOR_EHIP;
  if (grad_host && !mlp_ok(hipMemcpyAsync(grad_host, m->g, m->n_params * 4, hipMemcpyDeviceToHost, m->stream), "copy grad"))
    return THOR_EHIP;
  if (!mlp_ok(hipStreamSynchronize(m->stream), "loss synchronize")) return THOR_EHIP;
  double s = 0.0;
  for (float v : part) s += v;
  if (loss) *loss = s / ((double)B * m->w[m->nl]);
  return THOR_OK;
}

int thor_mlp_train_step(thor_mlp *m, const void *x_bf16, const float *t, int B, float lr) {
  clear_error();
  if (!m || !x_bf16 || !t) { set_error("thor_mlp_train_step: NULL argument"); return THOR_EINVAL; }
  if (B < 1 || B > m->max_batch || B % 32 || !(lr > 0)) { set_error("thor_mlp_train_step: batch must be a multiple of 32 within max_batch, lr > 0"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, true);
  backward(m, (const __bf16 *)x_bf16, t, B);
  m->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(nb(m->n_params)), dim3(256), 0, m->stream, m->p, m->g, m->m, m->v, m->n_params, lr,
                     b1, b2, 1e-8f, c1, c2);
  refresh_bf16(m);
  return mlp_ok(hipGetLastError(), "train step") ? THOR_OK : THOR_EHIP;
}

void thor_mlp_free(thor_mlp *m) { delete m; }

}  // extern "C"
