// Per-column corrector network on gfx950: multilayer perceptron with GELU
// hidden layers, BF16 operands and FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), forward, backward and Adam on the GPU.
//
// Layout: weights W[out][in] and activations [batch][width], row-major.  One
// GEMM kernel C[M][N] = sum_k A(m, k) B(n, k) reads either operand with k
// contiguous (A[m][k], B[n][k]) or with k as the outer index (A[k][m],
// B[k][n]) through LDS, so no transposed copies are kept:
//   forward    Z  = H_prev W^T     A = H_prev [B][in],   B = W [out][in]
//   input grad dH = dZ W           A = dZ [B][out],      B = W read as [k=out][n=in]
//   weight grad dW = dZ^T H_prev   A = dZ read as [k=B][m=out], B = H_prev read as [k=B][n=in]
// The weight gradient reduces over the batch in fixed chunks (split K) whose
// partial sums are added in a fixed order, so results are reproducible.
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

constexpr int kTile = 64;    // C tile per workgroup (4 wavefronts of 32 x 32)
constexpr int kStepK = 64;   // k per staged tile (two MFMA k-steps of 32)
constexpr int kRow = kStepK + 8;   // LDS row of a staged tile (bf16), padded
constexpr int kMaxSplit = 8;       // batch chunks of the weight gradient
constexpr int kBiasSplit = 32;     // batch chunks of the bias gradient

enum Epilogue { EPI_STORE = 0, EPI_GELU = 1, EPI_GELU_ONLY = 2 };

// erf by Abramowitz & Stegun 7.1.26: erf x = 1 - t (a1 + t (a2 + ... a5 t))
// e^(-x^2), t = 1 / (1 + p x) for x >= 0, odd in x; absolute error below
// 1.5e-7, far under the BF16 rounding of the activations it feeds, and
// branch-free (the epilogues evaluate it for every hidden activation).
__device__ __forceinline__ float erf_as(float x) {
  const float a = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.f + 0.3275911f * a);
  const float poly =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = 1.f - poly * __expf(-a * a);
  return copysignf(e, x);
}
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erf_as(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erf_as(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// Piece h (0, 1) of a 64 x 64 operand tile, 16 bytes per thread (256
// threads), read from global memory: rows r0.. of an operand with `rows`
// rows, k from k0, zero at k >= k_hi (k_hi a multiple of 32).  KOUTER:
// stored [k][row] with leading dimension ld, else [row][k].
template <bool KOUTER>
__device__ __forceinline__ bf16x8 tile_load(const __bf16 *P, int ld, int rows, int r0, int k0, int k_hi, int h) {
  const int t = threadIdx.x;
  const bf16x8 zero = {};
  if (!KOUTER) {
    const int row = r0 + (t >> 2), k = k0 + (t & 3) * 16 + 8 * h;
    return row < rows && k < k_hi ? *reinterpret_cast<const bf16x8 *>(P + (size_t)row * ld + k) : zero;
  } else {
    const int k = k0 + (t >> 3) + 32 * h, rc = r0 + (t & 7) * 8;   // rows is a multiple of 8
    return rc < rows && k < k_hi ? *reinterpret_cast<const bf16x8 *>(P + (size_t)k * ld + rc) : zero;
  }
}

// The same piece into the LDS tile S[row][k] (rows of kRow values).
template <bool KOUTER>
__device__ __forceinline__ void tile_store(__bf16 *S, const bf16x8 v, int h) {
  const int t = threadIdx.x;
  if (!KOUTER) {
    *reinterpret_cast<bf16x8 *>(S + (t >> 2) * kRow + (t & 3) * 16 + 8 * h) = v;
  } else {
    const int kr = (t >> 3) + 32 * h, rc = (t & 7) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[(rc + i) * kRow + kr] = v[i];
  }
}

// C tile (m0, n0) of the product over k in [k_lo, k_hi), 4 wavefronts, LDS
// double-buffered in tiles of 64 k.  Wavefront w owns rows 32 (w / 2) .. + 31 and columns
// 32 (w % 2) .. + 31 of the tile as 2 x 2 MFMA tiles of 16 x 16; lane l holds
// A(row l % 16, k0 + 8 (l / 16) .. + 7), B(col l % 16, same k) and
// accumulates D[4 (l / 16) + i][l % 16], i = 0..3.
//   EPI_STORE: C = acc (+ bias), or the split's partial C + z M ldc.
//   EPI_GELU:  C = acc + bias (pre-activation), H = gelu(C) in bf16.
//   EPI_GELU_ONLY: H only (inference keeps no pre-activation).
template <bool AK, bool BK, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const __bf16 *__restrict__ A, int lda, const __bf16 *__restrict__ B,
                                              int ldb, float *__restrict__ C, int ldc, const float *__restrict__ bias,
                                              __bf16 *__restrict__ H, int M, int N, int K, int k_chunk) {
  __shared__ __align__(16) __bf16 As[2][kTile * kRow];
  __shared__ __align__(16) __bf16 Bs[2][kTile * kRow];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;
  const int wm = 32 * (w >> 1), wn = 32 * (w & 1);
  const int r = lane & 15, kq = (lane >> 4) * 8;
  const int k_lo = blockIdx.z * k_chunk, k_hi = min(K, k_lo + k_chunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  if (k_lo < k_hi) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      tile_store<AK>(As[0], tile_load<AK>(A, lda, M, m0, k_lo, k_hi, h), h);
      tile_store<BK>(Bs[0], tile_load<BK>(B, ldb, N, n0, k_lo, k_hi, h), h);
    }
  }
  __syncthreads();
  for (int k0 = k_lo; k0 < k_hi; k0 += kStepK) {
    const bool more = k0 + kStepK < k_hi;
    bf16x8 na[2], nbv[2];
    if (more) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        na[h] = tile_load<AK>(A, lda, M, m0, k0 + kStepK, k_hi, h);
        nbv[h] = tile_load<BK>(B, ldb, N, n0, k0 + kStepK, k_hi, h);
      }
    }
#pragma unroll
    for (int kk = 0; kk < kStepK; kk += 32) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][(wm + 16 * i + r) * kRow + kk + kq]);
        b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][(wn + 16 * i + r) * kRow + kk + kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        tile_store<AK>(As[buf ^ 1], na[h], h);
        tile_store<BK>(Bs[buf ^ 1], nbv[h], h);
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  float *Cz = C + (size_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 16 * j + r;
      if (col >= N) continue;
      const float bb = bias ? bias[col] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wm + 16 * i + (lane >> 4) * 4 + q;
        if (row >= M) continue;
        const float z = acc[i][j][q] + bb;
        if (EPI != EPI_GELU_ONLY) Cz[(size_t)row * ldc + col] = z;
        if (EPI != EPI_STORE) H[(size_t)row * N + col] = (__bf16)gelu_f(z);
      }
    }
}

// ---------------------------------------------------------------------------
// Fused inference of a 4-layer network whose hidden widths are all kFH =
// 256 (the corrector's shape): one workgroup of kFW = 8 wavefronts (2 per
// SIMD) per tile of kFM = 48 rows runs every layer (214 workgroups for the
// g5 corrector's 10242 columns, one per CU, against 161 for 64-row tiles).
//   * The tile's inputs (48 rows x in, bf16) are staged once into LDS by
//     direct global-to-LDS loads (global_load_lds_dwordx4), all issued
//     before the first wait, laid out [k / 8][row slot][8] with 64 row slots
//     (one per lane of the loading wavefront), so that a wavefront's 16-byte
//     operand reads hit 64 distinct banks.
//   * The hidden activations then live in the same LDS ([row][k], rows
//     padded) from one layer to the next, so only the inputs, the weights
//     (from L2) and the outputs cross the memory hierarchy.
//   * The weights are read from a copy in MFMA fragment order
//     (k_weights_frag), one contiguous KiB per wavefront load.  Each layer
//     is its own loop over k in substeps of 32; a wavefront streams its
//     weight fragments through a ring of kFD substeps in registers, kFD - 1
//     substeps in flight while one is multiplied, with no barrier inside a
//     layer, and the next layer's first kFD substeps go in flight before the
//     current layer's epilogue.
// Wavefront w owns the 16-column tiles w + kFW j (j < kFT) of a layer
// below its width / 16, over the tile's rows (kFI MFMA tiles of 16 x 16
// each).  Per tile the products and their order (k ascending in steps of
// 32) equal k_gemm's, so the outputs equal the layer-by-layer path bit for
// bit.
// ---------------------------------------------------------------------------
#ifndef MLP_FI
#define MLP_FI 3
#endif
constexpr int kFI = MLP_FI;          // 16-row MFMA tiles per workgroup
constexpr int kFM = 16 * kFI;        // rows per workgroup
constexpr int kFR = 64;              // row slots per staged k block (one per lane of a wavefront)
constexpr int kFH = 256;             // hidden width
#ifndef MLP_FW
#define MLP_FW 8
#endif
constexpr int kFW = MLP_FW;          // wavefronts per workgroup
constexpr int kFT = kFH / 16 / kFW;  // 16-column tiles per wavefront (2)
constexpr int kFK0Max = 1152;        // widest input the LDS tile holds
#ifndef MLP_FD
#define MLP_FD 6
#endif
constexpr int kFD = MLP_FD;          // 32-k substeps in the weight ring
constexpr int kHRow = kFH + 8;       // LDS row of the hidden activations, padded
constexpr int kFLds = kFK0Max / 8 * kFR * 8;   // bf16 values of the LDS tile (147,456 bytes)
static_assert(kFM * kHRow <= kFLds, "hidden activations must fit the input tile's LDS");

struct FusedNet {
  const __bf16 *W[4];   // bf16 in MFMA fragment order (k_weights_frag)
  const float *b[4];
  int in, out;          // widths of the input and output layers
};

// A wavefront's weight stream of one layer: its fragment of tile j at
// substep 0 and the layer's number of 32-k substeps.
struct FusedW {
  const __bf16 *row[kFT];
  int nsub;
};

__device__ __forceinline__ FusedW fused_w(const __bf16 *W, int K, const int tile[kFT]) {
  FusedW fw;
  fw.nsub = K >> 5;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kFT; ++j) fw.row[j] = W + ((size_t)tile[j] * fw.nsub * 64 + lane) * 8;
  return fw;
}

// Substep t's fragments (a substep past the end reloads the last one).
__device__ __forceinline__ void fused_load(const FusedW &fw, int t, bf16x8 fr[kFT]) {
  const int tt = min(t, fw.nsub - 1);
#pragma unroll
  for (int j = 0; j < kFT; ++j) fr[j] = *reinterpret_cast<const bf16x8 *>(fw.row[j] + (size_t)tt * 512);
}

// acc[i][j] += A(rows 16 i + .., k) W(rows 16 tile[j] + .., k) over the
// layer's k, with ring[d] holding substep d on entry (the caller issues
// those loads early: before the input tile's wait, or before the previous
// layer's epilogue).  KC: the layer's k width if known at compile time,
// else 0.  XS: A is the staged input tile ([k / 8][row][8]), else the
// hidden activations ([row][kHRow]).  Tiles with use[j] false are loaded
// (from a valid row) but not multiplied.  The ring is refilled
// unconditionally, so every substep issues the same loads and the wait
// before a substep's products covers only its own fragments, kFD substeps
// old.
template <bool XS, int KC>
__device__ __forceinline__ void fused_layer(const FusedW &fw, const bool use[kFT], const __bf16 *lds,
                                            f32x4 acc[kFI][kFT], bf16x8 ring[kFD][kFT]) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = (lane >> 4) * 8;
  const int nsub = KC ? KC >> 5 : fw.nsub, nfull = nsub / kFD;
  auto mul = [&](int t, const bf16x8 fr[kFT]) {
    bf16x8 a[kFI];
#pragma unroll
    for (int i = 0; i < kFI; ++i)
      a[i] = XS ? *reinterpret_cast<const bf16x8 *>(lds + ((((32 * t + kq) >> 3) * kFR) + 16 * i + r) * 8)
                : *reinterpret_cast<const bf16x8 *>(lds + (16 * i + r) * kHRow + 32 * t + kq);
#pragma unroll
    for (int j = 0; j < kFT; ++j)
      if (use[j])
#pragma unroll
        for (int i = 0; i < kFI; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], fr[j], acc[i][j], 0, 0, 0);
  };
  for (int b = 0; b < nfull; ++b) {
#pragma unroll
    for (int d = 0; d < kFD; ++d) {
      const int t = b * kFD + d;
      mul(t, ring[d]);
      if (!KC || t + kFD < nsub) fused_load(fw, t + kFD, ring[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < kFD; ++d)
    if (nfull * kFD + d < nsub) mul(nfull * kFD + d, ring[d]);
}

// Tiles of wavefront w in layer l (out of n_tiles): w + kFW j.
__device__ __forceinline__ void fused_tiles(int w, int n_tiles, int tile[kFT], bool use[kFT]) {
#pragma unroll
  for (int j = 0; j < kFT; ++j) {
    use[j] = w + kFW * j < n_tiles;
    tile[j] = use[j] ? w + kFW * j : 0;
  }
}

__global__ __launch_bounds__(64 * kFW) void k_mlp_fused4(FusedNet net, const __bf16 *__restrict__ X, int B,
                                                         float *__restrict__ Y) {
  __shared__ __align__(16) __bf16 lds[kFLds];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15;
  const int m0 = blockIdx.x * kFM;
  const int K0 = net.in, N3 = net.out;
  // stage the input tile: wavefront w takes k blocks w, w + kFW, ...; lane =
  // row (lanes past the tile or the batch repeat its last row; their outputs
  // are dropped)
  {
    const __bf16 *xrow = X + (size_t)min(m0 + min(lane, kFM - 1), B - 1) * K0;
    for (int kb = w; kb < K0 / 8; kb += kFW)
      __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(xrow + 8 * kb),
                                       (__attribute__((address_space(3))) void *)(lds + kb * (kFR * 8)), 16, 0, 0);
  }
  int tile[kFT];
  bool use[kFT];
  fused_tiles(w, kFH / 16, tile, use);
  FusedW fw = fused_w(net.W[0], K0, tile);
  bf16x8 ring[kFD][kFT];
#pragma unroll
  for (int d = 0; d < kFD; ++d) fused_load(fw, d, ring[d]);
  __builtin_amdgcn_s_waitcnt(0);   // the direct-to-LDS loads (and the first weights) have landed
  __syncthreads();
  f32x4 acc[kFI][kFT];
  for (int l = 0; l < 4; ++l) {
#pragma unroll
    for (int i = 0; i < kFI; ++i)
#pragma unroll
      for (int j = 0; j < kFT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (l == 0)
      fused_layer<true, 0>(fw, use, lds, acc, ring);
    else
      fused_layer<false, kFH>(fw, use, lds, acc, ring);
    // the next layer's first weights go in flight before this epilogue
    int tile_n[kFT];
    bool use_n[kFT];
    FusedW fw_n = fw;
    if (l < 3) {
      fused_tiles(w, (l == 2 ? N3 : kFH) / 16, tile_n, use_n);
      fw_n = fused_w(net.W[l + 1], kFH, tile_n);
#pragma unroll
      for (int d = 0; d < kFD; ++d) fused_load(fw_n, d, ring[d]);
    }
    const float *bias = net.b[l];
    if (l < 3) __syncthreads();   // every wavefront is done reading this layer's input
#pragma unroll
    for (int j = 0; j < kFT; ++j) {
      if (!use[j]) continue;
      const int col = 16 * tile[j] + r;
      const float bb = bias[col];
#pragma unroll
      for (int i = 0; i < kFI; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * i + (lane >> 4) * 4 + q;
          const float z = acc[i][j][q] + bb;
          if (l < 3)
            lds[row * kHRow + col] = (__bf16)gelu_f(z);
          else if (m0 + row < B)
            Y[(size_t)(m0 + row) * N3 + col] = z;
        }
    }
    if (l < 3) {
      __syncthreads();   // the activations are the next layer's input
      fw = fw_n;
#pragma unroll
      for (int j = 0; j < kFT; ++j) {
        tile[j] = tile_n[j];
        use[j] = use_n[j];
      }
    }
  }
}

// out[i] = sum_{z < S} part[z][i] in order z = 0, 1, ...
__global__ void k_reduce(const float *part, int S, size_t n, float *out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
}

// Column sums of X[B][N] over row chunk blockIdx.y into part[chunk][N]:
// 64 columns per workgroup, 4 row groups combined in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float *X, int B, int N, int rows_per, float *part) {
  __shared__ float sm[4][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int b0 = blockIdx.y * rows_per, b1 = min(B, b0 + rows_per);
  float s = 0.f;
  if (n < N)
    for (int b = b0 + g; b < b1; b += 4) s += X[(size_t)b * N + n];
  sm[g][c] = s;
  __syncthreads();
  if (g == 0 && n < N) part[(size_t)blockIdx.y * N + n] = ((sm[0][c] + sm[1][c]) + sm[2][c]) + sm[3][c];
}

// Output layer: dZ = 2 (Y - T) / (B N); per-workgroup partial loss sums.
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *T, float *dZ, __bf16 *dZb,
                                              float *partial, int B, int N) {
  __shared__ float sm[256];
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < (size_t)B * N) {
    const float d = Y[i] - T[i];
    l = d * d;
    const float g = 2.f * d / ((float)B * (float)N);
    dZ[i] = g;
    dZb[i] = (__bf16)g;
  }
  sm[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// Hidden layer: dZ = dH * g'(Z) in fp32 and bf16.
__global__ void k_act_grad(const float *dH, const float *Z, float *dZ, __bf16 *dZb, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = dH[i] * gelu_grad_f(Z[i]);
  dZ[i] = g;
  dZb[i] = (__bf16)g;
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

// bf16 copy of one layer's fp32 weights.
__global__ void k_weights_bf16(const float *W, __bf16 *Wb, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Wb[i] = (__bf16)W[i];
}

// W[N][K] (FP32) into BF16 MFMA fragment order for the fused kernel:
// fragment (tile j, 32-k substep t, lane l) holds the 8 values
// W[16 j + l % 16][32 t + 8 (l / 16) .. + 7] at ((j K/32 + t) 64 + l) 8,
// so a wavefront's operand load for one tile and substep is 1 KiB
// contiguous.  N % 16 == 0, K % 32 == 0.
__global__ void k_weights_frag(const float *W, __bf16 *Wf, int N, int K) {
  const size_t f = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int nsub = K / 32;
  if (f >= (size_t)N * K / 8) return;
  const int lane = (int)(f % 64), t = (int)((f / 64) % nsub), j = (int)(f / 64 / nsub);
  const float *src = W + (size_t)(16 * j + lane % 16) * K + 32 * t + 8 * (lane / 16);
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (__bf16)src[e];
  *reinterpret_cast<bf16x8 *>(Wf + f * 8) = v;
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
  std::vector<__bf16 *> Wb;      // bf16 copies of W_l [out][in]
  std::vector<__bf16 *> Wf;      // the same in MFMA fragment order (fused inference)
  std::vector<float *> Z;        // pre-activations, [B][w_{l+1}]
  std::vector<__bf16 *> H;       // hidden activations, [B][w_{l+1}]
  std::vector<float *> dZ;
  std::vector<__bf16 *> dZb;
  float *dH = nullptr;           // [B][max width]
  float *split = nullptr;        // split-K partial sums of one weight gradient
  float *partial = nullptr;      // loss partial sums
  int adam_t = 0;
  bool fused = true;             // inference through k_mlp_fused4 where the shape allows
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
  size_t wprod = 0;
  for (int x : M->w) wmax = std::max(wmax, x);
  for (int l = 0; l < nl; ++l) wprod = std::max(wprod, (size_t)M->w[l] * M->w[l + 1]);
  M->p = (float *)take(M->n_params * 4);
  M->g = (float *)take(M->n_params * 4);
  M->m = (float *)take(M->n_params * 4);
  M->v = (float *)take(M->n_params * 4);
  M->Wb.assign(nl, nullptr);
  M->Wf.assign(nl, nullptr);
  M->Z.assign(nl, nullptr);
  M->H.assign(nl, nullptr);
  M->dZ.assign(nl, nullptr);
  M->dZb.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    const size_t wsz = (size_t)M->w[l] * M->w[l + 1];
    M->Wb[l] = (__bf16 *)take(wsz * 2);
    M->Wf[l] = (__bf16 *)take(wsz * 2);
    M->Z[l] = (float *)take((size_t)B * M->w[l + 1] * 4);
    M->H[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
    M->dZ[l] = (float *)take((size_t)B * M->w[l + 1] * 4);
    M->dZb[l] = (__bf16 *)take((size_t)B * M->w[l + 1] * 2);
  }
  M->dH = (float *)take((size_t)B * wmax * 4);
  M->split = (float *)take(std::max((size_t)kMaxSplit * wprod, (size_t)kBiasSplit * wmax) * 4);
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
    hipLaunchKernelGGL(k_weights_bf16, dim3(nb(n)), dim3(256), 0, M->stream, M->p + M->woff[l], M->Wb[l], n);
    hipLaunchKernelGGL(k_weights_frag, dim3(nb(n / 8)), dim3(256), 0, M->stream, M->p + M->woff[l], M->Wf[l],
                       M->w[l + 1], M->w[l]);
  }
}

// C[M][N] = sum_k A(m, k) B(n, k); see k_gemm for the operand forms.
template <bool AK, bool BK, int EPI>
void gemm(const __bf16 *A, int lda, const __bf16 *B, int ldb, float *C, int ldc, const float *bias, __bf16 *H,
          int Mr, int N, int K, int splits, hipStream_t s) {
  const int chunk = ((K + splits - 1) / splits + kStepK - 1) / kStepK * kStepK;
  const int S = (K + chunk - 1) / chunk;
  dim3 grid((Mr + kTile - 1) / kTile, (N + kTile - 1) / kTile, S);
  hipLaunchKernelGGL((k_gemm<AK, BK, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, bias, H, Mr, N, K, chunk);
}

// Number of batch chunks of a weight gradient: chunks of at least 256 rows.
int grad_splits(int B) { return std::max(1, std::min(kMaxSplit, B / 256)); }

// The fused inference kernel serves 4-layer networks with hidden widths
// kFH, an input width of at most kFK0Max and an output width of at most kFH.
bool fused_shape(const thor_mlp *M) {
  return M->nl == 4 && M->w[0] <= kFK0Max && M->w[1] == kFH && M->w[2] == kFH && M->w[3] == kFH &&
         M->w[4] <= kFH;
}

// Forward pass; the output layer's pre-activation goes to y if given
// (inference: hidden pre-activations are not kept), else to Z[nl - 1].
void forward(thor_mlp *M, const __bf16 *X, int B, float *y) {
  if (y && fused_shape(M) && M->fused) {
    FusedNet net;
    for (int l = 0; l < 4; ++l) {
      net.W[l] = M->Wf[l];
      net.b[l] = M->p + M->boff[l];
    }
    net.in = M->w[0];
    net.out = M->w[4];
    hipLaunchKernelGGL(k_mlp_fused4, dim3((B + kFM - 1) / kFM), dim3(64 * kFW), 0, M->stream, net, X, B, y);
    return;
  }
  const __bf16 *in = X;
  for (int l = 0; l < M->nl; ++l) {
    const int K = M->w[l], N = M->w[l + 1];
    const float *bias = M->p + M->boff[l];
    if (l + 1 < M->nl) {
      if (y)
        gemm<false, false, EPI_GELU_ONLY>(in, K, M->Wb[l], K, M->Z[l], N, bias, M->H[l], B, N, K, 1, M->stream);
      else
        gemm<false, false, EPI_GELU>(in, K, M->Wb[l], K, M->Z[l], N, bias, M->H[l], B, N, K, 1, M->stream);
      in = M->H[l];
    } else {
      gemm<false, false, EPI_STORE>(in, K, M->Wb[l], K, y ? y : M->Z[l], N, bias, nullptr, B, N, K, 1, M->stream);
    }
  }
}

// Gradients of the mean-squared loss into M->g; partial loss sums in M->partial.
void backward(thor_mlp *M, const __bf16 *X, const float *T, int B) {
  const int nl = M->nl;
  hipStream_t s = M->stream;
  const int No = M->w[nl];
  hipLaunchKernelGGL(k_loss, dim3(nb((size_t)B * No)), dim3(256), 0, s, M->Z[nl - 1], T, M->dZ[nl - 1],
                     M->dZb[nl - 1], M->partial, B, No);
  const int S = grad_splits(B);
  for (int l = nl - 1; l >= 0; --l) {
    const int K = M->w[l], N = M->w[l + 1];
    const __bf16 *prev = l == 0 ? X : M->H[l - 1];
    // dW[N][K] = dZ^T H_prev: both operands read with the batch as outer index
    gemm<true, true, EPI_STORE>(M->dZb[l], N, prev, K, M->split, K, nullptr, nullptr, N, K, B, S, s);
    const size_t nw = (size_t)N * K;
    hipLaunchKernelGGL(k_reduce, dim3(nb(nw)), dim3(256), 0, s, M->split, S, nw, M->g + M->woff[l]);
    // db[N] = column sums of dZ
    const int rows = (B + kBiasSplit - 1) / kBiasSplit;
    hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64, kBiasSplit), dim3(256), 0, s, M->dZ[l], B, N, rows, M->split);
    hipLaunchKernelGGL(k_reduce, dim3(nb(N)), dim3(256), 0, s, M->split, kBiasSplit, (size_t)N, M->g + M->boff[l]);
    if (l > 0) {
      // dH[B][K] = dZ W, W read as [k = out][n = in]; then through the activation
      gemm<false, true, EPI_STORE>(M->dZb[l], N, M->Wb[l], K, M->dH, K, nullptr, nullptr, B, K, N, 1, s);
      const size_t n = (size_t)B * K;
      hipLaunchKernelGGL(k_act_grad, dim3(nb(n)), dim3(256), 0, s, M->dH, M->Z[l - 1], M->dZ[l - 1], M->dZb[l - 1], n);
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

namespace thor {
void mlp_shape_of(const thor_mlp *m, int *in, int *out, int *max_batch) {
  *in = m->w.front();
  *out = m->w.back();
  *max_batch = m->max_batch;
}
}  // namespace thor

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
  if (((uintptr_t)x_bf16 & 15) != 0) { set_error("thor_mlp_forward: inputs must be 16-byte aligned"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, y);
  return mlp_ok(hipGetLastError(), "mlp forward") ? THOR_OK : THOR_EHIP;
}

int thor_mlp_loss_grad(thor_mlp *m, const void *x_bf16, const float *t, int B, double *loss, float *grad_host) {
  clear_error();
  if (!m || !x_bf16 || !t) { set_error("thor_mlp_loss_grad: NULL argument"); return THOR_EINVAL; }
  if (B < 1 || B > m->max_batch || B % 32) { set_error("thor_mlp_loss_grad: batch must be a multiple of 32 within max_batch"); return THOR_EINVAL; }
  if (((uintptr_t)x_bf16 & 15) != 0) { set_error("thor_mlp_loss_grad: inputs must be 16-byte aligned"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, nullptr);
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
  if (((uintptr_t)x_bf16 & 15) != 0) { set_error("thor_mlp_train_step: inputs must be 16-byte aligned"); return THOR_EINVAL; }
  forward(m, (const __bf16 *)x_bf16, B, nullptr);
  backward(m, (const __bf16 *)x_bf16, t, B);
  m->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(nb(m->n_params)), dim3(256), 0, m->stream, m->p, m->g, m->m, m->v, m->n_params, lr,
                     b1, b2, 1e-8f, c1, c2);
  refresh_bf16(m);
  return mlp_ok(hipGetLastError(), "train step") ? THOR_OK : THOR_EHIP;
}

int thor_mlp_set_fused(thor_mlp *m, int on) {
  clear_error();
  if (!m) { set_error("thor_mlp_set_fused: NULL network"); return THOR_EINVAL; }
  m->fused = on != 0;
  return THOR_OK;
}

void thor_mlp_free(thor_mlp *m) { delete m; }

}  // extern "C"
