// Surrogate initialiser network: hand-written training and inference kernels.
//
// A small CNN maps a source's 5-band 32x32 patch to its 27 parameters (in
// standardised unconstrained coordinates) so that the trust-region fit starts
// closer to the optimum; the plain start remains the fallback.  Layers: four
// 3x3 same convolutions (5->32->64->64->128, ReLU, 2x2 max-pool after the last
// three) and dense 2048->256 (ReLU) -> 27.  Every matrix product (convolution
// forward, data gradient and weight gradient as implicit GEMMs, dense layers)
// runs on one gather-GEMM kernel on the BF16 matrix cores (16x16x32 MFMA, FP32
// accumulation, split-K partials summed in a fixed order; the convolution forward's bias,
// ReLU and BF16 store fused into the product where it needs no split).  Activations and
// gradients feeding a product are BF16; master weights, Adam moments, biases and
// all reductions are FP32.
#include <math.h>

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <new>
#include <string>

#include "celeste_internal.h"

namespace celeste {

typedef __bf16 bf16;

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;

__device__ __forceinline__ bf16 to_bf16(float x) { return (bf16)x; }
__device__ __forceinline__ float from_bf16(bf16 x) { return (float)x; }

constexpr int TM = 64, TK = 32, TKP = TK + 8;

// ------------------------------------------------------------------ gather loaders
// A loader gives 8 consecutive k of A(m, k) (a8), zero for k >= kend or an index out of range.
// For B(k, n) it gives either 8 consecutive k at one n (b8; kRunN false) or, for the
// convolution operands built from images, 8 consecutive n at one k (b8n; kRunN true): n is a
// multiple of 8 and the images are square with a power-of-two width of at least 8, so the 8
// pixels lie in one image row and the tap and channel decomposition is done once per run.

// kk -> (ky, kx) of a 3x3 kernel tap
__device__ __forceinline__ int tap_y(int kk) { return (kk * 11) >> 5; }   // kk / 3 for kk < 9
__device__ __forceinline__ int tap_x(int kk) { return kk - 3 * tap_y(kk); }

__device__ __forceinline__ bf16x8_t zero8() {
  bf16x8_t z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = (bf16)0.f;
  return z;
}

// 8 contiguous BF16 values at p: one 16-byte load where p is aligned and all 8 are wanted, else
// element by element (the first n_valid).
__device__ __forceinline__ bf16x8_t load8(const bf16* p, int n_valid, bool aligned) {
  if (n_valid >= 8 && aligned && ((uintptr_t)p & 15) == 0) return *reinterpret_cast<const bf16x8_t*>(p);
  bf16x8_t v = zero8();
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < n_valid) v[j] = p[j];
  return v;
}

// The 8 pixels px + sh .. px + sh + 7 of one image row (zero outside 0 .. wd-1), px a multiple of 8,
// sh in {-1, 0, 1}, row 16-byte aligned: the aligned 16 bytes at px and, for sh = -1 (+1), the 16 bytes
// before (after) them, shifted by one element with funnel shifts; a neighbour chunk outside the row
// reads as zeros.
__device__ __forceinline__ bf16x8_t row8(const bf16* __restrict__ row, int px, int sh, int wd) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;
  const u32x4_t zero = {0u, 0u, 0u, 0u};
  const u32x4_t mid = *reinterpret_cast<const u32x4_t*>(row + px);
  const u32x4_t lo = (sh < 0 && px > 0) ? *reinterpret_cast<const u32x4_t*>(row + px - 8) : zero;
  const u32x4_t hi = (sh > 0 && px + 8 < wd) ? *reinterpret_cast<const u32x4_t*>(row + px + 8) : zero;
  // window w = {lo.w, mid.x, mid.y, mid.z, mid.w, hi.x}; output dword i = (w[i+1+up] : w[i+up]) >> bits
  const unsigned w[6] = {lo.w, mid.x, mid.y, mid.z, mid.w, hi.x};
  const unsigned bits = sh == 0 ? 0u : 16u;
  const int up = sh < 0 ? 0 : 1;
  u32x4_t o;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned a = up ? w[i + 2] : w[i + 1], b = up ? w[i + 1] : w[i];
    o[i] = __builtin_amdgcn_alignbit(a, b, bits);
  }
  return __builtin_bit_cast(bf16x8_t, o);
}

// row8 for a shift sh that is the same on every lane: one scalar branch instead of per-lane selects
// (the same 8 values as row8).
__device__ __forceinline__ bf16x8_t row8u(const bf16* __restrict__ row, int px, int sh, int wd) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;
  const u32x4_t zero = {0u, 0u, 0u, 0u};
  const u32x4_t mid = *reinterpret_cast<const u32x4_t*>(row + px);
  if (sh == 0) return __builtin_bit_cast(bf16x8_t, mid);
  u32x4_t o;
  if (sh < 0) {
    const u32x4_t lo = px > 0 ? *reinterpret_cast<const u32x4_t*>(row + px - 8) : zero;
    o[0] = __builtin_amdgcn_alignbit(mid.x, lo.w, 16u);
    o[1] = __builtin_amdgcn_alignbit(mid.y, mid.x, 16u);
    o[2] = __builtin_amdgcn_alignbit(mid.z, mid.y, 16u);
    o[3] = __builtin_amdgcn_alignbit(mid.w, mid.z, 16u);
  } else {
    const u32x4_t hi = px + 8 < wd ? *reinterpret_cast<const u32x4_t*>(row + px + 8) : zero;
    o[0] = __builtin_amdgcn_alignbit(mid.y, mid.x, 16u);
    o[1] = __builtin_amdgcn_alignbit(mid.z, mid.y, 16u);
    o[2] = __builtin_amdgcn_alignbit(mid.w, mid.z, 16u);
    o[3] = __builtin_amdgcn_alignbit(hi.x, mid.w, 16u);
  }
  return __builtin_bit_cast(bf16x8_t, o);
}

// Per-thread state of an n-run of a convolution operand: the run's image plane 0 and its first
// pixel (row py, column px, a multiple of 8); fixed over the K loop.
struct RunState {
  const bf16* plane0;
  int py, px;
};

struct LdConvFwd {        // Y[co][img*HW+p] = sum_{ci,kk} W[co][ci*9+kk] X[img][ci][p + off(kk)]
  static constexpr bool kRunN = true;
  const bf16* W;
  const bf16* X;
  int Cin, hwl, wl;       // image side 2^wl, HW = 2^hwl
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    const size_t o = (size_t)m * Cin * 9 + k;
    return load8(W + o, kend - k, (o & 7) == 0);
  }
  __device__ RunState run(int n) const {
    const int img = n >> hwl, p = n & ((1 << hwl) - 1);
    return RunState{X + (((size_t)img * Cin) << hwl), p >> wl, p & ((1 << wl) - 1)};
  }
  __device__ bf16x8_t b8n(int k0, int kb, const RunState& r) const {
    const int k = k0 + kb;
    const int ci = k / 9, kk = k - ci * 9;
    const int y = r.py + tap_y(kk) - 1;
    if (y < 0 || y >= (1 << wl)) return zero8();
    return row8(r.plane0 + ((size_t)ci << hwl) + ((size_t)y << wl), r.px, tap_x(kk) - 1, 1 << wl);
  }
};

// The same product with K ordered tap-major, k = kk*Cin + ci, for Cin a power of two of at least
// 32: a 32-deep K step (K splits start at multiples of 32) then lies within one tap, so the tap's
// row and column shift are the same on every lane.  W is the layer's weights re-laid as
// W[co][kk*Cin + ci] (k_wf).
struct LdConvFwdT {
  static constexpr bool kRunN = true;
  const bf16* W;
  const bf16* X;
  int Cin, cl, hwl, wl;   // Cin = 2^cl
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    const size_t o = (size_t)m * Cin * 9 + k;
    return load8(W + o, kend - k, (o & 7) == 0);
  }
  __device__ RunState run(int n) const {
    const int img = n >> hwl, p = n & ((1 << hwl) - 1);
    return RunState{X + (((size_t)img * Cin) << hwl), p >> wl, p & ((1 << wl) - 1)};
  }
  __device__ bf16x8_t b8n(int k0, int kb, const RunState& r) const {
    const int kk = k0 >> cl, ci = (k0 & (Cin - 1)) + kb;
    const int y = r.py + tap_y(kk) - 1;
    if (y < 0 || y >= (1 << wl)) return zero8();
    return row8u(r.plane0 + ((size_t)ci << hwl) + ((size_t)y << wl), r.px, tap_x(kk) - 1, 1 << wl);
  }
};

struct LdConvDgrad {      // dX[ci][img*HW+p] = sum_{co,kk} W[co][ci][kk] dY[img][co][p - off(kk)]
  static constexpr bool kRunN = true;
  const bf16* Wt;         // the layer's weights as Wt[ci][kk*Cout+co] (k_wt)
  const bf16* dY;
  int Cin, Cout, col, hwl, wl;   // K ordered tap-major, k = kk*Cout + co, Cout = 2^col >= 32 (as LdConvFwdT)
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    const size_t o = (size_t)m * Cout * 9 + k;
    return load8(Wt + o, kend - k, (o & 7) == 0);
  }
  __device__ RunState run(int n) const {
    const int img = n >> hwl, p = n & ((1 << hwl) - 1);
    return RunState{dY + (((size_t)img * Cout) << hwl), p >> wl, p & ((1 << wl) - 1)};
  }
  __device__ bf16x8_t b8n(int k0, int kb, const RunState& r) const {
    const int kk = k0 >> col, co = (k0 & (Cout - 1)) + kb;
    const int y = r.py - tap_y(kk) + 1;
    if (y < 0 || y >= (1 << wl)) return zero8();
    return row8u(r.plane0 + ((size_t)co << hwl) + ((size_t)y << wl), r.px, 1 - tap_x(kk), 1 << wl);
  }
};

struct LdConvWgrad {      // dW[co][ci*9+kk] = sum_{img,p} dY[img][co][p] X[img][ci][p + off(kk)]
  static constexpr bool kRunN = false;
  const bf16* dY;
  const bf16* X;
  int Cin, Cout, hwl, wl;   // image side 2^wl, HW = 2^hwl
  // k = img*HW + p; HW, the K splits and the run's first k are multiples of 8, so a run is whole
  // and stays in one image row (the image side is a power of two of at least 8)
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    const int img = k >> hwl, p = k & ((1 << hwl) - 1);
    return load8(dY + ((((size_t)img * Cout + m) << hwl) + p), kend - k, true);
  }
  __device__ bf16x8_t b8(int k, int n, int) const {
    const int img = k >> hwl, p = k & ((1 << hwl) - 1), py = p >> wl, px = p & ((1 << wl) - 1);
    const int ci = n / 9, kk = n - ci * 9;
    const int y = py + tap_y(kk) - 1;
    if (y < 0 || y >= (1 << wl)) return zero8();
    return row8(X + ((((size_t)img * Cin + ci) << hwl) + ((size_t)y << wl)), px, tap_x(kk) - 1, 1 << wl);
  }
};

struct LdFcFwd {          // Y[o][b] = sum_i W[o][i] X[b][i]
  static constexpr bool kRunN = false;
  const bf16* W;
  const bf16* X;
  int In;
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    return load8(W + (size_t)m * In + k, kend - k, (In & 7) == 0);
  }
  __device__ bf16x8_t b8(int k, int n, int kend) const {
    return load8(X + (size_t)n * In + k, kend - k, (In & 7) == 0);
  }
};

struct LdFcDgrad {        // dX[i][b] = sum_o W[o][i] dY[b][o]
  static constexpr bool kRunN = false;
  const bf16* W;
  const bf16* dY;
  int In, Out;
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    bf16x8_t v = zero8();
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k + j < kend) v[j] = W[(size_t)(k + j) * In + m];
    return v;
  }
  __device__ bf16x8_t b8(int k, int n, int kend) const {
    return load8(dY + (size_t)n * Out + k, kend - k, ((size_t)n * Out + k) % 8 == 0);
  }
};

struct LdFcWgrad {        // dW[o][i] = sum_b dY[b][o] X[b][i]
  static constexpr bool kRunN = false;
  const bf16* dY;
  const bf16* X;
  int In, Out;
  __device__ bf16x8_t a8(int m, int k, int kend) const {
    bf16x8_t v = zero8();
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k + j < kend) v[j] = dY[(size_t)(k + j) * Out + m];
    return v;
  }
  __device__ bf16x8_t b8(int k, int n, int kend) const {
    bf16x8_t v = zero8();
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k + j < kend) v[j] = X[(size_t)(k + j) * In + n];
    return v;
  }
};

// Optional fused epilogue of a product with one K split: the convolution forward's
// act[img][co][p] = bf16(relu(C[co][img*HW+p] + bias[co])) instead of storing C.
struct EpConvFwd {
  const float* bias;
  bf16* act;
  int hwl;                // HW = 2^hwl pixels per image
};

// Tile width in N: 128 for the convolution operands built from images (n-runs), 64 otherwise
// (the dense layers and the weight gradients, whose N is small).
template <class LD>
constexpr int tile_n() { return LD::kRunN ? 128 : 64; }

// C[z][m][n] = sum over the z-th K split of A(m,k) B(k,n).  Block 256 = 4 waves in a 2x2
// arrangement over a 64 x TNB tile, each wave a 32 x TNB/2 sub-tile of 2 x TNB/32 MFMA
// 16x16x32 tiles.  Operand runs of 8 BF16 go to LDS (k-runs as 16-byte stores, n-runs
// transposed element by element) and come back as single 16-byte reads; the next K step's
// operands are loaded into registers while the current step's products run.  With ep.act set
// (and one split) the convolution forward epilogue is applied in place of the C store.
template <class LD>
__global__ __launch_bounds__(256) void k_gemm(LD ld, int M, int N, int K, int kchunk, float* __restrict__ C,
                                              EpConvFwd ep) {
  constexpr int TNB = tile_n<LD>(), NJ = TNB / 32, NR = TNB / 64;
  __shared__ __align__(16) bf16 As[TM][TKP];
  __shared__ __align__(16) bf16 Bs[TNB][TKP];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TNB;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * (TNB / 2);
  f32x4_t acc[2][NJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // A: row t / 4, k-run (t % 4) * 8.  B k-runs: rows t / 4 (+ 64), k-run (t % 4) * 8.  B n-runs
  // (TNB = 128): k = t % 32, columns 8 (t / 32) .. + 7 and the same + 64 (the 32 lanes of one
  // n-run write 32 consecutive k of a row of Bs, so the transposed stores spread over the banks).
  const int ar = t >> 2, ak = (t & 3) * 8;
  const int nb = 8 * (t >> 5), kb = t & 31;
  bf16x8_t an, bn[NR];
  // n-run states (fixed over the K loop; unused for k-run operands)
  RunState rs[NR];
  bool rv[NR];
  if constexpr (LD::kRunN) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int n = n0 + nb + 64 * r;
      rv[r] = n < N;
      rs[r] = ld.run(rv[r] ? n : 0);
    }
  }
  auto fetch = [&](int k0) {
    {
      const int m = m0 + ar, k = k0 + ak;
      an = (m < M && k < kend) ? ld.a8(m, k, kend) : zero8();
    }
    if constexpr (LD::kRunN) {
      const int k = k0 + kb;
#pragma unroll
      for (int r = 0; r < NR; ++r) bn[r] = (rv[r] && k < kend) ? ld.b8n(k0, kb, rs[r]) : zero8();
    } else {
      const int k = k0 + ak;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int n = n0 + ar + 64 * r;
        bn[r] = (n < N && k < kend) ? ld.b8(k, n, kend) : zero8();
      }
    }
  };
  bf16x8_t a[2], b[NJ];
  fetch(kbeg);
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    *reinterpret_cast<bf16x8_t*>(&As[ar][ak]) = an;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if constexpr (LD::kRunN) {
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[nb + 64 * r + j][kb] = bn[r][j];
      } else {
        *reinterpret_cast<bf16x8_t*>(&Bs[ar + 64 * r][ak]) = bn[r];
      }
    }
    __syncthreads();
    if (k0 + TK < kend) fetch(k0 + TK);   // next step's operands, in flight during the products
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8_t*>(&As[wm + i * 16 + r16][kq]);
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn + j * 16 + r16][kq]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  float* Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mm = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int nn = n0 + wn + j * 16 + (lane & 15);
        if (mm < M && nn < N) {
          if (ep.act) {
            const int img = nn >> ep.hwl, p = nn & ((1 << ep.hwl) - 1);
            ep.act[((((size_t)img * M + mm) << ep.hwl) + p)] = to_bf16(fmaxf(acc[i][j][r] + ep.bias[mm], 0.f));
          } else {
            Cz[(size_t)mm * N + nn] = acc[i][j][r];
          }
        }
      }
}

// Sum over the K splits in split order; 8 loads in flight at a time.
__device__ __forceinline__ float split_sum(const float* C, int S, size_t MN, size_t idx) {
  float s = C[idx];
  int z = 1;
  for (; z + 8 <= S; z += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = C[(size_t)(z + j) * MN + idx];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; z < S; ++z) s += C[(size_t)z * MN + idx];
  return s;
}

// ------------------------------------------------------------------ epilogues and elementwise

// conv forward: act[img][co][p] = bf16(relu(C[co][img*HW+p] + bias[co]))
__global__ void k_ep_conv_fwd(const float* __restrict__ C, int S, int Cout, int B, int HW,
                              const float* __restrict__ bias, bf16* __restrict__ act) {
  const size_t total = (size_t)B * Cout * HW;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int p = i % HW;
    const int co = (i / HW) % Cout;
    const int img = i / ((size_t)HW * Cout);
    const float v = split_sum(C, S, (size_t)Cout * B * HW, (size_t)co * B * HW + (size_t)img * HW + p) + bias[co];
    act[i] = to_bf16(fmaxf(v, 0.f));
  }
}

// dense forward: out[b][o] = C[o][b] + bias[o], ReLU + BF16 (hidden) or FP32 (output)
__global__ void k_ep_fc_fwd(const float* __restrict__ C, int S, int Out, int B, const float* __restrict__ bias,
                            bf16* __restrict__ act, float* __restrict__ outf) {
  const int total = Out * B;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int o = i % Out, b = i / Out;
    const float v = split_sum(C, S, (size_t)Out * B, (size_t)o * B + b) + bias[o];
    if (act) act[i] = to_bf16(fmaxf(v, 0.f));
    if (outf) outf[i] = v;
  }
}

// weight gradient: dW[m][n] = sum_z C[z][m][n]
__global__ void k_ep_sum(const float* __restrict__ C, int S, int MN, float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MN; i += gridDim.x * blockDim.x)
    out[i] = split_sum(C, S, MN, i);
}

// 2x2 max-pool (BF16)
__global__ void k_pool_fwd(const bf16* __restrict__ in, int BC, int H, int W, bf16* __restrict__ out) {
  const int Ho = H / 2, Wo = W / 2;
  const size_t total = (size_t)BC * Ho * Wo;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int x = i % Wo, y = (i / Wo) % Ho;
    const size_t bc = i / ((size_t)Ho * Wo);
    const bf16* q = in + bc * H * W + (2 * y) * W + 2 * x;
    const float v = fmaxf(fmaxf(from_bf16(q[0]), from_bf16(q[1])), fmaxf(from_bf16(q[W]), from_bf16(q[W + 1])));
    out[i] = to_bf16(v);
  }
}

// Backward through (optional) 2x2 max-pool and ReLU.  g comes from a GEMM as C[c*Hg*Wg + q][img]
// (dense) or C[c][img*Hg*Wg + q] (convolution), summed over splits; r is the post-ReLU
// activation at full resolution (H x W).  The pooled gradient goes to the first maximal
// input of its window (row-major), then is masked by r > 0.
__global__ void k_pool_relu_bwd(const float* __restrict__ C, int S, int dense_layout, int B, int Cch, int H, int W,
                                int pooled, const bf16* __restrict__ r, float* __restrict__ dz,
                                bf16* __restrict__ dzb) {
  const int Hg = pooled ? H / 2 : H, Wg = pooled ? W / 2 : W;
  const size_t MN = (size_t)Cch * Hg * Wg * B;
  const size_t total = (size_t)B * Cch * H * W;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int x = i % W, y = (i / W) % H;
    const int c = (i / ((size_t)W * H)) % Cch;
    const int img = i / ((size_t)W * H * Cch);
    const bf16* rr = r + ((size_t)img * Cch + c) * H * W;
    const float rv = from_bf16(rr[y * W + x]);
    float g = 0.f;
    if (rv > 0.f) {
      int gy = y, gx = x;
      bool take = true;
      if (pooled) {
        gy = y / 2;
        gx = x / 2;
        const int y0 = 2 * gy, x0 = 2 * gx;
        const float a0 = from_bf16(rr[y0 * W + x0]), a1 = from_bf16(rr[y0 * W + x0 + 1]);
        const float a2 = from_bf16(rr[(y0 + 1) * W + x0]), a3 = from_bf16(rr[(y0 + 1) * W + x0 + 1]);
        const float mx = fmaxf(fmaxf(a0, a1), fmaxf(a2, a3));
        const int first = (a0 == mx) ? 0 : (a1 == mx) ? 1 : (a2 == mx) ? 2 : 3;
        take = first == (y - y0) * 2 + (x - x0);
      }
      if (take) {
        const int q = gy * Wg + gx;
        const size_t idx = dense_layout ? ((size_t)(c * Hg * Wg + q) * B + img)
                                        : ((size_t)c * B * Hg * Wg + (size_t)img * Hg * Wg + q);
        g = split_sum(C, S, MN, idx);
      }
    }
    dz[i] = g;
    dzb[i] = to_bf16(g);
  }
}

// dense hidden-layer backward: dz[b][i] = C[i][b] * (h[b][i] > 0)
__global__ void k_relu_bwd_fc(const float* __restrict__ C, int S, int In, int B, const bf16* __restrict__ h,
                              float* __restrict__ dz, bf16* __restrict__ dzb) {
  const int total = In * B;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int f = i % In, b = i / In;
    const float g = from_bf16(h[i]) > 0.f ? split_sum(C, S, (size_t)In * B, (size_t)f * B + b) : 0.f;
    dz[i] = g;
    dzb[i] = to_bf16(g);
  }
}

// bias gradient: db[c] = sum over images and positions of dz[img][c][p] (one block per channel)
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ dz, int B, int Cch, int HW,
                                                   float* __restrict__ db) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < B * HW; i += 256) {
    const int img = i / HW, p = i - img * HW;
    s += dz[((size_t)img * Cch + c) * HW + p];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = sh[0];
}

// Conv-layer bias gradient in two fixed-order passes: block (c, q) sums the q-th of BP_PARTS
// slices of channel c over images and positions; then one thread per channel sums its slices.
constexpr int BP_PARTS = 64;

__global__ __launch_bounds__(256) void k_bias_part(const float* __restrict__ dz, int B, int Cch, int HW,
                                                   float* __restrict__ part) {
  __shared__ float sh[256];
  const int c = blockIdx.x, q = blockIdx.y;
  const int n = B * HW, per = (n + BP_PARTS - 1) / BP_PARTS;
  const int i0 = q * per, i1 = min(n, i0 + per);
  float s = 0.f;
  for (int i = i0 + threadIdx.x; i < i1; i += 256) {
    const int img = i / HW, p = i - img * HW;
    s += dz[((size_t)img * Cch + c) * HW + p];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c * BP_PARTS + q] = sh[0];
}

__global__ __launch_bounds__(128) void k_bias_fin(const float* __restrict__ part, int Cch, float* __restrict__ db) {
  const int c = blockIdx.x * 128 + threadIdx.x;
  if (c >= Cch) return;
  float s = 0.f;
  for (int q = 0; q < BP_PARTS; ++q) s += part[c * BP_PARTS + q];
  db[c] = s;
}

// MSE loss over the batch: dy = 2 (y - t) / (B*27); loss written by one block
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t, int n,
                                             float* __restrict__ dy, bf16* __restrict__ dyb,
                                             float* __restrict__ loss) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float d = y[i] - t[i];
    s += d * d;
    const float g = 2.f * d / (float)n;
    dy[i] = g;
    dyb[i] = to_bf16(g);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] / (float)n;
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, bf16* __restrict__ wb, int n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = to_bf16(wi);
  }
}

// One convolution layer's weights re-laid for the data-gradient product, tap-major:
// Wt[ci][kk*Cout+co] = W[co][ci*9+kk].
__global__ void k_wt(const bf16* __restrict__ W, int Cin, int Cout, bf16* __restrict__ Wt) {
  const int n = Cin * Cout * 9;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int ci = i / (Cout * 9), r = i - ci * Cout * 9, kk = r / Cout, co = r - kk * Cout;
    Wt[i] = W[((size_t)co * Cin + ci) * 9 + kk];
  }
}

// One convolution layer's weights re-laid for the tap-major forward product:
// Wf[co][kk*Cin+ci] = W[co][ci*9+kk].
__global__ void k_wf(const bf16* __restrict__ W, int Cin, int Cout, bf16* __restrict__ Wf) {
  const int n = Cin * Cout * 9;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int co = i / (Cin * 9), r = i - co * Cin * 9, kk = r / Cin, ci = r - kk * Cin;
    Wf[i] = W[((size_t)co * Cin + ci) * 9 + kk];
  }
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16* __restrict__ wb, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) wb[i] = to_bf16(w[i]);
}

__global__ void k_acc_loss(const float* __restrict__ loss, float* __restrict__ acc) { *acc += *loss; }

// network output (standardised) -> unconstrained coordinates: psi = mean + std * y
__global__ void k_destandardise(const float* __restrict__ y, const float* __restrict__ mean,
                                const float* __restrict__ sd, int n, float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int j = i % 27;
    out[i] = mean[j] + sd[j] * y[i];
  }
}

// minibatch gather: xb[i] = x[order[i]], tb[i] = t[order[i]]
__global__ void k_gather(const bf16* __restrict__ x, const float* __restrict__ t, const int* __restrict__ order,
                         int B, int xsz, int tsz, bf16* __restrict__ xb, float* __restrict__ tb) {
  const int i = blockIdx.x;
  const size_t src = (size_t)order[i];
  for (int k = threadIdx.x; k < xsz; k += blockDim.x) xb[(size_t)i * xsz + k] = x[src * xsz + k];
  for (int k = threadIdx.x; k < tsz; k += blockDim.x) tb[(size_t)i * tsz + k] = t[src * tsz + k];
}

// Network input: for each source and band, the first image of that band, centre-cropped
// (or zero-padded) to 32x32 around the catalog position, scaled as (x - sky) / sqrt(sky).
__global__ __launch_bounds__(256) void k_patches(const SrcDev* __restrict__ srcs, const ImgDev* __restrict__ imgs,
                                                 const double* __restrict__ theta, bf16* __restrict__ out) {
  const int s = blockIdx.x;
  const double ux = theta[(size_t)s * NP], uy = theta[(size_t)s * NP + 1];
  for (int b = 0; b < 5; ++b) {
    int sel = -1;
    for (int i = srcs[s].img_begin; i < srcs[s].img_end; ++i)
      if (imgs[i].band == b) {
        sel = i;
        break;
      }
    bf16* o = out + ((size_t)s * 5 + b) * 1024;
    if (sel < 0) {
      for (int k = threadIdx.x; k < 1024; k += 256) o[k] = to_bf16(0.f);
      continue;
    }
    const ImgDev& im = imgs[sel];
    const double px = im.wcs[0] * ux + im.wcs[1] * uy + im.wcs[4] - im.origin[0];
    const double py = im.wcs[2] * ux + im.wcs[3] * uy + im.wcs[5] - im.origin[1];
    const int c0 = (int)floor(px + 0.5) - 16, r0 = (int)floor(py + 0.5) - 16;
    const float inv = (float)(1.0 / sqrt(im.sky));
    for (int k = threadIdx.x; k < 1024; k += 256) {
      const int r = r0 + k / 32, c = c0 + k % 32;
      float v = 0.f;
      if (r >= 0 && r < im.h && c >= 0 && c < im.w)
        v = ((float)im.pix[(size_t)r * im.pitch + c] - (float)im.sky) * inv;
      o[k] = to_bf16(v);
    }
  }
}

// Launches the product with at most `splits` K-splits; *splits is set to the number used
// (the count the epilogue must sum).
// ep (optional): the convolution forward epilogue, applied in the product when it has one split.
template <class LD>
hipError_t gemm(LD ld, int M, int N, int K, float* C, int& splits, hipStream_t st, EpConvFwd ep = EpConvFwd{}) {
  const int kchunk = ((K + splits - 1) / splits + TK - 1) / TK * TK;
  const int S = (K + kchunk - 1) / kchunk;
  splits = S;
  if (S != 1) ep.act = nullptr;
  dim3 grid((N + tile_n<LD>() - 1) / tile_n<LD>(), (M + TM - 1) / TM, S);
  hipLaunchKernelGGL(k_gemm<LD>, grid, dim3(256), 0, st, ld, M, N, K, kchunk, C, ep);
  return hipGetLastError();
}

inline int nblk(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 16384); }

inline int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// a convolution product over c channels may order K tap-major: c a power of two of at least 32
inline bool tap_major(int c) { return c >= 32 && (c & (c - 1)) == 0; }

}  // namespace

// ============================================================ network object (host side)

struct NetLayout {
  static constexpr int NCONV = 4;
  int cin[4] = {5, 32, 64, 64}, cout[4] = {32, 64, 64, 128}, hw[4] = {32, 32, 16, 8};
  int pool[4] = {0, 1, 1, 1};
  size_t off[12];
  size_t total = 0;
  NetLayout() {
    size_t o = 0;
    for (int l = 0; l < 4; ++l) {
      off[2 * l] = o;
      o += (size_t)cout[l] * cin[l] * 9;
      off[2 * l + 1] = o;
      o += cout[l];
    }
    off[8] = o;
    o += 256 * 2048;
    off[9] = o;
    o += 256;
    off[10] = o;
    o += 27 * 256;
    off[11] = o;
    o += 27;
    total = o;
  }
};

struct NetState {
  NetLayout L;
  float* w = nullptr;     // FP32 master weights
  float* m = nullptr;     // Adam moments
  float* v = nullptr;
  float* g = nullptr;     // gradient
  bf16* wb = nullptr;     // BF16 weights
  bf16* wt = nullptr;     // convolution weights re-laid for the data-gradient products (conv offsets)
  bf16* wf = nullptr;     // convolution weights re-laid for the tap-major forward products (conv offsets)
  int step = 0;
  int cap_batch = 0;
  // activations (BF16) and gradients for cap_batch images
  bf16 *x = nullptr, *r[4] = {}, *p[4] = {}, *h = nullptr, *dyb = nullptr, *dzb = nullptr, *dhb = nullptr;
  float *y = nullptr, *t = nullptr, *dy = nullptr, *dz = nullptr, *dh = nullptr, *C = nullptr, *loss = nullptr;
  float* bpart = nullptr;   // conv bias-gradient slices (128 channels x BP_PARTS)
  size_t c_cap = 0;
};

hipError_t net_alloc(NetState* n) {
  const size_t P = n->L.total;
  hipError_t e;
  if ((e = hipMalloc(&n->w, P * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->m, P * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->v, P * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->g, P * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->wb, P * 2)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->wt, n->L.off[8] * 2)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->wf, n->L.off[8] * 2)) != hipSuccess) return e;
  if ((e = hipMemset(n->m, 0, P * 4)) != hipSuccess) return e;
  if ((e = hipMemset(n->v, 0, P * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&n->bpart, sizeof(float) * 128 * BP_PARTS)) != hipSuccess) return e;
  return hipMalloc(&n->loss, 16);
}

void net_free_work(NetState* n) {
  bf16* bb[] = {n->x, n->r[0], n->r[1], n->r[2], n->r[3], n->p[0], n->p[1], n->p[2], n->p[3], n->h, n->dyb,
                n->dzb, n->dhb};
  for (bf16* q : bb)
    if (q) (void)hipFree(q);
  float* ff[] = {n->y, n->t, n->dy, n->dz, n->dh, n->C};
  for (float* q : ff)
    if (q) (void)hipFree(q);
  n->x = n->h = n->dyb = n->dzb = n->dhb = nullptr;
  for (int l = 0; l < 4; ++l) n->r[l] = n->p[l] = nullptr;
  n->y = n->t = n->dy = n->dz = n->dh = n->C = nullptr;
  n->cap_batch = 0;
}

void net_free(NetState* n) {
  net_free_work(n);
  float* ff[] = {n->w, n->m, n->v, n->g, n->loss, n->bpart};
  for (float* q : ff)
    if (q) (void)hipFree(q);
  if (n->wb) (void)hipFree(n->wb);
  if (n->wt) (void)hipFree(n->wt);
  if (n->wf) (void)hipFree(n->wf);
}

static const int kSplitTarget = 1024;   // aim for about this many GEMM blocks

hipError_t net_reserve(NetState* n, int B) {
  if (B <= n->cap_batch) return hipSuccess;
  net_free_work(n);
  const NetLayout& L = n->L;
  hipError_t e;
#define ALLOC(ptr, bytes) \
  if ((e = hipMalloc(&(ptr), (bytes))) != hipSuccess) return e
  ALLOC(n->x, (size_t)B * 5 * 1024 * 2);
  size_t maxact = 0;
  for (int l = 0; l < 4; ++l) {
    const size_t a = (size_t)B * L.cout[l] * L.hw[l] * L.hw[l];
    ALLOC(n->r[l], a * 2);
    const int ho = L.pool[l] ? L.hw[l] / 2 : L.hw[l];
    ALLOC(n->p[l], (size_t)B * L.cout[l] * ho * ho * 2);
    maxact = std::max(maxact, a);
  }
  ALLOC(n->h, (size_t)B * 256 * 2);
  ALLOC(n->dyb, (size_t)B * 27 * 2);
  ALLOC(n->dzb, maxact * 2);
  ALLOC(n->dhb, (size_t)B * 256 * 2);
  ALLOC(n->y, (size_t)B * 27 * 4);
  ALLOC(n->t, (size_t)B * 27 * 4);
  ALLOC(n->dy, (size_t)B * 27 * 4);
  ALLOC(n->dz, maxact * 4);
  ALLOC(n->dh, (size_t)B * 2048 * 4);
  // split-K partial products: the largest M*N times the split count
  n->c_cap = std::max(maxact * 2, (size_t)8 << 20);
  ALLOC(n->C, n->c_cap * 4);
#undef ALLOC
  n->cap_batch = B;
  return hipSuccess;
}

static int splits_for(size_t M, size_t N, size_t K, size_t cap, size_t tn = 64) {
  const size_t blocks = ((M + TM - 1) / TM) * ((N + tn - 1) / tn);
  int s = 1;
  while (blocks * s < (size_t)kSplitTarget && K / (size_t)(s * 2) >= 256 && (size_t)(s * 2) * M * N <= cap) s *= 2;
  return s;
}

// Forward pass of B images at x_in (BF16, B x 5 x 32 x 32); leaves y (FP32, B x 27).
hipError_t net_forward(NetState* n, const bf16* x_in, int B, hipStream_t st) {
  const NetLayout& L = n->L;
  hipError_t e;
  const bf16* in = x_in;
  for (int l = 0; l < 4; ++l) {
    const int HW = L.hw[l] * L.hw[l];
    const size_t M = L.cout[l], N = (size_t)B * HW, K = (size_t)L.cin[l] * 9;
    int S = splits_for(M, N, K, n->c_cap, tile_n<LdConvFwd>());
    const int wl = ilog2(L.hw[l]);
    const EpConvFwd ep{n->w + L.off[2 * l + 1], n->r[l], 2 * wl};
    if (tap_major(L.cin[l])) {
      hipLaunchKernelGGL(k_wf, dim3(nblk((size_t)L.cin[l] * L.cout[l] * 9)), dim3(256), 0, st, n->wb + L.off[2 * l],
                         L.cin[l], L.cout[l], n->wf + L.off[2 * l]);
      LdConvFwdT ld{n->wf + L.off[2 * l], in, L.cin[l], ilog2(L.cin[l]), 2 * wl, wl};
      if ((e = gemm(ld, (int)M, (int)N, (int)K, n->C, S, st, ep)) != hipSuccess) return e;
    } else {
      LdConvFwd ld{n->wb + L.off[2 * l], in, L.cin[l], 2 * wl, wl};
      if ((e = gemm(ld, (int)M, (int)N, (int)K, n->C, S, st, ep)) != hipSuccess) return e;
    }
    if (S > 1)   // split products: the epilogue sums the splits
      hipLaunchKernelGGL(k_ep_conv_fwd, dim3(nblk(M * N)), dim3(256), 0, st, n->C, S, L.cout[l], B, HW,
                         n->w + L.off[2 * l + 1], n->r[l]);
    if (L.pool[l]) {
      hipLaunchKernelGGL(k_pool_fwd, dim3(nblk((size_t)B * L.cout[l] * HW / 4)), dim3(256), 0, st, n->r[l],
                         B * L.cout[l], L.hw[l], L.hw[l], n->p[l]);
      in = n->p[l];
    } else {
      in = n->r[l];
    }
  }
  {
    int S = splits_for(256, B, 2048, n->c_cap);
    LdFcFwd ld{n->wb + L.off[8], in, 2048};
    if ((e = gemm(ld, 256, B, 2048, n->C, S, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ep_fc_fwd, dim3(nblk((size_t)256 * B)), dim3(256), 0, st, n->C, S, 256, B,
                       n->w + L.off[9], n->h, (float*)nullptr);
  }
  {
    int S = splits_for(27, B, 256, n->c_cap);
    LdFcFwd ld{n->wb + L.off[10], n->h, 256};
    if ((e = gemm(ld, 27, B, 256, n->C, S, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ep_fc_fwd, dim3(nblk((size_t)27 * B)), dim3(256), 0, st, n->C, S, 27, B,
                       n->w + L.off[11], (bf16*)nullptr, n->y);
  }
  return hipGetLastError();
}

// Loss and full gradient (into n->g) for the B images at x_in (the forward input) with
// targets in n->t.
hipError_t net_backward(NetState* n, const bf16* x_in, int B, hipStream_t st) {
  const NetLayout& L = n->L;
  hipError_t e;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, n->y, n->t, B * 27, n->dy, n->dyb, n->loss);
  // dense output layer
  {
    int S = splits_for(27, 256, B, n->c_cap);
    LdFcWgrad ld{n->dyb, n->h, 256, 27};
    if ((e = gemm(ld, 27, 256, B, n->C, S, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ep_sum, dim3(nblk(27 * 256)), dim3(256), 0, st, n->C, S, 27 * 256, n->g + L.off[10]);
    hipLaunchKernelGGL(k_bias_grad, dim3(27), dim3(256), 0, st, n->dy, B, 27, 1, n->g + L.off[11]);
    int S2 = splits_for(256, B, 27, n->c_cap);
    LdFcDgrad ld2{n->wb + L.off[10], n->dyb, 256, 27};
    if ((e = gemm(ld2, 256, B, 27, n->C, S2, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_relu_bwd_fc, dim3(nblk((size_t)256 * B)), dim3(256), 0, st, n->C, S2, 256, B, n->h, n->dh,
                       n->dhb);
  }
  // dense hidden layer
  {
    int S = splits_for(256, 2048, B, n->c_cap);
    LdFcWgrad ld{n->dhb, n->p[3], 2048, 256};
    if ((e = gemm(ld, 256, 2048, B, n->C, S, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ep_sum, dim3(nblk(256 * 2048)), dim3(256), 0, st, n->C, S, 256 * 2048, n->g + L.off[8]);
    hipLaunchKernelGGL(k_bias_grad, dim3(256), dim3(256), 0, st, n->dh, B, 256, 1, n->g + L.off[9]);
    int S2 = splits_for(2048, B, 256, n->c_cap);
    LdFcDgrad ld2{n->wb + L.off[8], n->dhb, 2048, 256};
    if ((e = gemm(ld2, 2048, B, 256, n->C, S2, st)) != hipSuccess) return e;
    // into conv4's post-ReLU activation through its pool (dense layout C[c*16+q][img])
    hipLaunchKernelGGL(k_pool_relu_bwd, dim3(nblk((size_t)B * 128 * 64)), dim3(256), 0, st, n->C, S2, 1, B, 128, 8, 8,
                       1, n->r[3], n->dz, n->dzb);
  }
  for (int l = 3; l >= 0; --l) {
    const int HW = L.hw[l] * L.hw[l];
    const bf16* xin = l == 0 ? x_in : (L.pool[l - 1] ? n->p[l - 1] : n->r[l - 1]);
    // weight and bias gradients
    {
      const size_t M = L.cout[l], N = (size_t)L.cin[l] * 9, K = (size_t)B * HW;
      int S = splits_for(M, N, K, n->c_cap);
      const int wl = ilog2(L.hw[l]);
      LdConvWgrad ld{n->dzb, xin, L.cin[l], L.cout[l], 2 * wl, wl};
      if ((e = gemm(ld, (int)M, (int)N, (int)K, n->C, S, st)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_ep_sum, dim3(nblk(M * N)), dim3(256), 0, st, n->C, S, (int)(M * N), n->g + L.off[2 * l]);
      hipLaunchKernelGGL(k_bias_part, dim3(L.cout[l], BP_PARTS), dim3(256), 0, st, n->dz, B, L.cout[l], HW,
                         n->bpart);
      hipLaunchKernelGGL(k_bias_fin, dim3((L.cout[l] + 127) / 128), dim3(128), 0, st, n->bpart, L.cout[l],
                         n->g + L.off[2 * l + 1]);
    }
    if (l == 0) break;
    // data gradient into the previous layer's post-ReLU activation (through its pool)
    {
      const size_t M = L.cin[l], N = (size_t)B * HW, K = (size_t)L.cout[l] * 9;
      int S = splits_for(M, N, K, n->c_cap, tile_n<LdConvDgrad>());
      hipLaunchKernelGGL(k_wt, dim3(nblk((size_t)L.cin[l] * L.cout[l] * 9)), dim3(256), 0, st, n->wb + L.off[2 * l],
                         L.cin[l], L.cout[l], n->wt + L.off[2 * l]);
      const int wl = ilog2(L.hw[l]);
      if (!tap_major(L.cout[l])) return hipErrorInvalidValue;   // the layout has Cout >= 32 here
      LdConvDgrad ld{n->wt + L.off[2 * l], n->dzb, L.cin[l], L.cout[l], ilog2(L.cout[l]), 2 * wl, wl};
      if ((e = gemm(ld, (int)M, (int)N, (int)K, n->C, S, st)) != hipSuccess) return e;
      const int Hp = L.hw[l - 1];
      hipLaunchKernelGGL(k_pool_relu_bwd, dim3(nblk((size_t)B * L.cout[l - 1] * Hp * Hp)), dim3(256), 0, st, n->C, S,
                         0, B, L.cout[l - 1], Hp, Hp, L.pool[l - 1], n->r[l - 1], n->dz, n->dzb);
    }
  }
  return hipGetLastError();
}

hipError_t net_adam(NetState* n, float lr, hipStream_t st) {
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)n->step), c2 = 1.f - powf(b2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n->L.total)), dim3(256), 0, st, n->w, n->m, n->v, n->g, n->wb,
                     (int)n->L.total, lr, b1, b2, c1, c2, 1e-8f);
  return hipGetLastError();
}

hipError_t net_sync_bf16(NetState* n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n->L.total)), dim3(256), 0, st, n->w, n->wb, (int)n->L.total);
  return hipGetLastError();
}

hipError_t net_gather(NetState* n, const void* x, const float* t, const int* order, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(B), dim3(256), 0, st, (const bf16*)x, t, order, B, 5 * 1024, t ? 27 : 0, n->x,
                     n->t);
  return hipGetLastError();
}

hipError_t net_acc_loss(NetState* n, float* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_acc_loss, dim3(1), dim3(1), 0, st, n->loss, acc);
  return hipGetLastError();
}

hipError_t launch_patches(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* theta, void* out,
                          hipStream_t st) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_patches, dim3(n_src), dim3(256), 0, st, srcs, imgs, theta, (bf16*)out);
  return hipGetLastError();
}

hipError_t net_destandardise(const float* y, const float* mean, const float* sd, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_destandardise, dim3(nblk(n)), dim3(256), 0, st, y, mean, sd, n, out);
  return hipGetLastError();
}

}  // namespace celeste

// ============================================================ C ABI of the network

using celeste::NetState;

struct celeste_net {
  NetState s;
  int device = 0;
  hipStream_t stream = nullptr;
  float* psi_mean = nullptr;   // device, 27
  float* psi_std = nullptr;    // device, 27
  float* acc = nullptr;        // device per-epoch loss accumulators
  int acc_cap = 0;
  void* patches = nullptr;     // device BF16 inputs for inference inside fits
  size_t patches_cap = 0;
};

namespace {
thread_local std::string g_net_err;
int net_fail(int code, const char* msg, hipError_t e = hipSuccess) {
  g_net_err = msg;
  if (e != hipSuccess) {
    g_net_err += ": ";
    g_net_err += hipGetErrorString(e);
  }
  celeste::set_error(g_net_err.c_str());
  return code;
}
#define NETCHK(x, msg)                                     \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return net_fail(CELESTE_E_DEVICE, msg, e_); \
  } while (0)
}  // namespace

namespace celeste {

// Predicted start for each source of a packed batch: patches around the catalog
// positions (theta's u), network forward in chunks, and psi = mean + std * y.
int surrogate_predict(celeste_net* net, const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* theta_cat,
                      float* psi_out, hipStream_t st) {
  const size_t need = (size_t)n_src * 5 * 1024 * 2;
  if (need > net->patches_cap) {
    if (net->patches) (void)hipFree(net->patches);
    net->patches = nullptr;
    net->patches_cap = 0;
    NETCHK(hipMalloc(&net->patches, need), "surrogate patch buffer");
    net->patches_cap = need;
  }
  NETCHK(launch_patches(srcs, n_src, imgs, theta_cat, net->patches, st), "patch extraction");
  const int chunk = 4096;
  NETCHK(net_reserve(&net->s, std::min(chunk, n_src)), "network workspace");
  for (int a = 0; a < n_src; a += chunk) {
    const int B = std::min(chunk, n_src - a);
    NETCHK(net_forward(&net->s, (const bf16*)net->patches + (size_t)a * 5 * 1024, B, st), "network forward");
    NETCHK(net_destandardise(net->s.y, net->psi_mean, net->psi_std, B * 27, psi_out + (size_t)a * 27, st),
           "destandardise");
  }
  return CELESTE_OK;
}

}  // namespace celeste

extern "C" {

int64_t celeste_net_num_params(void) { return (int64_t)celeste::NetLayout().total; }

int celeste_net_create(celeste_ctx* ctx, const float* params, int64_t n_params, const float* psi_mean,
                       const float* psi_std, celeste_net** out) {
  if (!ctx || !params || !psi_mean || !psi_std || !out) return net_fail(CELESTE_E_INVALID, "NULL argument");
  *out = nullptr;
  celeste_net* net = new (std::nothrow) celeste_net();
  if (!net) return net_fail(CELESTE_E_NOMEM, "network allocation");
  if (n_params != (int64_t)net->s.L.total) {
    delete net;
    return net_fail(CELESTE_E_INVALID, "parameter count does not match the network");
  }
  for (int j = 0; j < 27; ++j)
    if (!(psi_std[j] > 0.f) || !std::isfinite(psi_mean[j])) {
      delete net;
      return net_fail(CELESTE_E_INVALID, "psi_std must be positive and psi_mean finite");
    }
  net->device = celeste::ctx_device(ctx);
  net->stream = celeste::ctx_stream(ctx);
  hipError_t e = hipSetDevice(net->device);
  if (e == hipSuccess) e = celeste::net_alloc(&net->s);
  if (e == hipSuccess) e = hipMalloc(&net->psi_mean, 27 * 4);
  if (e == hipSuccess) e = hipMalloc(&net->psi_std, 27 * 4);
  if (e == hipSuccess) e = hipMemcpy(net->s.w, params, net->s.L.total * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->psi_mean, psi_mean, 27 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->psi_std, psi_std, 27 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = celeste::net_sync_bf16(&net->s, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (e != hipSuccess) {
    celeste::net_free(&net->s);
    delete net;
    return net_fail(CELESTE_E_DEVICE, "network set-up", e);
  }
  *out = net;
  return CELESTE_OK;
}

void celeste_net_destroy(celeste_net* net) {
  if (!net) return;
  (void)hipSetDevice(net->device);
  (void)hipStreamSynchronize(net->stream);
  celeste::net_free(&net->s);
  if (net->psi_mean) (void)hipFree(net->psi_mean);
  if (net->psi_std) (void)hipFree(net->psi_std);
  if (net->acc) (void)hipFree(net->acc);
  if (net->patches) (void)hipFree(net->patches);
  delete net;
}

int celeste_net_get_params(celeste_net* net, float* out) {
  if (!net || !out) return net_fail(CELESTE_E_INVALID, "NULL argument");
  NETCHK(hipSetDevice(net->device), "set device");
  NETCHK(hipStreamSynchronize(net->stream), "sync");
  NETCHK(hipMemcpy(out, net->s.w, net->s.L.total * 4, hipMemcpyDeviceToHost), "read parameters");
  return CELESTE_OK;
}

int celeste_net_loss_grad(celeste_net* net, const void* x, const float* t, int batch, float* loss, float* grad) {
  if (!net || !x || !t || !loss || batch < 1) return net_fail(CELESTE_E_INVALID, "bad argument");
  if ((reinterpret_cast<uintptr_t>(x) & 15) != 0) return net_fail(CELESTE_E_INVALID, "x must be 16-byte aligned");
  NETCHK(hipSetDevice(net->device), "set device");
  hipStream_t st = net->stream;
  NETCHK(celeste::net_reserve(&net->s, batch), "network workspace");
  NETCHK(hipMemcpyAsync(net->s.t, t, (size_t)batch * 27 * 4, hipMemcpyDeviceToDevice, st), "targets");
  NETCHK(celeste::net_forward(&net->s, (const celeste::bf16*)x, batch, st), "forward");
  NETCHK(celeste::net_backward(&net->s, (const celeste::bf16*)x, batch, st), "backward");
  NETCHK(hipMemcpyAsync(loss, net->s.loss, 4, hipMemcpyDeviceToHost, st), "loss");
  if (grad) NETCHK(hipMemcpyAsync(grad, net->s.g, net->s.L.total * 4, hipMemcpyDeviceToHost, st), "gradient");
  NETCHK(hipStreamSynchronize(st), "sync");
  return CELESTE_OK;
}

int celeste_net_forward(celeste_net* net, const void* x, int64_t n, float* y) {
  if (!net || !x || !y || n < 1) return net_fail(CELESTE_E_INVALID, "bad argument");
  if ((reinterpret_cast<uintptr_t>(x) & 15) != 0) return net_fail(CELESTE_E_INVALID, "x must be 16-byte aligned");
  NETCHK(hipSetDevice(net->device), "set device");
  hipStream_t st = net->stream;
  const int chunk = 4096;
  NETCHK(celeste::net_reserve(&net->s, (int)std::min<int64_t>(chunk, n)), "network workspace");
  for (int64_t a = 0; a < n; a += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n - a);
    NETCHK(celeste::net_forward(&net->s, (const celeste::bf16*)x + a * 5 * 1024, B, st), "forward");
    NETCHK(hipMemcpyAsync(y + a * 27, net->s.y, (size_t)B * 27 * 4, hipMemcpyDeviceToDevice, st), "output");
  }
  NETCHK(hipStreamSynchronize(st), "sync");
  return CELESTE_OK;
}

int celeste_net_train(celeste_net* net, const void* x, const float* t, int64_t n, const int32_t* orders, int epochs,
                      int batch, float lr, float* epoch_loss) {
  if (!net || !x || !t || !orders || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.f))
    return net_fail(CELESTE_E_INVALID, "bad argument");
  NETCHK(hipSetDevice(net->device), "set device");
  hipStream_t st = net->stream;
  NETCHK(celeste::net_reserve(&net->s, batch), "network workspace");
  if (epochs > net->acc_cap) {
    if (net->acc) (void)hipFree(net->acc);
    net->acc = nullptr;
    NETCHK(hipMalloc(&net->acc, (size_t)epochs * 4), "loss accumulators");
    net->acc_cap = epochs;
  }
  NETCHK(hipMemsetAsync(net->acc, 0, (size_t)epochs * 4, st), "zero accumulators");
  const int64_t nb = (n + batch - 1) / batch;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t b = 0; b < nb; ++b) {
      const int B = (int)std::min<int64_t>(batch, n - b * batch);
      NETCHK(celeste::net_gather(&net->s, x, t, (const int*)orders + (size_t)e * n + b * batch, B, st), "gather");
      NETCHK(celeste::net_forward(&net->s, net->s.x, B, st), "forward");
      NETCHK(celeste::net_backward(&net->s, net->s.x, B, st), "backward");
      NETCHK(celeste::net_adam(&net->s, lr, st), "adam");
      NETCHK(celeste::net_acc_loss(&net->s, net->acc + e, st), "loss");
    }
  }
  if (epoch_loss) {
    NETCHK(hipMemcpyAsync(epoch_loss, net->acc, (size_t)epochs * 4, hipMemcpyDeviceToHost, st), "losses");
    NETCHK(hipStreamSynchronize(st), "sync");
    for (int e = 0; e < epochs; ++e) epoch_loss[e] /= (float)nb;
  }
  NETCHK(hipStreamSynchronize(st), "sync");
  return CELESTE_OK;
}

}  // extern "C"
