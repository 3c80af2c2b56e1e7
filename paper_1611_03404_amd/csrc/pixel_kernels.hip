// Pixel-sum kernels: the hot loop of the per-source ELBO (sections III-A/B).
//
// One work item = a band of rows of one image; a block takes one work item and
// its wavefronts walk the band in 64-pixel tiles, one pixel per lane (by default 8-row bands
// in column-major order, so tiles are 8 x 8 squares packed without gaps at the image's right
// edge; see TileMap).  For a pixel subsample an item is instead a run of the image's kept
// 8-row blocks (not necessarily adjacent), read through a list of their first rows.  Per pixel the kernel
// evaluates the PSF-convolved star mixture and the exp/dev galaxy mixtures with
// all derivatives needed for the gradient and dense Hessian, forms the mean and
// variance of the Poisson rate under q, applies the delta-method expected
// log-likelihood, and accumulates value, z-gradient and z-Hessian in FP64.
//
// Galaxy shape derivatives are not taken component by component.  For a Gaussian
// N(p; mu, C), dN/dC = (1/2) d2N/dmu2 (the heat equation), so derivatives with
// respect to the covariance are position-space derivatives: per pixel the kernel
// accumulates Hermite moments of orders 0-4 weighted by nu^k, and maps them onto
// (e_axis, e_angle, e_scale) once per pixel with per-image coefficients of dW/deta.
//
// Work that is exactly zero is skipped, never approximated: a mixture component whose
// exponent is below -160 on every lane of a wavefront has density exactly 0 in FP32
// there (2^-160 is far below the smallest subnormal), so all its contributions are
// exactly 0 and the wavefront branches over it.  Lanes of a tile that fall outside the
// image evaluate a point far from every component with a zero count and zero
// background variance, which makes every one of their terms exactly 0 as well.
//
// Accumulation: the ELBO value is accumulated per lane in FP64.  The gradient and the
// Hessian in z (J^T W J + a second-order part per pixel, J = [dT; dU], 2 x 11) are summed
// per lane in FP32 and every FLUSH tile steps go through a pairwise FP32 butterfly across
// the wavefront into FP64 accumulators.  Variant MF instead sums J^T W J over the 64
// pixels of a tile step (a contraction of depth 128) on the matrix cores: FP32 MFMA
// 16x16x4 in two independent accumulator chains with operands staged through LDS, added
// to FP64 every JFLUSH steps.
#include <algorithm>

#include "celeste_internal.h"

namespace celeste {

namespace {

using namespace tab;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// log(1 + u) for u >= 0.  Below u = 1/2: log(1 + u) = 2 atanh(s), s = u / (2 + u) <= 1/5, by the
// series 2 (s + s^3/3 + s^5/5 + s^7/7 + s^9/9) (the first omitted term is below 1e-8 of the sum),
// accurate relative to the result however small u is; from u = 1/2 on, the hardware base-2
// logarithm of 1 + u (log(1 + u) >= 0.4 there, so its absolute error is a small relative one).
__device__ __forceinline__ float log1p_pos(float u) {
  const float sv = u * __builtin_amdgcn_rcpf(2.f + u), s2 = sv * sv;
  const float ser = 2.f * fmaf(sv * s2, fmaf(s2, fmaf(s2, fmaf(s2, 1.f / 9.f, 1.f / 7.f), 1.f / 5.f), 1.f / 3.f), sv);
  const float lg = __builtin_amdgcn_logf(1.f + u) * 0.693147180559945309f;
  return u < 0.5f ? ser : lg;
}

// Exact-zero threshold on log2 of a component's density, a launch argument: -160 in general
// (2^-160 lies below the smallest FP32 subnormal), -127 where v_exp_f32 flushes results below
// 2^-126 to zero, which the library checks on the device when a context is created.
constexpr float FAR = 1.0e4f;      // offset used by lanes outside the image
constexpr int FLUSH = 16;          // tile steps of lane sums in FP32 before a butterfly into FP64
constexpr int JFLUSH = 8;          // tile steps of matrix-core sums in FP32 before FP64
constexpr int JP = 68;             // LDS row pitch (floats) of the staged J^T W J operands

typedef float floatx4 __attribute__((ext_vector_type(4)));

// True if the predicate holds on some lane of the wavefront (a uniform branch condition).
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Hermite moments of one galaxy profile type (exp or dev), summed over components.
struct GalAcc {
  float a0, a1x, a1y;          // sum N, N b
  float a2xx, a2xy, a2yy;      // sum N H2
  float b2xx, b2xy, b2yy;      // sum nu N H2
  float b3[4];                 // sum nu N H3: xxx, xxy, xyy, yyy
  float b4[5];                 // sum nu^2 N H4: xxxx, xxxy, xxyy, xyyy, yyyy
};

__device__ __forceinline__ void zero(GalAcc& A) {
  A.a0 = A.a1x = A.a1y = 0.f;
  A.a2xx = A.a2xy = A.a2yy = 0.f;
  A.b2xx = A.b2xy = A.b2yy = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) A.b3[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) A.b4[i] = 0.f;
}

// One galaxy component: N and the Hermite polynomials H1..H4 of b = P d,
// i.e. the derivatives of N with respect to its mean up to order 4.  Returns false (the same
// on every lane) when the component is exactly 0 on the whole tile and was skipped.
__device__ __forceinline__ bool gal_comp(const float* __restrict__ r, float dx, float dy, float dxx, float dxy,
                                         float dyy, float e_zero, GalAcc& A) {
  const float e = fmaf(r[R_QXX], dxx, fmaf(r[R_QXY], dxy, fmaf(r[R_QYY], dyy, r[R_C0])));
  if (!wave_any(e >= e_zero)) return false;
  const float N = ex2(e);
  const float Pxx = r[R_PXX], Pxy = r[R_PXY], Pyy = r[R_PYY];
  const float bx = fmaf(Pxx, dx, Pxy * dy);
  const float by = fmaf(Pxy, dx, Pyy * dy);
  const float bxx = bx * bx, bxy = bx * by, byy = by * by;
  const float h2xx = bxx - Pxx, h2xy = bxy - Pxy, h2yy = byy - Pyy;
  const float u3x = bxx - r[R_3PXX], u3y = byy - r[R_3PYY];
  const float h3xxx = bx * u3x;
  const float h3xxy = fmaf(by, h2xx, -r[R_2PXY] * bx);
  const float h3xyy = fmaf(bx, h2yy, -r[R_2PXY] * by);
  const float h3yyy = by * u3y;
  // each FMA reads at most one table value (an FP32 FMA takes one scalar-register operand)
  const float h40 = fmaf(bxx, bxx - r[R_6PXX], r[R_K4A]);
  const float h41 = fmaf(-r[R_3PXY], bxx, fmaf(bxy, u3x, r[R_K4B]));
  const float h42 = fmaf(-r[R_4PXY], bxy, fmaf(h2xx, h2yy, r[R_K4C]));
  const float h43 = fmaf(-r[R_3PXY], byy, fmaf(bxy, u3y, r[R_K4D]));
  const float h44 = fmaf(byy, byy - r[R_6PYY], r[R_K4E]);
  const float Nn = N * r[R_NU];
  const float Nn2 = Nn * r[R_NU];
  A.a0 += N;
  A.a1x = fmaf(N, bx, A.a1x);
  A.a1y = fmaf(N, by, A.a1y);
  A.a2xx = fmaf(N, h2xx, A.a2xx);
  A.a2xy = fmaf(N, h2xy, A.a2xy);
  A.a2yy = fmaf(N, h2yy, A.a2yy);
  A.b2xx = fmaf(Nn, h2xx, A.b2xx);
  A.b2xy = fmaf(Nn, h2xy, A.b2xy);
  A.b2yy = fmaf(Nn, h2yy, A.b2yy);
  A.b3[0] = fmaf(Nn, h3xxx, A.b3[0]);
  A.b3[1] = fmaf(Nn, h3xxy, A.b3[1]);
  A.b3[2] = fmaf(Nn, h3xyy, A.b3[2]);
  A.b3[3] = fmaf(Nn, h3yyy, A.b3[3]);
  A.b4[0] = fmaf(Nn2, h40, A.b4[0]);
  A.b4[1] = fmaf(Nn2, h41, A.b4[1]);
  A.b4[2] = fmaf(Nn2, h42, A.b4[2]);
  A.b4[3] = fmaf(Nn2, h43, A.b4[3]);
  A.b4[4] = fmaf(Nn2, h44, A.b4[4]);
  return true;
}

// acc += density of one component (value path).  No exact-zero skip here: one exp costs less
// than the wavefront test and branch (measured: 24.7 ms without, 29.7 ms as a select, 42.4 ms as
// a branch, for one value pass over 1.9e9 pixels).
__device__ __forceinline__ void gal_value(const float* __restrict__ r, float dxx, float dxy, float dyy, float& acc) {
  acc += ex2(fmaf(r[R_QXX], dxx, fmaf(r[R_QXY], dxy, fmaf(r[R_QYY], dyy, r[R_C0]))));
}

// Pixel -> lane layout of a work item.  Unpacked (tile width 16, 32 or 64): a grid of
// tw x (64 / tw) tiles over the item's rows; lanes past the image edge are dead.  Packed (tile
// width 8): the item's rows as 8-row bands (the image's last band may be shorter), each band's
// pixels in column-major order and the bands back to back; a tile is 64 consecutive pixels of
// that order, an 8 x 8 square except where it wraps from one band into the next, and only the
// item's last tile has dead lanes.  Bands are row_begin + 8 b for a dense item and the kept
// blocks kept[row_begin + b] for a subsampled one.
struct TileMap {
  bool packed;
  int w, rb, tw_log2, th_log2, tiles_x, q_log2, row_lim, row_safe, n_tiles;
  int nb, hl, bw, npx;
  float inv_bw, inv_hl;
  const int* kept;

  __device__ __forceinline__ TileMap(const WorkItem& wi, int w_, int h, int tw_log2_, const int* kept_) {
    w = w_;
    rb = wi.row_begin;
    kept = kept_;
    tw_log2 = tw_log2_;
    th_log2 = 6 - tw_log2;
    packed = tw_log2 == 3;
    row_lim = kept ? h : wi.row_end;
    row_safe = kept ? 0 : wi.row_begin;
    tiles_x = (w + (1 << tw_log2) - 1) >> tw_log2;
    q_log2 = 3 - th_log2;
    nb = kept ? wi.row_end - wi.row_begin : (wi.row_end - wi.row_begin + 7) >> 3;
    const int r_last = kept ? kept[wi.row_end - 1] : wi.row_begin + ((nb - 1) << 3);
    hl = min(8, row_lim - r_last);
    bw = w << 3;
    npx = (nb - 1) * bw + hl * w;
    inv_bw = 1.0f / (float)bw;
    inv_hl = 1.0f / (float)hl;
    if (packed) {
      n_tiles = (npx + 63) >> 6;
    } else {
      const int n_rows = kept ? nb << 3 : wi.row_end - wi.row_begin;
      n_tiles = tiles_x * ((n_rows + (1 << th_log2) - 1) >> th_log2);
    }
  }

  // row, column and liveness of this lane's pixel in tile t; dead lanes get an in-image pixel
  __device__ __forceinline__ void pixel(int t, int lane, int& row, int& col, bool& live) const {
    if (packed) {
      const int q = (t << 6) + lane;
      live = q < npx;
      const int qc = live ? q : 0;
      int b = (int)(((float)qc + 0.5f) * inv_bw);   // within one of the true band index
      b -= (b * bw > qc) ? 1 : 0;
      b += ((b + 1) * bw <= qc) ? 1 : 0;
      b = min(b, nb - 1);
      const int qq = qc - b * bw;
      const bool full = b < nb - 1;
      int cl = (int)(((float)qq + 0.5f) * inv_hl);   // within one of qq / hl
      cl -= (cl * hl > qq) ? 1 : 0;
      cl += ((cl + 1) * hl <= qq) ? 1 : 0;
      col = full ? qq >> 3 : cl;
      const int r = full ? (qq & 7) : qq - cl * hl;
      row = (kept ? kept[rb + b] : rb + (b << 3)) + r;
    } else {
      const int ty = t / tiles_x, tx = t - ty * tiles_x;
      const int row0 = kept ? kept[rb + (ty >> q_log2)] + ((ty & ((1 << q_log2) - 1)) << th_log2)
                            : rb + (ty << th_log2);
      row = row0 + (lane >> tw_log2);
      col = (tx << tw_log2) + (lane & ((1 << tw_log2) - 1));
      live = row < row_lim && col < w;
      if (!live) {
        row = row_safe;
        col = 0;
      }
    }
  }
};

constexpr int tri(int i, int j) { return i * NZ - (i * (i - 1)) / 2 + (j - i); }

// Brightness entries from product sums. The brightness z-derivatives of T and U are per-image
// constants times the profile values Gs, Gg:
//   dT/dz_i = ts_i Gs + tg_i Gg,   dU/dz_i = us_i Gs^2 + ug_i Gg^2 + usg_i Gs Gg   (i = 0..4),
// and so are d2T/dz_i dz_j and d2U/dz_i dz_j. The brightness gradient entries wT dT_i + wU dU_i
// and the brightness x brightness Hessian entries
//   wTT dT_i dT_j + wTU (dT_i dU_j + dU_i dT_j) + wT d2T_ij + wU d2U_ij
// are therefore fixed combinations of NBP per-pixel products
//   wT Gs, wT Gg, wU Gs^2, wU Gg^2, wU Gs Gg, wTT Gs^2, wTT Gs Gg, wTT Gg^2,
//   wTU Gs^3, wTU Gs^2 Gg, wTU Gs Gg^2, wTU Gg^3:
// the pixel loop sums the products (in 12 of the 20 brightness accumulator slots, the other 8
// stay 0) and the work item's epilogue forms the 20 entries from the sums in FP64.
constexpr int NBP = 12;
__device__ __forceinline__ constexpr int bp_slot(int p) {
  return p < 5 ? p : p < 10 ? NZ + (p - 5) : p == 10 ? NZ + tri(1, 1) : NZ + tri(1, 2);
}

// Entry e of a partial (1 + e is its index: e < 5 a brightness gradient entry, e = NZ + tri(i, j)
// with i <= j < 5 a brightness x brightness entry) from the product sums P (indexed by
// accumulator slot); other entries keep v.
__device__ double bright_entry(const float* __restrict__ T, int e, const double* P, double v) {
  const double cs = T[CS], cg = T[CG], Ks = T[KS], Kg = T[KG], Ksg = T[KSG];
  const double ts[5] = {T[MU_S], cs, 0.5 * cs, 0.0, 0.0};
  const double tg[5] = {-(double)T[MU_G], 0.0, 0.0, cg, 0.5 * cg};
  const double us[5] = {T[KA_S], 2.0 * Ks, T[KV_S], 0.0, 0.0};
  const double ug[5] = {T[KA_G], 0.0, 0.0, 2.0 * Kg, T[KV_G]};
  const double usg[5] = {T[KA_SG], Ksg, 0.5 * Ksg, Ksg, 0.5 * Ksg};
  double p[NBP];
#pragma unroll
  for (int k = 0; k < NBP; ++k) p[k] = P[bp_slot(k)];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    if (e == i) v = ts[i] * p[0] + tg[i] * p[1] + us[i] * p[2] + ug[i] * p[3] + usg[i] * p[4];
#pragma unroll
    for (int j = i; j < 5; ++j) {
      if (e != NZ + tri(i, j)) continue;
      // second-order parts d2T_ij = a Gs + b Gg, d2U_ij = c Gs^2 + d Gg^2 + f Gs Gg
      double a = 0.0, b = 0.0, c = 0.0, d = 0.0, f = 0.0;
      if (i == 0 && j == 0) { c = T[KS_AA]; d = T[KG_AA]; f = T[KSG_AA]; }
      if (i == 0 && j == 1) { a = ts[0]; c = T[KS_AM]; f = T[KSG_AM]; }
      if (i == 0 && j == 2) { a = 0.5 * ts[0]; c = T[KS_AV]; f = T[KSG_AV]; }
      if (i == 0 && j == 3) { b = tg[0]; d = T[KG_AM]; f = T[KSG_AM]; }
      if (i == 0 && j == 4) { b = 0.5 * tg[0]; d = T[KG_AV]; f = T[KSG_AV]; }
      if (i == 1 && j == 1) { a = cs; c = T[KS_MM]; f = Ksg; }
      if (i == 1 && j == 2) { a = 0.5 * cs; c = T[KS_MV]; f = 0.5 * Ksg; }
      if (i == 1 && j == 3) f = Ksg;
      if (i == 1 && j == 4) f = 0.5 * Ksg;
      if (i == 2 && j == 2) { a = 0.25 * cs; c = T[KS_VV]; f = 0.25 * Ksg; }
      if (i == 2 && j == 3) f = 0.5 * Ksg;
      if (i == 2 && j == 4) f = 0.25 * Ksg;
      if (i == 3 && j == 3) { b = cg; d = T[KG_MM]; f = Ksg; }
      if (i == 3 && j == 4) { b = 0.5 * cg; d = T[KG_MV]; f = 0.5 * Ksg; }
      if (i == 4 && j == 4) { b = 0.25 * cg; d = T[KG_VV]; f = 0.25 * Ksg; }
      v = a * p[0] + b * p[1] + c * p[2] + d * p[3] + f * p[4] + ts[i] * ts[j] * p[5] +
          (ts[i] * tg[j] + tg[i] * ts[j]) * p[6] + tg[i] * tg[j] * p[7] + (ts[i] * us[j] + us[i] * ts[j]) * p[8] +
          (ts[i] * usg[j] + tg[i] * us[j] + usg[i] * ts[j] + us[i] * tg[j]) * p[9] +
          (ts[i] * ug[j] + tg[i] * usg[j] + ug[i] * ts[j] + usg[i] * tg[j]) * p[10] +
          (tg[i] * ug[j] + ug[i] * tg[j]) * p[11];
    }
  }
  return v;
}

// Wavefront sum of 80 lane values by recursive halving (masks 32, 16, 8, 4) and a
// butterfly over the last 4 lanes: on return the lanes of each quad hold the wavefront
// sums of the 5 entries starting at quad_base(lane) = 40*b5 + 20*b4 + 10*b3 + 5*b2
// (b_k = lane bit k).
template <int N>
__device__ __forceinline__ void halvef(const float* v, float* o, int mask, bool up) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const float send = up ? v[i] : v[i + N / 2];
    const float keep = up ? v[i + N / 2] : v[i];
    o[i] = keep + __shfl_xor(send, mask);
  }
}

__device__ __forceinline__ int quad_base(int lane) {
  return ((lane >> 5) & 1) * 40 + ((lane >> 4) & 1) * 20 + ((lane >> 3) & 1) * 10 + ((lane >> 2) & 1) * 5;
}

template <int N>
__device__ __forceinline__ void halved(const double* v, double* o, int mask, bool up) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double send = up ? v[i] : v[i + N / 2];
    const double keep = up ? v[i + N / 2] : v[i];
    o[i] = keep + __shfl_xor(send, mask);
  }
}

// As wave_sum80f with every addition in FP64: the 80 FP32 values of each lane enter FP64
// before the first exchange.
__device__ __forceinline__ void wave_sum80d(const float* v, double* out5) {
  const int lane = threadIdx.x & 63;
  const bool up = (lane & 32) != 0;
  double t40[40], t20[20], t10[10];
#pragma unroll
  for (int i = 0; i < 40; ++i) {
    const float send = up ? v[i] : v[i + 40];
    const float keep = up ? v[i + 40] : v[i];
    t40[i] = (double)keep + (double)__shfl_xor(send, 32);
  }
  halved<40>(t40, t20, 16, lane & 16);
  halved<20>(t20, t10, 8, lane & 8);
  halved<10>(t10, out5, 4, lane & 4);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    out5[i] += __shfl_xor(out5[i], 2);
    out5[i] += __shfl_xor(out5[i], 1);
  }
}

__device__ __forceinline__ void wave_sum80f(const float* v, float* out5) {
  const int lane = threadIdx.x & 63;
  float t40[40], t20[20], t10[10];
  halvef<80>(v, t40, 32, lane & 32);
  halvef<40>(t40, t20, 16, lane & 16);
  halvef<20>(t20, t10, 8, lane & 8);
  halvef<10>(t10, out5, 4, lane & 4);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    out5[i] += __shfl_xor(out5[i], 2);
    out5[i] += __shfl_xor(out5[i], 1);
  }
}

// NE, ND > 0: compile-time component counts (fully unrolled loops); 0: runtime counts.
// MINW: minimum resident waves per SIMD the register allocation must allow.
// MF: the J^T W J part on the matrix cores (true) or in the per-lane FP32 sums (false).
// S64: every tile step's gradient and Hessian terms are summed across the wavefront in FP64
// (no FP32 sums across pixels; MF must be false).
template <int BLOCK, int MINW, int NE, int ND, bool MF, bool S64>
__global__ __launch_bounds__(BLOCK, MINW) void k_eval_full(const WorkItem* __restrict__ items,
                                                     const ImgDev* __restrict__ imgs,
                                                     const float* __restrict__ tables, int tstride, int n_exp,
                                                     int n_dev, const int* __restrict__ src_flag,
                                                     int tw_log2, float e_zero, const int* __restrict__ kept,
                                                     double* __restrict__ partials, WorkQueue q) {
  __shared__ double red[BLOCK / 64][80];
  // per wavefront: [A rows (dT, dU) | B columns (hT, hU)][T or U part][z index][pixel]
  __shared__ __align__(16) float jbuf[MF ? BLOCK / 64 : 1][2][2][MF ? NZ : 1][MF ? JP : 4];
  __shared__ __align__(16) float zrow[64];   // operand row of zeros for the padding rows 11..15
  if (MF) {
    if (threadIdx.x < 64) zrow[threadIdx.x] = 0.f;
    __syncthreads();
  }
  // one work item per block, or (with a queue) the items of flagged sources drawn in turn
  for (int pass = 0;; ++pass) {
  int it = blockIdx.x;
  if (q.items) {
    it = queue_next(q);
    if (it < 0) break;
  } else if (pass) {
    break;
  }
  const WorkItem wi = items[it];
  if (!q.items && src_flag && !src_flag[wi.src]) break;
  const ImgDev& im = imgs[wi.img];
  const float* __restrict__ T = tables + (size_t)wi.img * tstride;
  const int w = im.w, pitch = im.pitch, npitch = im.nbr_pitch, npsf = im.n_psf;
  const float* __restrict__ pix = im.pix;
  const float* __restrict__ nbrE = im.nbr_mean;
  const float* __restrict__ nbrV = im.nbr_var;
  const int ne = NE > 0 ? NE : n_exp;
  const int ncomp = NE > 0 ? NE + ND : n_exp + n_dev;
  const float psx = T[PSX], psy = T[PSY], io = T[CALIB], sky = T[SKY];
  const float io2 = io * io, io3 = io2 * io;

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const TileMap tm(wi, w, im.h, tw_log2, kept);
  const int n_tiles = tm.n_tiles;
  double val = 0.0;                 // ELBO value, per lane
  double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // wavefront sums of 5 derivative entries (quad-uniform)
  const int base5 = quad_base(lane);              // first of the 5 entries this lane's quad holds
  float accf[80];                   // per-lane FP32 sums of the derivative entries since the last flush
#pragma unroll
  for (int i = 0; i < 80; ++i) accf[i] = 0.f;
  int since = 0;                    // tile steps since the last flush (wavefront-uniform)
  // J^T W J: this lane holds entries (4 * (lane / 16) + r, lane % 16), r = 0..3, of the sum
  const int mi = lane & 15, kq = lane >> 4;
  const bool mrow = mi < NZ;
  double accJ[4] = {0.0, 0.0, 0.0, 0.0};
  floatx4 C0 = {0.f, 0.f, 0.f, 0.f}, C1 = {0.f, 0.f, 0.f, 0.f};   // two independent MFMA chains
  auto flushJ = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) accJ[r] += (double)C0[r] + (double)C1[r];
    C0 = floatx4{0.f, 0.f, 0.f, 0.f};
    C1 = floatx4{0.f, 0.f, 0.f, 0.f};
  };
  auto flush = [&]() {
    if constexpr (S64) {
      double part[5];
      wave_sum80d(accf, part);
#pragma unroll
      for (int i = 0; i < 5; ++i) acc5[i] += part[i];
    } else {
      float part[5];
      wave_sum80f(accf, part);
#pragma unroll
      for (int i = 0; i < 5; ++i) acc5[i] += (double)part[i];
    }
#pragma unroll
    for (int i = 0; i < 80; ++i) accf[i] = 0.f;
  };

  for (int t = wv; t < n_tiles; t += BLOCK / 64) {
    int row, col;
    bool live;
    tm.pixel(t, lane, row, col, live);   // (row, col) is inside the image on every lane
    const float x = live ? pix[(size_t)row * pitch + col] : 0.f;
    const float ebg = sky + (nbrE && live ? nbrE[(size_t)row * npitch + col] : 0.f);
    const float vbg = nbrV && live ? nbrV[(size_t)row * npitch + col] : 0.f;
    const float dx0 = live ? (float)col - psx : FAR, dy0 = live ? (float)row - psy : FAR;

    // ---- star: N, dN/dp, d2N/dp2
    bool hit = false;   // some component is not exactly 0 on this tile (wavefront-uniform)
    float s0 = 0.f, s1x = 0.f, s1y = 0.f, s2xx = 0.f, s2xy = 0.f, s2yy = 0.f;
    for (int k = 0; k < npsf; ++k) {
      const float* __restrict__ r = T + STAR + k * STAR_REC;
      const float dx = dx0 - r[S_XIX], dy = dy0 - r[S_XIY];
      const float e = fmaf(r[R_QXX], dx * dx, fmaf(r[R_QXY], dx * dy, fmaf(r[R_QYY], dy * dy, r[R_C0])));
      if (!wave_any(e >= e_zero)) continue;
      hit = true;
      const float N = ex2(e);
      const float bx = fmaf(r[R_PXX], dx, r[R_PXY] * dy), by = fmaf(r[R_PXY], dx, r[R_PYY] * dy);
      s0 += N;
      s1x = fmaf(N, bx, s1x);
      s1y = fmaf(N, by, s1y);
      s2xx = fmaf(N, fmaf(bx, bx, -r[R_PXX]), s2xx);
      s2xy = fmaf(N, fmaf(bx, by, -r[R_PXY]), s2xy);
      s2yy = fmaf(N, fmaf(by, by, -r[R_PYY]), s2yy);
    }

    // ---- galaxy: Hermite moments per profile type
    GalAcc X, D;
    zero(X);
    zero(D);
    for (int k = 0; k < npsf; ++k) {
      const float* __restrict__ sr = T + STAR + k * STAR_REC;
      const float dx = dx0 - sr[S_XIX], dy = dy0 - sr[S_XIY];
      const float dxx = dx * dx, dxy = dx * dy, dyy = dy * dy;
      // the whole galaxy group is exactly 0 on the tile when its bound is (a margin of 1 covers the
      // FP32 rounding of the bound and of the components' exponents)
      if (!wave_any(fmaf(sr[S_GMU], dxx + dyy, sr[S_GC0]) >= e_zero - 1.f)) continue;
      const float* __restrict__ base = T + GAL + k * ncomp * GAL_REC;
      if constexpr (NE > 0) {
#pragma unroll
        for (int j = 0; j < NE; ++j) hit |= gal_comp(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, X);
#pragma unroll
        for (int j = NE; j < NE + ND; ++j) hit |= gal_comp(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, D);
      } else {
        for (int j = 0; j < ne; ++j) hit |= gal_comp(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, X);
        for (int j = ne; j < ncomp; ++j) hit |= gal_comp(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, D);
      }
    }
    if (!hit) {
      // No component reaches the tile: T, U and all their derivatives are exactly 0, so the
      // gradient and Hessian terms are 0 and the pixel term keeps only its neighbour-variance
      // part, the same value as the general formula below with T = U = 0.
      const float rE = __builtin_amdgcn_rcpf(ebg);
      const float xr2 = (x * rE) * rE;
      val += (double)(0.f - 0.5f * vbg * xr2);
    } else {

      // ---- galaxy profile and its derivatives in y = (p_x, p_y, e_dev, e_axis, e_angle, e_scale)
      const float ed = T[EDEV];
      auto mix = [ed](float d, float x_) { return fmaf(ed, d - x_, x_); };
      const float Gg = mix(D.a0, X.a0);
      float dG[6], d2G[6][6];
      dG[0] = mix(D.a1x, X.a1x);
      dG[1] = mix(D.a1y, X.a1y);
      dG[2] = D.a0 - X.a0;
      const float b2c[3] = {mix(D.b2xx, X.b2xx), mix(D.b2xy, X.b2xy), mix(D.b2yy, X.b2yy)};
      const float b2d[3] = {D.b2xx - X.b2xx, D.b2xy - X.b2xy, D.b2yy - X.b2yy};
      float b3c[4], b4c[5];
#pragma unroll
      for (int i = 0; i < 4; ++i) b3c[i] = mix(D.b3[i], X.b3[i]);
#pragma unroll
      for (int i = 0; i < 5; ++i) b4c[i] = mix(D.b4[i], X.b4[i]);
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const float w0 = T[W1 + 3 * e], w1 = T[W1 + 3 * e + 1], w2 = T[W1 + 3 * e + 2];
        dG[3 + e] = fmaf(w0, b2c[0], fmaf(w1, b2c[1], w2 * b2c[2]));
        d2G[0][3 + e] = fmaf(w0, b3c[0], fmaf(w1, b3c[1], w2 * b3c[2]));
        d2G[1][3 + e] = fmaf(w0, b3c[1], fmaf(w1, b3c[2], w2 * b3c[3]));
        d2G[2][3 + e] = fmaf(w0, b2d[0], fmaf(w1, b2d[1], w2 * b2d[2]));
      }
      d2G[0][0] = mix(D.a2xx, X.a2xx);
      d2G[0][1] = mix(D.a2xy, X.a2xy);
      d2G[1][1] = mix(D.a2yy, X.a2yy);
      d2G[0][2] = D.a1x - X.a1x;
      d2G[1][2] = D.a1y - X.a1y;
      d2G[2][2] = 0.f;
      {
        int k = 0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
#pragma unroll
          for (int f = e; f < 3; ++f, ++k) {
            const float* w4 = T + W4 + 5 * k;
            const float* w2 = T + W2 + 3 * k;
            float v = w4[0] * b4c[0];
#pragma unroll
            for (int q = 1; q < 5; ++q) v = fmaf(w4[q], b4c[q], v);
            v = fmaf(w2[0], b2c[0], fmaf(w2[1], b2c[1], fmaf(w2[2], b2c[2], v)));
            d2G[3 + e][3 + f] = v;
          }
        }
      }
      // star derivatives in the same y coordinates (zero beyond the position)
      const float dGs[2] = {s1x, s1y};

      // ---- mean T and variance U of the source's contribution, and their z-derivatives
      const float cs = T[CS], cg = T[CG], mus = T[MU_S], mug = T[MU_G];
      const float Ks = T[KS], Kg = T[KG], Ksg = T[KSG];
      const float Gs = s0;
      const float Gs2 = Gs * Gs, Gg2 = Gg * Gg, Gsg = Gs * Gg;
      const float Tv = fmaf(cs, Gs, cg * Gg);
      const float Uv = fmaf(Ks, Gs2, fmaf(Kg, Gg2, Ksg * Gsg));
      const float rhos = fmaf(2.f * Ks, Gs, Ksg * Gg), rhog = fmaf(2.f * Kg, Gg, Ksg * Gs);
      float Tz[NZ], Uz[NZ];
      Tz[0] = fmaf(mus, Gs, -mug * Gg);
      Tz[1] = cs * Gs;
      Tz[2] = 0.5f * Tz[1];
      Tz[3] = cg * Gg;
      Tz[4] = 0.5f * Tz[3];
      Uz[0] = fmaf(T[KA_S], Gs2, fmaf(T[KA_G], Gg2, T[KA_SG] * Gsg));
      Uz[1] = fmaf(2.f * Ks, Gs2, Ksg * Gsg);
      Uz[2] = fmaf(T[KV_S], Gs2, 0.5f * Ksg * Gsg);
      Uz[3] = fmaf(2.f * Kg, Gg2, Ksg * Gsg);
      Uz[4] = fmaf(T[KV_G], Gg2, 0.5f * Ksg * Gsg);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const float gs = k < 2 ? dGs[k] : 0.f;
        Tz[5 + k] = fmaf(cs, gs, cg * dG[k]);
        Uz[5 + k] = fmaf(rhos, gs, rhog * dG[k]);
      }

      // ---- delta-method pixel term and its partials in (E, V)
      const float E = fmaf(io, Tv, ebg);
      const float V = fmaf(io2, Uv, vbg);
      const float rE = __builtin_amdgcn_rcpf(E);
      const float xr = x * rE, xr2 = xr * rE, xr3 = xr2 * rE;
      const float lval = fmaf(x, log1p_pos(io * Tv * __builtin_amdgcn_rcpf(ebg)), -io * Tv) - 0.5f * V * xr2;
      const float lE = fmaf(x - E, rE, V * xr3);
      const float lV = -0.5f * xr2;
      const float lEE = -fmaf(3.f * V * xr3, rE, xr2);
      const float lEV = xr3;
      const float wT = io * lE, wU = io2 * lV, wTT = io2 * lEE, wTU = io3 * lEV;

      // ---- value in FP64 per lane; gradient and second-order part in the per-lane FP32 sums
      val += (double)lval;
      const float als = fmaf(wT, cs, wU * rhos), alg = fmaf(wT, cg, wU * rhog);
      if constexpr (!MF) {
        // The geometry derivatives of T and U combine two vectors: a, the star's shape gradient
        // (zero beyond the position), and b = dG, the galaxy's:
        //   dT/dy = cs a + cg b,   dU/dy = rhos a + rhog b.
        // Every geometry entry of the gradient and Hessian terms is therefore a short combination
        // of a and b; it is formed in that basis, with no products against the zeros of a. Each
        // entry still reaches its FP32 lane sum by a single addition.
        const float* a = dGs;
        const float* b = dG;
        // brightness gradient and brightness x brightness entries: the product sums (see bp_slot)
        {
          const float tS = wTU * Gs2, tG = wTU * Gg2;
          accf[bp_slot(0)] = fmaf(wT, Gs, accf[bp_slot(0)]);
          accf[bp_slot(1)] = fmaf(wT, Gg, accf[bp_slot(1)]);
          accf[bp_slot(2)] = fmaf(wU, Gs2, accf[bp_slot(2)]);
          accf[bp_slot(3)] = fmaf(wU, Gg2, accf[bp_slot(3)]);
          accf[bp_slot(4)] = fmaf(wU, Gsg, accf[bp_slot(4)]);
          accf[bp_slot(5)] = fmaf(wTT, Gs2, accf[bp_slot(5)]);
          accf[bp_slot(6)] = fmaf(wTT, Gsg, accf[bp_slot(6)]);
          accf[bp_slot(7)] = fmaf(wTT, Gg2, accf[bp_slot(7)]);
          accf[bp_slot(8)] = fmaf(tS, Gs, accf[bp_slot(8)]);
          accf[bp_slot(9)] = fmaf(tS, Gg, accf[bp_slot(9)]);
          accf[bp_slot(10)] = fmaf(tG, Gs, accf[bp_slot(10)]);
          accf[bp_slot(11)] = fmaf(tG, Gg, accf[bp_slot(11)]);
        }
        // geometry gradient
#pragma unroll
        for (int k = 0; k < 2; ++k) accf[5 + k] += fmaf(als, a[k], alg * b[k]);
#pragma unroll
        for (int k = 2; k < 6; ++k) accf[5 + k] = fmaf(alg, b[k], accf[5 + k]);

        // brightness x geometry: entry (i, k) = P_i a_k + Q_i b_k. The geometry parts of hT and hU
        // are hTa a + hTb b and hUa a + hUb b; sa_i and sb_i are the a and b coefficients of the
        // second-order part.
        const float hTa = fmaf(wTT, cs, wTU * rhos), hTb = fmaf(wTT, cg, wTU * rhog);
        const float hUa = wTU * cs, hUb = wTU * cg;
        const float sa[5] = {fmaf(wT, mus, wU * fmaf(2.f * T[KA_S], Gs, T[KA_SG] * Gg)),
                             fmaf(wT, cs, wU * fmaf(4.f * Ks, Gs, Ksg * Gg)),
                             fmaf(wT, 0.5f * cs, wU * fmaf(2.f * T[KV_S], Gs, 0.5f * Ksg * Gg)),
                             wU * (Ksg * Gg),
                             wU * (0.5f * Ksg * Gg)};
        const float sb[5] = {fmaf(wT, -mug, wU * fmaf(2.f * T[KA_G], Gg, T[KA_SG] * Gs)),
                             wU * (Ksg * Gs),
                             wU * (0.5f * Ksg * Gs),
                             fmaf(wT, cg, wU * fmaf(4.f * Kg, Gg, Ksg * Gs)),
                             fmaf(wT, 0.5f * cg, wU * fmaf(2.f * T[KV_G], Gg, 0.5f * Ksg * Gs))};
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          const float P = fmaf(Tz[i], hTa, fmaf(Uz[i], hUa, sa[i]));
          const float Q = fmaf(Tz[i], hTb, fmaf(Uz[i], hUb, sb[i]));
#pragma unroll
          for (int k = 0; k < 2; ++k) accf[NZ + tri(i, 5 + k)] += fmaf(P, a[k], Q * b[k]);
#pragma unroll
          for (int k = 2; k < 6; ++k) accf[NZ + tri(i, 5 + k)] = fmaf(Q, b[k], accf[NZ + tri(i, 5 + k)]);
        }

        // geometry x geometry: entry (k, l) = m_aa a_k a_l + m_ab (a_k b_l + b_k a_l) + m_bb b_k b_l
        //   + als d2Gs_kl + alg d2G_kl, written as a_k v_l + b_k u_l + ...
        const float maa = fmaf(cs, hTa, fmaf(rhos, hUa, 2.f * wU * Ks));
        const float mab = fmaf(cs, hTb, fmaf(rhos, hUb, wU * Ksg));
        const float mbb = fmaf(cg, hTb, fmaf(rhog, hUb, 2.f * wU * Kg));
        float u[6], v[6];
#pragma unroll
        for (int l = 0; l < 6; ++l) {
          u[l] = l < 2 ? fmaf(mab, a[l], mbb * b[l]) : mbb * b[l];
          v[l] = l < 2 ? fmaf(maa, a[l], mab * b[l]) : mab * b[l];
        }
        const float d2Gs[3] = {s2xx, s2xy, s2yy};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
#pragma unroll
          for (int l = k; l < 6; ++l) {
            float& h = accf[NZ + tri(5 + k, 5 + l)];
            if (k == 2 && l == 2) {
              h = fmaf(u[2], b[2], h);   // d2G[2][2] = 0: e_dev enters G linearly
            } else {
              float e = alg * d2G[k][l];
              if (k < 2 && l < 2) e = fmaf(als, d2Gs[k + l], e);
              e = fmaf(u[l], b[k], e);
              if (k < 2) e = fmaf(v[l], a[k], e);
              h += e;
            }
          }
        }
      } else {
        // the second-order entries, then J^T W J by MFMA
#pragma unroll
        for (int j = 0; j < NZ; ++j) accf[j] += fmaf(wT, Tz[j], wU * Uz[j]);
        // second-order part wT d2T + wU d2U of the brightness x brightness entries (upper triangle)
        float S[NZ * (NZ + 1) / 2];
        S[tri(0, 0)] = wU * fmaf(T[KS_AA], Gs2, fmaf(T[KG_AA], Gg2, T[KSG_AA] * Gsg));
        S[tri(0, 1)] = fmaf(wT, mus * Gs, wU * fmaf(T[KS_AM], Gs2, T[KSG_AM] * Gsg));
        S[tri(0, 2)] = fmaf(wT, 0.5f * mus * Gs, wU * fmaf(T[KS_AV], Gs2, T[KSG_AV] * Gsg));
        S[tri(0, 3)] = fmaf(wT, -mug * Gg, wU * fmaf(T[KG_AM], Gg2, T[KSG_AM] * Gsg));
        S[tri(0, 4)] = fmaf(wT, -0.5f * mug * Gg, wU * fmaf(T[KG_AV], Gg2, T[KSG_AV] * Gsg));
        S[tri(1, 1)] = fmaf(wT, Tz[1], wU * fmaf(T[KS_MM], Gs2, Ksg * Gsg));
        S[tri(1, 2)] = fmaf(wT, 0.5f * Tz[1], wU * fmaf(T[KS_MV], Gs2, 0.5f * Ksg * Gsg));
        S[tri(1, 3)] = wU * Ksg * Gsg;
        S[tri(1, 4)] = 0.5f * wU * Ksg * Gsg;
        S[tri(2, 2)] = fmaf(wT, 0.25f * Tz[1], wU * fmaf(T[KS_VV], Gs2, 0.25f * Ksg * Gsg));
        S[tri(2, 3)] = 0.5f * wU * Ksg * Gsg;
        S[tri(2, 4)] = 0.25f * wU * Ksg * Gsg;
        S[tri(3, 3)] = fmaf(wT, Tz[3], wU * fmaf(T[KG_MM], Gg2, Ksg * Gsg));
        S[tri(3, 4)] = fmaf(wT, 0.5f * Tz[3], wU * fmaf(T[KG_MV], Gg2, 0.5f * Ksg * Gsg));
        S[tri(4, 4)] = fmaf(wT, 0.25f * Tz[3], wU * fmaf(T[KG_VV], Gg2, 0.25f * Ksg * Gsg));
        float hT[NZ], hU[NZ];
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
          hT[j] = fmaf(wTT, Tz[j], wTU * Uz[j]);
          hU[j] = wTU * Tz[j];
        }
        {
          // brightness x geometry block
          const float dks[5] = {T[KA_S], 2.f * Ks, T[KV_S], 0.f, 0.f};
          const float dkg[5] = {T[KA_G], 0.f, 0.f, 2.f * Kg, T[KV_G]};
          const float dksg[5] = {T[KA_SG], Ksg, 0.5f * Ksg, Ksg, 0.5f * Ksg};
          const float cts[5] = {mus, cs, 0.5f * cs, 0.f, 0.f};
          const float ctg[5] = {-mug, 0.f, 0.f, cg, 0.5f * cg};
#pragma unroll
          for (int i = 0; i < 5; ++i) {
            const float sgs = fmaf(wT, cts[i], wU * fmaf(2.f * dks[i], Gs, dksg[i] * Gg));
            const float sgg = fmaf(wT, ctg[i], wU * fmaf(2.f * dkg[i], Gg, dksg[i] * Gs));
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              const float gs = k < 2 ? dGs[k] : 0.f;
              S[tri(i, 5 + k)] = fmaf(sgs, gs, sgg * dG[k]);
            }
          }
          // geometry x geometry block
          const float d2Gs[3] = {s2xx, s2xy, s2yy};
#pragma unroll
          for (int k = 0; k < 6; ++k) {
#pragma unroll
            for (int l = k; l < 6; ++l) {
              const float gsk = k < 2 ? dGs[k] : 0.f, gsl = l < 2 ? dGs[l] : 0.f;
              const float hs = (k < 2 && l < 2) ? d2Gs[k + l] : 0.f;
              float v = fmaf(als, hs, alg * d2G[k][l]);
              const float q =
                  fmaf(2.f * Ks, gsk * gsl, fmaf(2.f * Kg, dG[k] * dG[l], Ksg * fmaf(gsk, dG[l], gsl * dG[k])));
              S[tri(5 + k, 5 + l)] = fmaf(wU, q, v);
            }
          }
        }
#pragma unroll
        for (int t = 0; t < NZ * (NZ + 1) / 2; ++t) accf[NZ + t] += S[t];
        // ---- J^T W J over the tile: C = sum_k A[:, k] B[k, :], k = 4 m + kq over (pixel, part)
        float(*J)[2][MF ? NZ : 1][MF ? JP : 4] = jbuf[wv];
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
          J[0][0][i][lane] = Tz[i];
          J[0][1][i][lane] = Uz[i];
          J[1][0][i][lane] = hT[i];
          J[1][1][i][lane] = hU[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lane (mi, kq) feeds A[mi][4m + kq] and B[4m + kq][mi]: part kq & 1 of pixel 32 (kq >> 1) + m
        const float* ar = mrow ? &J[0][kq & 1][mi][32 * (kq >> 1)] : &zrow[32 * (kq >> 1)];
        const float* br = mrow ? &J[1][kq & 1][mi][32 * (kq >> 1)] : &zrow[32 * (kq >> 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 a = *reinterpret_cast<const float4*>(ar + 4 * q);
          const float4 b = *reinterpret_cast<const float4*>(br + 4 * q);
          C0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, C0, 0, 0, 0);
          C1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, C1, 0, 0, 0);
          C0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, C0, 0, 0, 0);
          C1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, C1, 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }   // hit
    if constexpr (S64) {
      // a skipped tile step's terms are exactly 0, and adding them would leave the FP64 sums as
      // they are
      if (hit) flush();
    } else {
      // every tile step counts, so the flush points (and every bit of the result) do not depend
      // on which exactly-zero work was skipped
      ++since;
      if (MF && (since % JFLUSH) == 0) flushJ();
      if (since == FLUSH) {
        flush();
        since = 0;
      }
    }
  }
  if (MF && (since % JFLUSH)) flushJ();
  if (!S64 && since > 0) flush();

  // ---- block reduction (deterministic order) and one FP64 partial per work item
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) val += __shfl_xor(val, o);
  if (lane == 0) red[wv][0] = val;
  if ((lane & 3) == 0) {
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if (base5 + i < NACC - 1) red[wv][1 + base5 + i] = acc5[i];
  }
  if constexpr (MF) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // add the J^T W J sums (symmetric: the upper triangle is kept)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * kq + r;
      if (mrow && i <= mi) red[wv][1 + NZ + tri(i, mi)] += accJ[r];
    }
  }
  __syncthreads();
  if (threadIdx.x < NACC) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) s += red[k][threadIdx.x];
    if constexpr (MF)
      partials[(size_t)it * NACC + threadIdx.x] = s;
    else
      red[0][threadIdx.x] = s;   // each thread reads and writes only its own column here
  }
  if constexpr (!MF) {
    // the brightness entries from the product sums (the other entries pass through)
    __syncthreads();
    if (threadIdx.x < NACC)
      partials[(size_t)it * NACC + threadIdx.x] =
          bright_entry(T, (int)threadIdx.x - 1, red[0] + 1, red[0][threadIdx.x]);
  }
  }   // items
}

template <int BLOCK, int NE, int ND>
__global__ __launch_bounds__(BLOCK) void k_eval_value(const WorkItem* __restrict__ items,
                                                      const ImgDev* __restrict__ imgs,
                                                      const float* __restrict__ tables, int tstride, int n_exp_rt,
                                                      int n_dev_rt, const int* __restrict__ src_flag,
                                                      int tw_log2, const int* __restrict__ kept,
                                                      double* __restrict__ partials) {
  const int n_exp = NE > 0 ? NE : n_exp_rt, n_dev = NE > 0 ? ND : n_dev_rt;
  __shared__ double red[BLOCK / 64];
  const WorkItem wi = items[blockIdx.x];
  if (src_flag && !src_flag[wi.src]) return;
  const ImgDev& im = imgs[wi.img];
  const float* __restrict__ T = tables + (size_t)wi.img * tstride;
  const int w = im.w, pitch = im.pitch, npitch = im.nbr_pitch, npsf = im.n_psf;
  const float* __restrict__ pix = im.pix;
  const float* __restrict__ nbrE = im.nbr_mean;
  const float* __restrict__ nbrV = im.nbr_var;
  const int ncomp = n_exp + n_dev;
  const float psx = T[PSX], psy = T[PSY], io = T[CALIB], sky = T[SKY];
  const float ed = T[EDEV];
  const float cs = T[CS], cg = T[CG], Ks = T[KS], Kg = T[KG], Ksg = T[KSG];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const TileMap tm(wi, w, im.h, tw_log2, kept);
  const int n_tiles = tm.n_tiles;
  double acc = 0.0;
  for (int t = wv; t < n_tiles; t += BLOCK / 64) {
    int row, col;
    bool live;
    tm.pixel(t, lane, row, col, live);   // (row, col) is inside the image on every lane
    const float x = live ? pix[(size_t)row * pitch + col] : 0.f;
    const float ebg = sky + (nbrE && live ? nbrE[(size_t)row * npitch + col] : 0.f);
    const float vbg = nbrV && live ? nbrV[(size_t)row * npitch + col] : 0.f;
    const float dx0 = live ? (float)col - psx : FAR, dy0 = live ? (float)row - psy : FAR;
    float Gs = 0.f, gx = 0.f, gd = 0.f;
    for (int k = 0; k < npsf; ++k) {
      const float* __restrict__ r = T + STAR + k * STAR_REC;
      const float dx = dx0 - r[S_XIX], dy = dy0 - r[S_XIY];
      const float dxx = dx * dx, dxy = dx * dy, dyy = dy * dy;
      gal_value(r, dxx, dxy, dyy, Gs);
      const float* __restrict__ base = T + GAL + k * ncomp * GAL_REC;
      if constexpr (NE > 0) {
#pragma unroll
        for (int j = 0; j < NE; ++j) gal_value(base + j * GAL_REC, dxx, dxy, dyy, gx);
#pragma unroll
        for (int j = NE; j < NE + ND; ++j) gal_value(base + j * GAL_REC, dxx, dxy, dyy, gd);
      } else {
        for (int j = 0; j < n_exp; ++j) gal_value(base + j * GAL_REC, dxx, dxy, dyy, gx);
        for (int j = n_exp; j < ncomp; ++j) gal_value(base + j * GAL_REC, dxx, dxy, dyy, gd);
      }
    }
    const float Gg = fmaf(ed, gd - gx, gx);
    const float Tv = fmaf(cs, Gs, cg * Gg);
    const float Uv = fmaf(Ks, Gs * Gs, fmaf(Kg, Gg * Gg, Ksg * Gs * Gg));
    const float E = fmaf(io, Tv, ebg);
    const float V = fmaf(io * io, Uv, vbg);
    const float rE = __builtin_amdgcn_rcpf(E);
    const float lval = fmaf(x, log1p_pos(io * Tv * __builtin_amdgcn_rcpf(ebg)), -io * Tv) - 0.5f * V * (x * rE * rE);
    acc += (double)lval;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) s += red[k];
    partials[blockIdx.x] = s;
  }
}

// First-order Hermite moments of one galaxy profile type: the value, its position gradient
// and the nu-weighted second moments that give the shape gradient (dN/dC = 1/2 d2N/dmu2).
struct GalAcc1 {
  float a0, a1x, a1y;
  float b2xx, b2xy, b2yy;
};

// One galaxy component, first order only; false (on every lane) when it is exactly 0 on the tile.
__device__ __forceinline__ bool gal_comp1(const float* __restrict__ r, float dx, float dy, float dxx, float dxy,
                                          float dyy, float e_zero, GalAcc1& A) {
  const float e = fmaf(r[R_QXX], dxx, fmaf(r[R_QXY], dxy, fmaf(r[R_QYY], dyy, r[R_C0])));
  if (!wave_any(e >= e_zero)) return false;
  const float N = ex2(e);
  const float Pxx = r[R_PXX], Pxy = r[R_PXY], Pyy = r[R_PYY];
  const float bx = fmaf(Pxx, dx, Pxy * dy);
  const float by = fmaf(Pxy, dx, Pyy * dy);
  const float Nn = N * r[R_NU];
  A.a0 += N;
  A.a1x = fmaf(N, bx, A.a1x);
  A.a1y = fmaf(N, by, A.a1y);
  A.b2xx = fmaf(Nn, fmaf(bx, bx, -Pxx), A.b2xx);
  A.b2xy = fmaf(Nn, fmaf(bx, by, -Pxy), A.b2xy);
  A.b2yy = fmaf(Nn, fmaf(by, by, -Pyy), A.b2yy);
  return true;
}

constexpr int NG = NGRAD;   // entries of a gradient partial: value and the 11 z-gradient entries

// Value and z-gradient of the pixel sum (no Hessian): the same per-pixel model as k_eval_full
// with first-order moments only (6 sums per galaxy component instead of 18) and no second-
// order terms; value and gradient accumulated per lane in FP64.  One partial of NG doubles per
// work item.  Exactly-zero components, galaxy groups and tiles are skipped as in k_eval_full.
template <int BLOCK, int NE, int ND>
__global__ __launch_bounds__(BLOCK) void k_eval_grad(const WorkItem* __restrict__ items,
                                                     const ImgDev* __restrict__ imgs,
                                                     const float* __restrict__ tables, int tstride, int n_exp_rt,
                                                     int n_dev_rt, const int* __restrict__ src_flag, int tw_log2,
                                                     float e_zero, const int* __restrict__ kept,
                                                     double* __restrict__ partials) {
  __shared__ double red[BLOCK / 64][NG];
  const WorkItem wi = items[blockIdx.x];
  if (src_flag && !src_flag[wi.src]) return;
  const int ne = NE > 0 ? NE : n_exp_rt;
  const int ncomp = NE > 0 ? NE + ND : n_exp_rt + n_dev_rt;
  const ImgDev& im = imgs[wi.img];
  const float* __restrict__ T = tables + (size_t)wi.img * tstride;
  const int w = im.w, pitch = im.pitch, npitch = im.nbr_pitch, npsf = im.n_psf;
  const float* __restrict__ pix = im.pix;
  const float* __restrict__ nbrE = im.nbr_mean;
  const float* __restrict__ nbrV = im.nbr_var;
  const float psx = T[PSX], psy = T[PSY], io = T[CALIB], sky = T[SKY];
  const float io2 = io * io;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const TileMap tm(wi, w, im.h, tw_log2, kept);
  double acc[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) acc[j] = 0.0;
  for (int t = wv; t < tm.n_tiles; t += BLOCK / 64) {
    int row, col;
    bool live;
    tm.pixel(t, lane, row, col, live);   // (row, col) is inside the image on every lane
    const float x = live ? pix[(size_t)row * pitch + col] : 0.f;
    const float ebg = sky + (nbrE && live ? nbrE[(size_t)row * npitch + col] : 0.f);
    const float vbg = nbrV && live ? nbrV[(size_t)row * npitch + col] : 0.f;
    const float dx0 = live ? (float)col - psx : FAR, dy0 = live ? (float)row - psy : FAR;

    bool hit = false;
    float s0 = 0.f, s1x = 0.f, s1y = 0.f;
    for (int k = 0; k < npsf; ++k) {
      const float* __restrict__ r = T + STAR + k * STAR_REC;
      const float dx = dx0 - r[S_XIX], dy = dy0 - r[S_XIY];
      const float e = fmaf(r[R_QXX], dx * dx, fmaf(r[R_QXY], dx * dy, fmaf(r[R_QYY], dy * dy, r[R_C0])));
      if (!wave_any(e >= e_zero)) continue;
      hit = true;
      const float N = ex2(e);
      s0 += N;
      s1x = fmaf(N, fmaf(r[R_PXX], dx, r[R_PXY] * dy), s1x);
      s1y = fmaf(N, fmaf(r[R_PXY], dx, r[R_PYY] * dy), s1y);
    }
    GalAcc1 X = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, D = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < npsf; ++k) {
      const float* __restrict__ sr = T + STAR + k * STAR_REC;
      const float dx = dx0 - sr[S_XIX], dy = dy0 - sr[S_XIY];
      const float dxx = dx * dx, dxy = dx * dy, dyy = dy * dy;
      if (!wave_any(fmaf(sr[S_GMU], dxx + dyy, sr[S_GC0]) >= e_zero - 1.f)) continue;
      const float* __restrict__ base = T + GAL + k * ncomp * GAL_REC;
      if constexpr (NE > 0) {
#pragma unroll
        for (int j = 0; j < NE; ++j) hit |= gal_comp1(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, X);
#pragma unroll
        for (int j = NE; j < NE + ND; ++j) hit |= gal_comp1(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, D);
      } else {
        for (int j = 0; j < ne; ++j) hit |= gal_comp1(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, X);
        for (int j = ne; j < ncomp; ++j) hit |= gal_comp1(base + j * GAL_REC, dx, dy, dxx, dxy, dyy, e_zero, D);
      }
    }
    if (!hit) {
      // no component reaches the tile: only the neighbour-variance part of the pixel term
      const float rE = __builtin_amdgcn_rcpf(ebg);
      acc[0] += (double)(0.f - 0.5f * vbg * ((x * rE) * rE));
      continue;
    }
    const float ed = T[EDEV];
    auto mix = [ed](float d, float x_) { return fmaf(ed, d - x_, x_); };
    const float Gg = mix(D.a0, X.a0);
    float dG[6];
    dG[0] = mix(D.a1x, X.a1x);
    dG[1] = mix(D.a1y, X.a1y);
    dG[2] = D.a0 - X.a0;
    const float b2c[3] = {mix(D.b2xx, X.b2xx), mix(D.b2xy, X.b2xy), mix(D.b2yy, X.b2yy)};
#pragma unroll
    for (int e = 0; e < 3; ++e)
      dG[3 + e] = fmaf(T[W1 + 3 * e], b2c[0], fmaf(T[W1 + 3 * e + 1], b2c[1], T[W1 + 3 * e + 2] * b2c[2]));
    const float cs = T[CS], cg = T[CG], mus = T[MU_S], mug = T[MU_G];
    const float Ks = T[KS], Kg = T[KG], Ksg = T[KSG];
    const float Gs = s0;
    const float Gs2 = Gs * Gs, Gg2 = Gg * Gg, Gsg = Gs * Gg;
    const float Tv = fmaf(cs, Gs, cg * Gg);
    const float Uv = fmaf(Ks, Gs2, fmaf(Kg, Gg2, Ksg * Gsg));
    const float rhos = fmaf(2.f * Ks, Gs, Ksg * Gg), rhog = fmaf(2.f * Kg, Gg, Ksg * Gs);
    float Tz[5], Uz[5];
    Tz[0] = fmaf(mus, Gs, -mug * Gg);
    Tz[1] = cs * Gs;
    Tz[2] = 0.5f * Tz[1];
    Tz[3] = cg * Gg;
    Tz[4] = 0.5f * Tz[3];
    Uz[0] = fmaf(T[KA_S], Gs2, fmaf(T[KA_G], Gg2, T[KA_SG] * Gsg));
    Uz[1] = fmaf(2.f * Ks, Gs2, Ksg * Gsg);
    Uz[2] = fmaf(T[KV_S], Gs2, 0.5f * Ksg * Gsg);
    Uz[3] = fmaf(2.f * Kg, Gg2, Ksg * Gsg);
    Uz[4] = fmaf(T[KV_G], Gg2, 0.5f * Ksg * Gsg);
    const float dGs[2] = {s1x, s1y};
    const float E = fmaf(io, Tv, ebg);
    const float V = fmaf(io2, Uv, vbg);
    const float rE = __builtin_amdgcn_rcpf(E);
    const float xr = x * rE, xr2 = xr * rE, xr3 = xr2 * rE;
    const float lval = fmaf(x, log1p_pos(io * Tv * __builtin_amdgcn_rcpf(ebg)), -io * Tv) - 0.5f * V * xr2;
    const float wT = io * fmaf(x - E, rE, V * xr3), wU = io2 * (-0.5f * xr2);
    acc[0] += (double)lval;
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[1 + j] += (double)fmaf(wT, Tz[j], wU * Uz[j]);
    // geometry: dT/dy = cs dGs + cg dG and dU/dy = rhos dGs + rhog dG, dGs zero beyond the position
    const float als = fmaf(wT, cs, wU * rhos), alg = fmaf(wT, cg, wU * rhog);
#pragma unroll
    for (int k = 0; k < 2; ++k) acc[6 + k] += (double)fmaf(als, dGs[k], alg * dG[k]);
#pragma unroll
    for (int k = 2; k < 6; ++k) acc[6 + k] += (double)(alg * dG[k]);
  }
  // fixed-order reduction: wavefront butterfly, then the waves in index order
#pragma unroll
  for (int j = 0; j < NG; ++j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o);
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NG; ++j) red[wv][j] = acc[j];
  }
  __syncthreads();
  if (threadIdx.x < NG) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) s += red[k][threadIdx.x];
    partials[(size_t)blockIdx.x * NG + threadIdx.x] = s;
  }
}

}  // namespace

namespace {
using FullKernel = decltype(&k_eval_full<256, 1, 6, 8, false, false>);

// The value+gradient+Hessian kernel instance for (block, variant). Variant bits: 0 = the higher
// occupancy register budget (3 resident waves per SIMD for the vector kernels, 2 with the
// matrix-core J^T W J; otherwise the compiler's choice, 2 waves per SIMD for this kernel), 1 =
// mixture loops unrolled for 6 exp + 8 dev components, 2 = J^T W J on the matrix cores, 3 = FP64
// lane sums.
FullKernel full_kernel(int block, int variant, int n_exp, int n_dev) {
  const bool hi = (variant & 1) != 0;
  const bool unroll = (variant & 2) != 0 && n_exp == 6 && n_dev == 8;
  const bool s64 = (variant & 8) != 0;
  const bool mf = (variant & 4) != 0 && unroll && !s64;
  if (block == 128) {
    if (s64) {
      if (unroll) return hi ? &k_eval_full<128, 3, 6, 8, false, true> : &k_eval_full<128, 1, 6, 8, false, true>;
      return hi ? &k_eval_full<128, 3, 0, 0, false, true> : &k_eval_full<128, 1, 0, 0, false, true>;
    }
    if (mf) return hi ? &k_eval_full<128, 2, 6, 8, true, false> : &k_eval_full<128, 1, 6, 8, true, false>;
    if (unroll) return hi ? &k_eval_full<128, 3, 6, 8, false, false> : &k_eval_full<128, 1, 6, 8, false, false>;
    return hi ? &k_eval_full<128, 3, 0, 0, false, false> : &k_eval_full<128, 1, 0, 0, false, false>;
  }
  if (s64) {
    if (unroll) return hi ? &k_eval_full<256, 3, 6, 8, false, true> : &k_eval_full<256, 1, 6, 8, false, true>;
    return hi ? &k_eval_full<256, 3, 0, 0, false, true> : &k_eval_full<256, 1, 0, 0, false, true>;
  }
  if (mf) return hi ? &k_eval_full<256, 2, 6, 8, true, false> : &k_eval_full<256, 1, 6, 8, true, false>;
  if (unroll) return hi ? &k_eval_full<256, 3, 6, 8, false, false> : &k_eval_full<256, 1, 6, 8, false, false>;
  return hi ? &k_eval_full<256, 3, 0, 0, false, false> : &k_eval_full<256, 1, 0, 0, false, false>;
}
}  // namespace

hipError_t launch_eval_full(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables, int tstride,
                            int n_exp, int n_dev, const int* src_flag, double* partials, int block, int variant,
                            int tw_log2, float e_zero, hipStream_t st, const int* kept, const WorkQueue* queue,
                            int persistent_grid) {
  if (n_items <= 0) return hipSuccess;
  const WorkQueue q = queue ? *queue : WorkQueue{};
  const dim3 g(queue ? std::min(n_items, persistent_grid) : n_items);
  const FullKernel k = full_kernel(block == 128 ? 128 : 256, variant, n_exp, n_dev);
  hipLaunchKernelGGL(k, g, dim3(block == 128 ? 128 : 256), 0, st, items, imgs, tables, tstride, n_exp, n_dev,
                     src_flag, tw_log2, e_zero, kept, partials, q);
  return hipGetLastError();
}

hipError_t eval_full_blocks_per_cu(int block, int variant, int n_exp, int n_dev, int* blocks) {
  const int b = block == 128 ? 128 : 256;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, full_kernel(b, variant, n_exp, n_dev), b, 0);
}

hipError_t launch_eval_grad(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables, int tstride,
                            int n_exp, int n_dev, const int* src_flag, double* partials, int block, int variant,
                            int tw_log2, float e_zero, hipStream_t st, const int* kept) {
  if (n_items <= 0) return hipSuccess;
  const bool unroll = (variant & 2) != 0 && n_exp == 6 && n_dev == 8;
  const dim3 g(n_items);
#define CELESTE_LAUNCH_GRAD(B, E, D) \
  hipLaunchKernelGGL((k_eval_grad<B, E, D>), g, dim3(B), 0, st, items, imgs, tables, tstride, n_exp, n_dev, \
                     src_flag, tw_log2, e_zero, kept, partials)
  if (block == 128) {
    if (unroll) CELESTE_LAUNCH_GRAD(128, 6, 8); else CELESTE_LAUNCH_GRAD(128, 0, 0);
  } else {
    if (unroll) CELESTE_LAUNCH_GRAD(256, 6, 8); else CELESTE_LAUNCH_GRAD(256, 0, 0);
  }
#undef CELESTE_LAUNCH_GRAD
  return hipGetLastError();
}

namespace {
__global__ void k_exp2_probe(const float* __restrict__ in, float* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ex2(in[i]);
}
}  // namespace

hipError_t launch_exp2_probe(const float* in, float* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exp2_probe, dim3((n + 63) / 64), dim3(64), 0, st, in, out, n);
  return hipGetLastError();
}

hipError_t launch_eval_value(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables, int tstride,
                             int n_exp, int n_dev, const int* src_flag, double* partials, int block, int variant,
                             int tw_log2, hipStream_t st, const int* kept) {
  if (n_items <= 0) return hipSuccess;
  const bool unroll = (variant & 2) != 0 && n_exp == 6 && n_dev == 8;
  const dim3 g(n_items);
#define CELESTE_LAUNCH_VALUE(B, E, D) \
  hipLaunchKernelGGL((k_eval_value<B, E, D>), g, dim3(B), 0, st, items, imgs, tables, tstride, n_exp, n_dev, \
                     src_flag, tw_log2, kept, partials)
  if (block == 128) {
    if (unroll) CELESTE_LAUNCH_VALUE(128, 6, 8); else CELESTE_LAUNCH_VALUE(128, 0, 0);
  } else {
    if (unroll) CELESTE_LAUNCH_VALUE(256, 6, 8); else CELESTE_LAUNCH_VALUE(256, 0, 0);
  }
#undef CELESTE_LAUNCH_VALUE
  return hipGetLastError();
}

}  // namespace celeste
