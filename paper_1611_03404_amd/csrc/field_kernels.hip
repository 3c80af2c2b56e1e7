// Crowded fields: rendering every source's expected counts and their variance into shared
// field images, and the per-source neighbour arrays (section III-B: each source is
// optimised with the other sources held fixed at their current estimates; pixels receive
// photons from several sources).
//
// Rendering is a gather, deterministic by construction: one block per 32x32 tile of a
// field walks the list of source patches overlapping the tile in source order and sums
// their contributions in FP64 per pixel.  The neighbour array of a source is the rendered
// field minus the source's own contribution, computed by the same per-pixel routine.
#include "celeste_internal.h"

namespace celeste {

namespace {

using namespace tab;

constexpr int RTILE = 32;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ float comp(const float* __restrict__ r, float dxx, float dxy, float dyy) {
  return ex2(fmaf(r[R_QXX], dxx, fmaf(r[R_QXY], dxy, fmaf(r[R_QYY], dyy, r[R_C0]))));
}

// Source contribution at one pixel, relative position (dx0, dy0) from the source in
// patch coordinates: expected counts calib*T and variance calib^2*U.  Kept out of line so
// rendering and self-subtraction run the identical instruction sequence.
__device__ __noinline__ void source_rate(const float* __restrict__ T, float dx0, float dy0, int npsf, int ne,
                                         int ncomp, float* e_out, float* v_out) {
  float Gs = 0.f, gx = 0.f, gd = 0.f;
  for (int k = 0; k < npsf; ++k) {
    const float* __restrict__ sr = T + STAR + k * STAR_REC;
    const float dx = dx0 - sr[S_XIX], dy = dy0 - sr[S_XIY];
    const float dxx = dx * dx, dxy = dx * dy, dyy = dy * dy;
    Gs += comp(sr, dxx, dxy, dyy);
    const float* __restrict__ base = T + GAL + k * ncomp * GAL_REC;
    for (int j = 0; j < ne; ++j) gx += comp(base + j * GAL_REC, dxx, dxy, dyy);
    for (int j = ne; j < ncomp; ++j) gd += comp(base + j * GAL_REC, dxx, dxy, dyy);
  }
  const float ed = T[EDEV];
  const float Gg = fmaf(ed, gd - gx, gx);
  const float io = T[CALIB];
  const float Tv = fmaf(T[CS], Gs, T[CG] * Gg);
  const float Uv = fmaf(T[KS], Gs * Gs, fmaf(T[KG], Gg * Gg, T[KSG] * Gs * Gg));
  *e_out = io * Tv;
  *v_out = io * io * Uv;
}

__global__ __launch_bounds__(256) void k_render(const int* __restrict__ tile_off, const int* __restrict__ tile_img,
                                                const ImgDev* __restrict__ imgs, const float* __restrict__ tables,
                                                int tstride, int n_exp, int n_dev, int H, int W, int tiles_x,
                                                int tiles_per_field, float* __restrict__ mean,
                                                float* __restrict__ var) {
  const int tile = blockIdx.x;
  const int f = tile / tiles_per_field, tt = tile - f * tiles_per_field;
  const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
  const int px = tx * RTILE + (threadIdx.x & (RTILE - 1));
  const int py0 = ty * RTILE + (threadIdx.x >> 5);
  double e[4] = {0.0, 0.0, 0.0, 0.0}, v[4] = {0.0, 0.0, 0.0, 0.0};
  const int ncomp = n_exp + n_dev;
  for (int q = tile_off[tile]; q < tile_off[tile + 1]; ++q) {
    const int i = tile_img[q];
    const ImgDev& im = imgs[i];
    const float* __restrict__ T = tables + (size_t)i * tstride;
    const int c0 = (int)im.origin[0], r0 = (int)im.origin[1];
    const float psx = T[PSX], psy = T[PSY];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int py = py0 + 8 * k;
      const int c = px - c0, r = py - r0;
      if (c >= 0 && c < im.w && r >= 0 && r < im.h) {
        float de, dv;
        source_rate(T, (float)c - psx, (float)r - psy, im.n_psf, n_exp, ncomp, &de, &dv);
        e[k] += (double)de;
        v[k] += (double)dv;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int py = py0 + 8 * k;
    if (px < W && py < H) {
      const size_t o = ((size_t)f * H + py) * W + px;
      mean[o] = (float)e[k];
      var[o] = (float)v[k];
    }
  }
}

// Neighbour arrays of one patch image: field totals minus the source's own contribution,
// clamped at zero against rounding.
__global__ __launch_bounds__(256) void k_neighbours(const ImgDev* __restrict__ imgs, const int* __restrict__ img_field,
                                                    const float* __restrict__ tables, int tstride, int n_exp,
                                                    int n_dev, int H, int W, const float* __restrict__ mean,
                                                    const float* __restrict__ var,
                                                    const long long* __restrict__ nbr_off,
                                                    float* __restrict__ nbr_mean, float* __restrict__ nbr_var) {
  const int i = blockIdx.x;
  const ImgDev& im = imgs[i];
  const float* __restrict__ T = tables + (size_t)i * tstride;
  const int c0 = (int)im.origin[0], r0 = (int)im.origin[1];
  const int f = img_field[i];
  const float psx = T[PSX], psy = T[PSY];
  const int n = im.h * im.w;
  float* om = nbr_mean + nbr_off[i];
  float* ov = nbr_var + nbr_off[i];
  for (int m = threadIdx.x; m < n; m += 256) {
    const int r = m / im.w, c = m - r * im.w;
    float de, dv;
    source_rate(T, (float)c - psx, (float)r - psy, im.n_psf, n_exp, n_exp + n_dev, &de, &dv);
    const size_t o = ((size_t)f * H + (r0 + r)) * W + (c0 + c);
    om[m] = fmaxf(mean[o] - de, 0.f);
    ov[m] = fmaxf(var[o] - dv, 0.f);
  }
}

// Moves the field images from one estimate of the batch's sources to another: each pixel of
// each patch gets (new - old) contribution of its source.  Patches of one launch must not
// overlap within a field, so every pixel has a single writer.
__global__ __launch_bounds__(256) void k_update(const ImgDev* __restrict__ imgs, const int* __restrict__ img_field,
                                                const float* __restrict__ t_old, const float* __restrict__ t_new,
                                                int tstride, int n_exp, int n_dev, int H, int W,
                                                float* __restrict__ mean, float* __restrict__ var) {
  const int i = blockIdx.x;
  const ImgDev& im = imgs[i];
  const float* __restrict__ To = t_old + (size_t)i * tstride;
  const float* __restrict__ Tn = t_new + (size_t)i * tstride;
  const int c0 = (int)im.origin[0], r0 = (int)im.origin[1];
  const int f = img_field[i];
  const int n = im.h * im.w;
  for (int m = threadIdx.x; m < n; m += 256) {
    const int r = m / im.w, c = m - r * im.w;
    float eo, vo, en, vn;
    source_rate(To, (float)c - To[PSX], (float)r - To[PSY], im.n_psf, n_exp, n_exp + n_dev, &eo, &vo);
    source_rate(Tn, (float)c - Tn[PSX], (float)r - Tn[PSY], im.n_psf, n_exp, n_exp + n_dev, &en, &vn);
    const size_t o = ((size_t)f * H + (r0 + r)) * W + (c0 + c);
    mean[o] = fmaxf(mean[o] + (en - eo), 0.f);
    var[o] = fmaxf(var[o] + (vn - vo), 0.f);
  }
}

// Delta-method expected log-likelihood of every field pixel in FP64 (E = sky + mean,
// Var = var), one partial sum per block.
__global__ __launch_bounds__(256) void k_field_terms(const float* __restrict__ x, const float* __restrict__ mean,
                                                     const float* __restrict__ var,
                                                     const double* __restrict__ sky, int H, int W, int n_fields,
                                                     int per_block, double* __restrict__ partials) {
  __shared__ double red[4];
  const size_t npf = (size_t)H * W, n = npf * n_fields;
  const size_t b0 = (size_t)blockIdx.x * per_block;
  double acc = 0.0;
  for (size_t k = b0 + threadIdx.x; k < b0 + per_block && k < n; k += 256) {
    const double xv = x[k], E = sky[k / npf] + (double)mean[k], V = var[k];
    acc += xv * (log(E) - V / (2.0 * E * E)) - E - lgamma(xv + 1.0);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

hipError_t launch_update_fields(const ImgDev* imgs, int n_img, const int* img_field, const float* t_old,
                                const float* t_new, int tstride, int n_exp, int n_dev, int H, int W, float* mean,
                                float* var, hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update, dim3(n_img), dim3(256), 0, st, imgs, img_field, t_old, t_new, tstride, n_exp, n_dev, H,
                     W, mean, var);
  return hipGetLastError();
}

hipError_t launch_field_terms(const float* x, const float* mean, const float* var, const double* sky, int H, int W,
                              int n_fields, int per_block, int n_blocks, double* partials, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_field_terms, dim3(n_blocks), dim3(256), 0, st, x, mean, var, sky, H, W, n_fields, per_block,
                     partials);
  return hipGetLastError();
}

hipError_t launch_render(const int* tile_off, const int* tile_img, int n_tiles, const ImgDev* imgs,
                         const float* tables, int tstride, int n_exp, int n_dev, int H, int W, int tiles_x,
                         int tiles_per_field, float* mean, float* var, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_render, dim3(n_tiles), dim3(256), 0, st, tile_off, tile_img, imgs, tables, tstride, n_exp,
                     n_dev, H, W, tiles_x, tiles_per_field, mean, var);
  return hipGetLastError();
}

hipError_t launch_neighbours(const ImgDev* imgs, int n_img, const int* img_field, const float* tables, int tstride,
                             int n_exp, int n_dev, int H, int W, const float* mean, const float* var,
                             const long long* nbr_off, float* nbr_mean, float* nbr_var, hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_neighbours, dim3(n_img), dim3(256), 0, st, imgs, img_field, tables, tstride, n_exp, n_dev, H,
                     W, mean, var, nbr_off, nbr_mean, nbr_var);
  return hipGetLastError();
}

}  // namespace celeste
