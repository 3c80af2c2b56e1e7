// Per-source reductions: pixel-sum partials -> ELBO, gradient and dense Hessian.
//
// Partials are summed in a fixed order (work items in index order), so results
// are bitwise reproducible and independent of the batch a source sits in.  Each
// image's z-space sums are mapped to the 27 natural parameters (theta -> z is
// linear per image: band colour signs and the WCS matrix), and the closed-form
// Kullback-Leibler terms of q(a), q(r|a), q(c|a) against their priors
// (sections III-A/B) are added with their exact gradient and Hessian.  For a pixel
// subsample the work items cover only the kept rows and px_weight (1/p) scales each
// image's pixel partials; the theta-free constant of the image is added unscaled.
#include <math.h>

#include "celeste_internal.h"

namespace celeste {

namespace {

__device__ __constant__ double kSigns[5][4] = {
    {-1.0, -1.0, 0.0, 0.0}, {0.0, -1.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 1.0, 1.0}};

constexpr int tri(int i, int j) { return i * NZ - (i * (i - 1)) / 2 + (j - i); }

// z-entries (index, coefficient) that theta_i feeds in one image.
__device__ inline int theta_to_z(int i, int band, const double* wcs, int* za, double* ca) {
  if (i == 0 || i == 1) {
    za[0] = 5;
    ca[0] = wcs[i];        // A_0i
    za[1] = 6;
    ca[1] = wcs[2 + i];    // A_1i
    return 2;
  }
  if (i == 2) { za[0] = 0; ca[0] = 1.0; return 1; }
  if (i <= 6) { za[0] = 7 + (i - 3); ca[0] = 1.0; return 1; }
  if (i == 7) { za[0] = 1; ca[0] = 1.0; return 1; }
  if (i == 8) { za[0] = 3; ca[0] = 1.0; return 1; }
  if (i == 9) { za[0] = 2; ca[0] = 1.0; return 1; }
  if (i == 10) { za[0] = 4; ca[0] = 1.0; return 1; }
  if (i < 15) { za[0] = 1; ca[0] = kSigns[band][i - 11]; return 1; }
  if (i < 19) { za[0] = 3; ca[0] = kSigns[band][i - 15]; return 1; }
  const double s = kSigns[band][(i - 19) & 3];
  za[0] = i < 23 ? 2 : 4;
  ca[0] = s * s;
  return 1;
}

// Prior part of the ELBO: value, gradient and one Hessian entry.
struct KL {
  double val;
  double g[NP];
  double dks[NP];   // gradient of the star KL (r and c terms), zero elsewhere
  double dkg[NP];   // gradient of the galaxy KL
  double a;
  double d2kla;
};

__device__ void kl_value_grad(const double* th, const PriorDev& pr, KL& k) {
  const double a = th[2], phi = pr.p_star;
  for (int i = 0; i < NP; ++i) k.dks[i] = k.dkg[i] = 0.0;
  const double kla = a * log(a / phi) + (1.0 - a) * log((1.0 - a) / (1.0 - phi));
  const double dkla = log(a / phi) - log((1.0 - a) / (1.0 - phi));
  k.d2kla = 1.0 / a + 1.0 / (1.0 - a);
  k.a = a;
  double ktype[2];
  for (int t = 0; t < 2; ++t) {
    double* dk = t == 0 ? k.dks : k.dkg;
    const int ir1 = 7 + t, ir2 = 9 + t, ic1 = 11 + 4 * t, ic2 = 19 + 4 * t;
    const double r1 = th[ir1], r2 = th[ir2];
    const double mu = pr.r_mean[t], s2 = pr.r_var[t];
    double kv = 0.5 * ((r2 + (r1 - mu) * (r1 - mu)) / s2 - 1.0 - log(r2 / s2));
    dk[ir1] = (r1 - mu) / s2;
    dk[ir2] = 0.5 * (1.0 / s2 - 1.0 / r2);
    double dc[4];
    for (int j = 0; j < 4; ++j) dc[j] = th[ic1 + j] - pr.c_mean[t][j];
    double quad = 0.0, tr = 0.0, slog = 0.0;
    for (int j = 0; j < 4; ++j) {
      double row = 0.0;
      for (int l = 0; l < 4; ++l) row += pr.c_inv[t][j][l] * dc[l];
      quad += dc[j] * row;
      dk[ic1 + j] = row;
      tr += pr.c_inv[t][j][j] * th[ic2 + j];
      slog += log(th[ic2 + j]);
      dk[ic2 + j] = 0.5 * (pr.c_inv[t][j][j] - 1.0 / th[ic2 + j]);
    }
    kv += 0.5 * (tr + quad - 4.0 + pr.c_logdet[t] - slog);
    ktype[t] = kv;
  }
  k.val = -kla - a * ktype[0] - (1.0 - a) * ktype[1];
  for (int i = 0; i < NP; ++i) k.g[i] = -a * k.dks[i] - (1.0 - a) * k.dkg[i];
  k.g[2] += -dkla - ktype[0] + ktype[1];
}

// Second derivative of a single-type KL (r and c terms) in natural coordinates.
__device__ inline double kl_type_hess(const double* th, const PriorDev& pr, int t, int i, int j) {
  const int ir1 = 7 + t, ir2 = 9 + t, ic1 = 11 + 4 * t, ic2 = 19 + 4 * t;
  if (i == ir1 && j == ir1) return 1.0 / pr.r_var[t];
  if (i == ir2 && j == ir2) return 0.5 / (th[ir2] * th[ir2]);
  if (i >= ic1 && i < ic1 + 4 && j >= ic1 && j < ic1 + 4) return pr.c_inv[t][i - ic1][j - ic1];
  if (i >= ic2 && i < ic2 + 4 && i == j) return 0.5 / (th[i] * th[i]);
  return 0.0;
}

__device__ inline double kl_hess(const double* th, const PriorDev& pr, const KL& k, int i, int j) {
  double h = -k.a * kl_type_hess(th, pr, 0, i, j) - (1.0 - k.a) * kl_type_hess(th, pr, 1, i, j);
  if (i == 2) h += -k.dks[j] + k.dkg[j];
  if (j == 2) h += -k.dks[i] + k.dkg[i];
  if (i == 2 && j == 2) h += -k.d2kla;
  return h;
}

constexpr int RB = 256;
constexpr int RSLOT = 80;              // threads per image slot in k_reduce_full (NACC of them busy)
constexpr int NSLOT = RB / RSLOT;      // images whose partials are summed at once
constexpr int ICH = 24;                // images per chunk of per-image sums held in LDS

// Adds one z-space sum (tmp: value, 11 gradient, 66 Hessian entries, in LDS) mapped to the 27
// natural parameters through the map of (band, WCS matrix) to Ht / gt.  All threads; tmp
// must be complete on entry (barrier before the call); ends with a barrier.
__device__ inline void project_add(const double* tmp, int band, const double* wcs, double* Hz, double* Ht,
                                   double* gt) {
  const int t = threadIdx.x;
  if (t < NZ * NZ) {
    const int a = t / NZ, b = t - a * NZ;
    Hz[t] = tmp[1 + NZ + (a <= b ? tri(a, b) : tri(b, a))];
  }
  __syncthreads();
  for (int k = t; k < NP * NP; k += RB) {
    const int r = k / NP, c = k - r * NP;
    int zr[2], zc[2];
    double cr[2], cc[2];
    const int nr = theta_to_z(r, band, wcs, zr, cr);
    const int nc = theta_to_z(c, band, wcs, zc, cc);
    double h = 0.0;
    for (int u = 0; u < nr; ++u)
      for (int v = 0; v < nc; ++v) h += cr[u] * cc[v] * Hz[zr[u] * NZ + zc[v]];
    Ht[k] += h;
  }
  if (t < NP) {
    int zr[2];
    double cr[2];
    const int nr = theta_to_z(t, band, wcs, zr, cr);
    double g = 0.0;
    for (int u = 0; u < nr; ++u) g += cr[u] * tmp[1 + zr[u]];
    gt[t] += g;
  }
  __syncthreads();
}

// The map theta -> z of an image depends only on its band and the linear part of its WCS, so
// the z-space sums of the images that share the source's first WCS matrix are added per band
// first and mapped once per band; images with another WCS matrix are mapped one by one.
__global__ __launch_bounds__(RB) void k_reduce_full(const SrcDev* __restrict__ srcs, const ImgDev* __restrict__ imgs,
                                                    const double* __restrict__ partials,
                                                    const double* __restrict__ img_const,
                                                    const double* __restrict__ theta, PriorDev prior,
                                                    const int* __restrict__ src_flag, double* __restrict__ elbo,
                                                    double* __restrict__ grad, double* __restrict__ hess,
                                                    unsigned long long* __restrict__ px_ctr, double px_weight) {
  __shared__ double tmp[NACC];
  __shared__ double grp[5][NACC];
  __shared__ double isum[ICH][NACC];
  __shared__ double Hz[NZ * NZ];
  __shared__ double Ht[NP * NP];
  __shared__ double gt[NP];
  __shared__ double vt;
  __shared__ KL kl;
  const int s = blockIdx.x;
  if (src_flag && !src_flag[s]) return;
  const int t = threadIdx.x;
  const double* th = theta + (size_t)s * NP;
  for (int k = t; k < NP * NP; k += RB) Ht[k] = 0.0;
  if (t < NP) gt[t] = 0.0;
  if (t < NACC)
    for (int b = 0; b < 5; ++b) grp[b][t] = 0.0;
  if (t == 0) vt = 0.0;
  __syncthreads();
  const SrcDev sr = srcs[s];
  const double* wref = imgs[sr.img_begin].wcs;
  unsigned used = 0;   // bands with images in grp (the same on every thread)
  const int e = t % RSLOT, slot = t / RSLOT;
  for (int c0 = sr.img_begin; c0 < sr.img_end; c0 += ICH) {
    const int c1 = min(sr.img_end, c0 + ICH);
    // the chunk's per-image sums of the work items' partials (items in order), NSLOT images at a
    // time, so that the loads of several images are in flight together
    if (slot < NSLOT && e < NACC)
      for (int i = c0 + slot; i < c1; i += NSLOT) {
        const ImgDev& im = imgs[i];
        double acc = 0.0;
        for (int it = im.item_begin; it < im.item_end; ++it) acc += partials[(size_t)it * NACC + e];
        isum[i - c0][e] = acc * px_weight;
      }
    __syncthreads();
    for (int i = c0; i < c1; ++i) {
      const ImgDev& im = imgs[i];
      const double* acc = isum[i - c0];
      if (t == 0) vt += img_const[i];
      const bool shared = im.wcs[0] == wref[0] && im.wcs[1] == wref[1] && im.wcs[2] == wref[2] && im.wcs[3] == wref[3];
      if (shared) {
        if (t < NACC) grp[im.band][t] += acc[t];   // each thread owns its entry: no barrier needed
        used |= 1u << im.band;
      } else {
        if (t == 0) vt += acc[0];
        project_add(acc, im.band, im.wcs, Hz, Ht, gt);
      }
    }
    __syncthreads();   // the chunk's sums are read before the next chunk overwrites them
  }
  for (int b = 0; b < 5; ++b) {
    if (!(used & (1u << b))) continue;
    if (t < NACC) tmp[t] = grp[b][t];
    __syncthreads();
    if (t == 0) vt += tmp[0];
    project_add(tmp, b, wref, Hz, Ht, gt);
  }
  if (t == 0) kl_value_grad(th, prior, kl);
  __syncthreads();
  if (t == 0) {
    elbo[s] = vt + kl.val;
    if (px_ctr) atomicAdd(px_ctr, (unsigned long long)sr.npix);
  }
  if (grad && t < NP) grad[(size_t)s * NP + t] = gt[t] + kl.g[t];
  if (hess) {
    for (int k = t; k < NP * NP; k += RB) {
      const int r = k / NP, c = k - r * NP;
      hess[(size_t)s * NP * NP + k] = Ht[k] + kl_hess(th, prior, kl, r, c);
    }
  }
}

// One 64-thread block per source: value and natural gradient from gradient partials (NGRAD per
// work item), images in order, each image's z-gradient mapped through its band and WCS matrix.
__global__ __launch_bounds__(64) void k_reduce_grad(const SrcDev* __restrict__ srcs, const ImgDev* __restrict__ imgs,
                                                    const double* __restrict__ partials,
                                                    const double* __restrict__ img_const,
                                                    const double* __restrict__ theta, PriorDev prior,
                                                    const int* __restrict__ src_flag, double* __restrict__ elbo,
                                                    double* __restrict__ grad, unsigned long long* __restrict__ px_ctr,
                                                    double px_weight) {
  __shared__ double tmp[NGRAD];
  __shared__ KL kl;
  const int s = blockIdx.x;
  if (src_flag && !src_flag[s]) return;
  const int t = threadIdx.x;
  const SrcDev sr = srcs[s];
  double gt = 0.0, vt = 0.0;
  for (int i = sr.img_begin; i < sr.img_end; ++i) {
    const ImgDev& im = imgs[i];
    if (t < NGRAD) {
      double a = 0.0;
      for (int it = im.item_begin; it < im.item_end; ++it) a += partials[(size_t)it * NGRAD + t];
      tmp[t] = a * px_weight;
    }
    __syncthreads();
    if (t == 0) vt += tmp[0] + img_const[i];
    if (t < NP) {
      int zr[2];
      double cr[2];
      const int nr = theta_to_z(t, im.band, im.wcs, zr, cr);
      for (int u = 0; u < nr; ++u) gt += cr[u] * tmp[1 + zr[u]];
    }
    __syncthreads();
  }
  if (t == 0) kl_value_grad(theta + (size_t)s * NP, prior, kl);
  __syncthreads();
  if (t == 0) {
    elbo[s] = vt + kl.val;
    if (px_ctr) atomicAdd(px_ctr, (unsigned long long)sr.npix);
  }
  if (t < NP) grad[(size_t)s * NP + t] = gt + kl.g[t];
}

// One thread per source: fixed-order sum of the source's value partials.
__global__ __launch_bounds__(64) void k_reduce_value_t(const SrcDev* __restrict__ srcs, int n_src,
                                                       const ImgDev* __restrict__ imgs,
                                                       const double* __restrict__ partials,
                                                       const double* __restrict__ img_const,
                                                       const double* __restrict__ theta, PriorDev prior,
                                                       const int* __restrict__ src_flag, double* __restrict__ elbo,
                                                       unsigned long long* __restrict__ px_ctr, double px_weight) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= n_src) return;
  if (src_flag && !src_flag[s]) return;
  const SrcDev sr = srcs[s];
  double v = 0.0;
  for (int i = sr.img_begin; i < sr.img_end; ++i) {
    const ImgDev& im = imgs[i];
    double a = 0.0;
    for (int it = im.item_begin; it < im.item_end; ++it) a += partials[it];
    v += a * px_weight + img_const[i];
  }
  KL k;
  kl_value_grad(theta + (size_t)s * NP, prior, k);
  elbo[s] = v + k.val;
  if (px_ctr) atomicAdd(px_ctr, (unsigned long long)sr.npix);
}

// Prior part of the ELBO (minus the KL terms) per source.
__global__ __launch_bounds__(64) void k_prior_term(const double* __restrict__ theta, int n_src, PriorDev prior,
                                                   double* __restrict__ out) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= n_src) return;
  KL k;
  kl_value_grad(theta + (size_t)s * NP, prior, k);
  out[s] = k.val;
}

}  // namespace

hipError_t launch_prior_term(const double* theta, int n_src, PriorDev prior, double* out, hipStream_t st) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior_term, dim3((n_src + 63) / 64), dim3(64), 0, st, theta, n_src, prior, out);
  return hipGetLastError();
}

hipError_t launch_reduce_full(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                              const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                              double* elbo, double* grad, double* hess, unsigned long long* px_ctr,
                              hipStream_t st, double px_weight) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_full, dim3(n_src), dim3(RB), 0, st, srcs, imgs, partials, img_const, theta, prior,
                     src_flag, elbo, grad, hess, px_ctr, px_weight);
  return hipGetLastError();
}

hipError_t launch_reduce_grad(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                              const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                              double* elbo, double* grad, unsigned long long* px_ctr, hipStream_t st,
                              double px_weight) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_grad, dim3(n_src), dim3(64), 0, st, srcs, imgs, partials, img_const, theta, prior,
                     src_flag, elbo, grad, px_ctr, px_weight);
  return hipGetLastError();
}

hipError_t launch_reduce_value(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                               const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                               double* elbo, unsigned long long* px_ctr, hipStream_t st, double px_weight) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_value_t, dim3((n_src + 63) / 64), dim3(64), 0, st, srcs, n_src, imgs, partials,
                     img_const, theta, prior, src_flag, elbo, px_ctr, px_weight);
  return hipGetLastError();
}

}  // namespace celeste
