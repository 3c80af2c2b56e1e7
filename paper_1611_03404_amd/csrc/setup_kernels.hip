// Per-image setup, per-image constants, pixel validation and the plain start.
//
// The setup kernel turns one source's parameters into the FP32 table its pixel
// work reads (section III-A model; III-B objective): the source position in the
// patch, the brightness moments of the Bernoulli/lognormal mixture in the image's
// band, the covariance precision and normaliser of every star and galaxy mixture
// component after convolution with the image's PSF, and the coefficients that map
// position-space Hermite moments onto derivatives with respect to the galaxy shape.
// All of this is computed in FP64 and rounded once to FP32.
#include <math.h>

#include "celeste_internal.h"

namespace celeste {

namespace {

// log l_b = log l_r + S_b . c, colours c_j = log(l_{j+1} / l_j), bands u,g,r,i,z.
__device__ __constant__ double kColourSigns[5][4] = {
    {-1.0, -1.0, 0.0, 0.0}, {0.0, -1.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 1.0, 1.0}};

constexpr double kLog2e = 1.4426950408889634;
constexpr double kTwoPi = 6.283185307179586;

struct Sym2 {
  double xx, xy, yy;
};

// A X A^T for symmetric X.
__device__ inline Sym2 congruence(const double* wcs, Sym2 X) {
  const double a00 = wcs[0], a01 = wcs[1], a10 = wcs[2], a11 = wcs[3];
  // rows of A X
  const double r0x = a00 * X.xx + a01 * X.xy, r0y = a00 * X.xy + a01 * X.yy;
  const double r1x = a10 * X.xx + a11 * X.xy, r1y = a10 * X.xy + a11 * X.yy;
  Sym2 o;
  o.xx = r0x * a00 + r0y * a01;
  o.xy = r0x * a10 + r0y * a11;
  o.yy = r1x * a10 + r1y * a11;
  return o;
}

struct ShapeDerivs {
  Sym2 W;         // shape matrix (image frame)
  Sym2 d[3];      // d/d(e_axis, e_angle, e_scale)
  Sym2 dd[6];     // pairs (0,0),(0,1),(0,2),(1,1),(1,2),(2,2)
};

// W = s^2 M(q,t), M = R(t) diag(1,q^2) R(t)^T, entries in closed form.
__device__ ShapeDerivs shape_derivs(double q, double t, double s, const double* wcs) {
  const double c = cos(t), sn = sin(t);
  const double c2t = cos(2.0 * t), s2t = sin(2.0 * t);
  const double omq = 1.0 - q * q;
  Sym2 M = {c * c + q * q * sn * sn, omq * c * sn, sn * sn + q * q * c * c};
  Sym2 Mq = {2.0 * q * sn * sn, -2.0 * q * c * sn, 2.0 * q * c * c};
  Sym2 Mt = {-omq * s2t, omq * c2t, omq * s2t};
  Sym2 Mqq = {2.0 * sn * sn, -2.0 * c * sn, 2.0 * c * c};
  Sym2 Mqt = {2.0 * q * s2t, -2.0 * q * c2t, -2.0 * q * s2t};
  Sym2 Mtt = {-2.0 * omq * c2t, -2.0 * omq * s2t, 2.0 * omq * c2t};
  auto sc = [](Sym2 a, double f) { return Sym2{a.xx * f, a.xy * f, a.yy * f}; };
  const double s2 = s * s;
  ShapeDerivs o;
  o.W = congruence(wcs, sc(M, s2));
  o.d[0] = congruence(wcs, sc(Mq, s2));
  o.d[1] = congruence(wcs, sc(Mt, s2));
  o.d[2] = congruence(wcs, sc(M, 2.0 * s));
  o.dd[0] = congruence(wcs, sc(Mqq, s2));
  o.dd[1] = congruence(wcs, sc(Mqt, s2));
  o.dd[2] = congruence(wcs, sc(Mq, 2.0 * s));
  o.dd[3] = congruence(wcs, sc(Mtt, s2));
  o.dd[4] = congruence(wcs, sc(Mt, 2.0 * s));
  o.dd[5] = congruence(wcs, sc(M, 2.0));
  return o;
}

__device__ inline void write_component(float* rec, double w, Sym2 C, bool galaxy, double nu) {
  const double det = C.xx * C.yy - C.xy * C.xy;
  const double inv = 1.0 / det;
  const double Pxx = C.yy * inv, Pxy = -C.xy * inv, Pyy = C.xx * inv;
  rec[tab::R_C0] = (float)(log2(w) - log2(kTwoPi) - 0.5 * log2(det));
  rec[tab::R_QXX] = (float)(-0.5 * kLog2e * Pxx);
  rec[tab::R_QXY] = (float)(-kLog2e * Pxy);
  rec[tab::R_QYY] = (float)(-0.5 * kLog2e * Pyy);
  rec[tab::R_PXX] = (float)Pxx;
  rec[tab::R_PXY] = (float)Pxy;
  rec[tab::R_PYY] = (float)Pyy;
  if (!galaxy) return;
  rec[tab::R_NU] = (float)nu;
  rec[tab::R_3PXX] = (float)(3.0 * Pxx);
  rec[tab::R_3PYY] = (float)(3.0 * Pyy);
  rec[tab::R_2PXY] = (float)(2.0 * Pxy);
  rec[tab::R_6PXX] = (float)(6.0 * Pxx);
  rec[tab::R_6PYY] = (float)(6.0 * Pyy);
  rec[tab::R_3PXY] = (float)(3.0 * Pxy);
  rec[tab::R_4PXY] = (float)(4.0 * Pxy);
  rec[tab::R_K4A] = (float)(3.0 * Pxx * Pxx);
  rec[tab::R_K4B] = (float)(3.0 * Pxx * Pxy);
  rec[tab::R_K4C] = (float)(2.0 * Pxy * Pxy);
  rec[tab::R_K4D] = (float)(3.0 * Pyy * Pxy);
  rec[tab::R_K4E] = (float)(3.0 * Pyy * Pyy);
}

// One 64-thread block per image: thread 0 writes the header and the shape
// coefficients, thread k < n_psf a star component, the rest galaxy components.
__global__ __launch_bounds__(64) void k_setup(const ImgDev* __restrict__ imgs, const double* __restrict__ theta,
                                               const int* __restrict__ src_flag, ProfDev prof,
                                               float* __restrict__ tables, int tstride) {
  const int i = blockIdx.x;
  const ImgDev& im = imgs[i];
  const int s = im.src;
  if (src_flag && !src_flag[s]) return;
  const double* th = theta + (size_t)s * NP;
  float* T = tables + (size_t)i * tstride;
  const int t = threadIdx.x;
  const double e_dev = th[3], e_axis = th[4], e_angle = th[5], e_scale = th[6];
  const ShapeDerivs sd = shape_derivs(e_axis, e_angle, e_scale, im.wcs);
  const int ncomp = prof.n_exp + prof.n_dev;

  if (t == 0) {
    const double* S = kColourSigns[im.band];
    double m_s = th[7], v_s = th[9], m_g = th[8], v_g = th[10];
    for (int j = 0; j < 4; ++j) {
      m_s += S[j] * th[11 + j];
      v_s += S[j] * S[j] * th[19 + j];
      m_g += S[j] * th[15 + j];
      v_g += S[j] * S[j] * th[23 + j];
    }
    const double a = th[2];
    const double px = im.wcs[0] * th[0] + im.wcs[1] * th[1] + im.wcs[4];
    const double py = im.wcs[2] * th[0] + im.wcs[3] * th[1] + im.wcs[5];
    const double mu_s = exp(m_s + 0.5 * v_s), mu_g = exp(m_g + 0.5 * v_g);
    const double B_s = mu_s * mu_s, B_g = mu_g * mu_g;      // E[l]^2
    const double em_s = expm1(v_s), em_g = expm1(v_g);       // e^v - 1
    const double Ks = a * B_s * (em_s + (1.0 - a));
    const double Kg = (1.0 - a) * B_g * (em_g + a);
    const double Ksg = -2.0 * a * (1.0 - a) * mu_s * mu_g;
    const double Ka_s = B_s * (em_s + 1.0 - 2.0 * a);
    const double Ka_g = -B_g * (em_g + 2.0 * a - 1.0);
    const double Ka_sg = -2.0 * (1.0 - 2.0 * a) * mu_s * mu_g;
    const double Kv_s = a * B_s * (2.0 * em_s + 2.0 - a);
    const double Kv_g = (1.0 - a) * B_g * (2.0 * em_g + 1.0 + a);
    T[tab::PSX] = (float)(px - im.origin[0]);
    T[tab::PSY] = (float)(py - im.origin[1]);
    T[tab::CALIB] = (float)im.calib;
    T[tab::SKY] = (float)im.sky;
    T[tab::CS] = (float)(a * mu_s);
    T[tab::CG] = (float)((1.0 - a) * mu_g);
    T[tab::MU_S] = (float)mu_s;
    T[tab::MU_G] = (float)mu_g;
    T[tab::KS] = (float)Ks;
    T[tab::KG] = (float)Kg;
    T[tab::KSG] = (float)Ksg;
    T[tab::KA_S] = (float)Ka_s;
    T[tab::KA_G] = (float)Ka_g;
    T[tab::KA_SG] = (float)Ka_sg;
    T[tab::KV_S] = (float)Kv_s;
    T[tab::KV_G] = (float)Kv_g;
    T[tab::EDEV] = (float)e_dev;
    T[tab::KS_AA] = (float)(-2.0 * B_s);
    T[tab::KS_AM] = (float)(2.0 * Ka_s);
    T[tab::KS_AV] = (float)(2.0 * B_s * (em_s + 1.0 - a));
    T[tab::KS_MM] = (float)(4.0 * Ks);
    T[tab::KS_MV] = (float)(2.0 * Kv_s);
    T[tab::KS_VV] = (float)(a * B_s * (4.0 * em_s + 4.0 - a));
    T[tab::KG_AA] = (float)(-2.0 * B_g);
    T[tab::KG_AM] = (float)(2.0 * Ka_g);
    T[tab::KG_AV] = (float)(-2.0 * B_g * (em_g + a));
    T[tab::KG_MM] = (float)(4.0 * Kg);
    T[tab::KG_MV] = (float)(2.0 * Kv_g);
    T[tab::KG_VV] = (float)((1.0 - a) * B_g * (4.0 * em_g + 3.0 + a));
    T[tab::KSG_AA] = (float)(4.0 * mu_s * mu_g);
    T[tab::KSG_AM] = (float)Ka_sg;
    T[tab::KSG_AV] = (float)(0.5 * Ka_sg);
    T[tab::NPSF] = (float)im.n_psf;
    // shape contractions
    for (int e = 0; e < 3; ++e) {
      T[tab::W1 + 3 * e + 0] = (float)(0.5 * sd.d[e].xx);
      T[tab::W1 + 3 * e + 1] = (float)(sd.d[e].xy);
      T[tab::W1 + 3 * e + 2] = (float)(0.5 * sd.d[e].yy);
    }
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
      const Sym2 U = sd.d[pa[k]], V = sd.d[pb[k]];
      float* w4 = T + tab::W4 + 5 * k;
      w4[0] = (float)(0.25 * U.xx * V.xx);
      w4[1] = (float)(0.5 * (U.xx * V.xy + U.xy * V.xx));
      w4[2] = (float)(0.25 * (U.xx * V.yy + 4.0 * U.xy * V.xy + U.yy * V.xx));
      w4[3] = (float)(0.5 * (U.xy * V.yy + U.yy * V.xy));
      w4[4] = (float)(0.25 * U.yy * V.yy);
      T[tab::W2 + 3 * k + 0] = (float)(0.5 * sd.dd[k].xx);
      T[tab::W2 + 3 * k + 1] = (float)(sd.dd[k].xy);
      T[tab::W2 + 3 * k + 2] = (float)(0.5 * sd.dd[k].yy);
    }
  }
  if (t < im.n_psf) {
    const double* ps = im.psf[t];
    float* rec = T + tab::STAR + t * tab::STAR_REC;
    write_component(rec, ps[0], Sym2{ps[3], ps[4], ps[5]}, false, 0.0);
    rec[tab::S_XIX] = (float)ps[1];
    rec[tab::S_XIY] = (float)ps[2];
    // bound of this PSF component's galaxy group: C_j = nu_j W + Sigma_k has
    // lambda_max(C_j) <= nu_max lambda_max(W) + lambda_max(Sigma_k) and det C_j >= det Sigma_k, so
    // each component's log2 density is at most log2(w_k amp_max / (2 pi sqrt(det Sigma_k))) -
    // log2(e) |d|^2 / (2 (nu_max lambda_max(W) + lambda_max(Sigma_k))); both rounded up
    double amp_max = 0.0, nu_max = 0.0;
    for (int j = 0; j < ncomp; ++j) {
      amp_max = fmax(amp_max, prof.amp[j]);
      nu_max = fmax(nu_max, prof.var[j]);
    }
    auto lam_max = [](double a, double b, double c) { return 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b); };
    const double lmax = nu_max * lam_max(sd.W.xx, sd.W.xy, sd.W.yy) + lam_max(ps[3], ps[4], ps[5]);
    const double c0b = log2(ps[0] * amp_max) - log2(kTwoPi) - 0.5 * log2(ps[3] * ps[5] - ps[4] * ps[4]);
    const double mub = -0.5 * kLog2e / lmax;
    float c0f = (float)c0b, muf = (float)mub;
    if ((double)c0f < c0b) c0f = nextafterf(c0f, INFINITY);
    if ((double)muf < mub) muf = nextafterf(muf, INFINITY);
    rec[tab::S_GC0] = c0f;
    rec[tab::S_GMU] = muf;
  }
  for (int c = t; c < im.n_psf * ncomp; c += blockDim.x) {
    const int k = c / ncomp, j = c - k * ncomp;
    const double* ps = im.psf[k];
    const double nu = prof.var[j];
    Sym2 C = {nu * sd.W.xx + ps[3], nu * sd.W.xy + ps[4], nu * sd.W.yy + ps[5]};
    write_component(T + tab::GAL + c * tab::GAL_REC, ps[0] * prof.amp[j], C, true, nu);
  }
}

template <int BLOCK>
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BLOCK / 64; ++k) r += sh[k];
  return r;
}

// log n! for the integer counts below LFACT_N, filled with the device's own lgamma(n + 1).
__global__ __launch_bounds__(256) void k_lfact(double* __restrict__ t) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < LFACT_N) t[i] = lgamma((double)i + 1.0);
}

// One pass over every pixel of an image (one block per image): flags any negative or
// non-finite pixel / neighbour value, and sums the theta-independent part of the pixel term,
// x log E_bg - E_bg - log x!, E_bg = sky + neighbour mean.  log x! of an integer count below
// LFACT_N is read from the table (the same value lgamma gives); without neighbour arrays E_bg
// is the sky at every pixel, so the first two terms are log(sky) sum x - n sky.
__global__ __launch_bounds__(256) void k_check_const(const ImgDev* __restrict__ imgs, const double* __restrict__ lfact,
                                                     double* __restrict__ out, int* __restrict__ bad) {
  __shared__ double sh[4];
  const ImgDev& im = imgs[blockIdx.x];
  const int n = im.h * im.w;
  double acc = 0.0, sx = 0.0;
  int cnt = 0, flag = 0;
  // four pixels per thread and step, their loads issued before any is used (the pass is bound by
  // memory latency, not bandwidth)
  constexpr int U = 4;
  for (int m0 = threadIdx.x; m0 < n; m0 += U * 256) {
    float xs[U], es[U], vs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = min(m0 + u * 256, n - 1);
      const int r = m / im.w, c = m - r * im.w;
      const size_t o = (size_t)r * im.pitch + c;
      const size_t on = (size_t)r * im.nbr_pitch + c;
      xs[u] = im.pix[o];
      es[u] = im.nbr_mean ? im.nbr_mean[on] : 0.f;
      vs[u] = im.nbr_var ? im.nbr_var[on] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (m0 + u * 256 >= n) break;
      const float xf = xs[u];
      if (!(xf >= 0.0f) || !isfinite(xf)) flag = 1;
      const double x = xf;
      double lg;
      if (x >= 0.0 && x < (double)LFACT_N && x == (double)(int)x)
        lg = lfact[(int)x];
      else
        lg = lgamma(x + 1.0);
      if (im.nbr_mean) {
        const float e = es[u];
        if (!(e >= 0.0f) || !isfinite(e)) flag = 1;
        const double ebg = im.sky + (double)e;
        acc += x * log(ebg) - ebg - lg;
      } else {
        sx += x;
        ++cnt;
        acc -= lg;
      }
      if (im.nbr_var) {
        const float v = vs[u];
        if (!(v >= 0.0f) || !isfinite(v)) flag = 1;
      }
    }
  }
  if (!im.nbr_mean) acc += log(im.sky) * sx - (double)cnt * im.sky;
  const double tot = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
  if (flag) atomicOr(bad, 1);
}

// Plain start: aperture flux (radius 3 px around the catalog position) in the
// r-band images, prior moments for the rest.  One block per source.
__global__ __launch_bounds__(256) void k_plain_init(const SrcDev* __restrict__ srcs, const ImgDev* __restrict__ imgs,
                                                    PriorDev prior, double* __restrict__ theta) {
  __shared__ double sh[4];
  __shared__ double flux_sum;
  __shared__ int n_r;
  const int s = blockIdx.x;
  double* th = theta + (size_t)s * NP;
  const double ux = th[0], uy = th[1];
  if (threadIdx.x == 0) {
    flux_sum = 0.0;
    n_r = 0;
  }
  __syncthreads();
  for (int i = srcs[s].img_begin; i < srcs[s].img_end; ++i) {
    const ImgDev& im = imgs[i];
    if (im.band != 2) continue;
    const double px = im.wcs[0] * ux + im.wcs[1] * uy + im.wcs[4];
    const double py = im.wcs[2] * ux + im.wcs[3] * uy + im.wcs[5];
    const int n = im.h * im.w;
    double acc = 0.0;
    for (int m = threadIdx.x; m < n; m += 256) {
      const int r = m / im.w, c = m - r * im.w;
      const double dx = im.origin[0] + c - px, dy = im.origin[1] + r - py;
      if (dx * dx + dy * dy <= 9.0) acc += ((double)im.pix[(size_t)r * im.pitch + c] - im.sky) / im.calib;
    }
    const double tot = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) {
      flux_sum += tot;
      n_r += 1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = n_r > 0 ? flux_sum / n_r : 1.0;
    const double r1 = log(fmax(f, 1.0));
    th[2] = 0.5;
    th[3] = 0.5;
    th[4] = 0.7;
    th[5] = 0.0;
    th[6] = 1.5;
    th[7] = r1;
    th[8] = r1;
    th[9] = prior.r_var[0];
    th[10] = prior.r_var[1];
    for (int j = 0; j < 4; ++j) {
      th[11 + j] = prior.c_mean[0][j];
      th[15 + j] = prior.c_mean[1][j];
      th[19 + j] = prior.c_diag[0][j];
      th[23 + j] = prior.c_diag[1][j];
    }
  }
}

}  // namespace

hipError_t launch_setup(const ImgDev* imgs, int n_img, const double* theta, const int* src_flag, ProfDev prof,
                        float* tables, int tstride, hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_setup, dim3(n_img), dim3(64), 0, st, imgs, theta, src_flag, prof, tables, tstride);
  return hipGetLastError();
}

hipError_t launch_lfact(double* table, hipStream_t st) {
  hipLaunchKernelGGL(k_lfact, dim3((LFACT_N + 255) / 256), dim3(256), 0, st, table);
  return hipGetLastError();
}

hipError_t launch_check_const(const ImgDev* imgs, int n_img, const double* lfact, double* img_const, int* bad,
                              hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_const, dim3(n_img), dim3(256), 0, st, imgs, lfact, img_const, bad);
  return hipGetLastError();
}

hipError_t launch_plain_init(const SrcDev* srcs, int n_src, const ImgDev* imgs, PriorDev prior, double* theta,
                             hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plain_init, dim3(n_src), dim3(256), 0, s, srcs, imgs, prior, theta);
  return hipGetLastError();
}

}  // namespace celeste
