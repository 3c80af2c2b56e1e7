// Host side of libceleste: the C ABI, argument validation, packing of ragged
// batches into device metadata (sources -> images -> work items), and the
// drivers of the evaluation and of the trust-region fits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "celeste_internal.h"

using namespace celeste;

namespace celeste {
hipError_t launch_fit_start(FitDev st, int n_src, hipStream_t s);
}

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace celeste {
void set_error(const char* msg) { g_err = msg; }
}  // namespace celeste

namespace {

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(CELESTE_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

#define CHK(x)                 \
  do {                         \
    int r_ = (x);              \
    if (r_ != CELESTE_OK) return r_; \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct celeste_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int chunk_px = 4096;
  int block = 256;
  int use_graph = 1;
  int variant = 3;   // pixel-kernel variant (register budget / unrolling), see CELESTE_OPT_VARIANT
  int tile_log2 = 3;     // log2 tile width of the value+gradient+Hessian kernel
  float e_zero = -160.f; // exact-zero threshold of the pixel kernels (log2 density)
  bool exp2_flushes = false;   // the device's exp2 returns 0 below 2^-126 (checked at creation)
  int vblock = 256;      // value kernel block size
  int vtile_log2 = 3;    // log2 tile width of the value kernel
  DevBuf imgs, items, srcs, tables, partials, img_const, staging, theta, o_elbo, o_grad, o_hess, flag;
  DevBuf st_buf;   // all trust-region state in one allocation
  DevBuf ctr;      // device counters: pixel evaluations [full, value, grad], subproblem paths and work [3..8]
  int profile = 0;
  celeste_stats stats{};

  celeste_net* net = nullptr;   // surrogate network (not owned)
  DevBuf sur;                   // surrogate predictions (float, S x 27)
  DevBuf tile_off, tile_img, img_field, nbr_off;   // crowded-field index buffers
  DevBuf tables2, fsky;                            // second setup table (field updates), field skies
  DevBuf kept;                                     // first rows of the kept blocks of a pixel subsample
  DevBuf lr_in, lr_cov, lr_status, lr_eval;        // linear-response covariance staging
  DevBuf lfact;                                    // log n! table of the pixel constants
  DevBuf lb_buf;                                   // L-BFGS state beyond the fit state
  DevBuf imgs_s, items_s, srcs_s, partials_s;      // the pixel-subsampled pack of a fit's early phase
  int persistent = -1;                             // fits: persistent pixel-kernel blocks per CU (0: off,
                                                   // -1: as many as the kernel instance keeps resident)
  int pgrid = 0;                                   // the current fit's persistent grid (blocks)
  int tr_chol = 1;                                 // fits: subproblem by Cholesky where -H is positive definite
  int fp64_sums = 0;                               // value+gradient+Hessian kernel: FP64 sums per tile step
  int trial_derivs = 1;                            // fits: gradient and Hessian evaluated at the trial point
  int n_cu = 0;                                    // compute units of the device
  DevBuf qbuf;                                     // the fits' device work queue
  bool lfact_ready = false;
  DevBuf h_imgs, h_items, h_srcs;                  // pinned host staging of the packed metadata
};

namespace {
// The value+gradient+Hessian kernel's variant with the context's summation precision (bit 3).
int full_variant(const celeste_ctx* c) { return c->variant | (c->fp64_sums ? 8 : 0); }
}  // namespace

namespace celeste {
int ctx_device(const celeste_ctx* c) { return c->device; }
hipStream_t ctx_stream(const celeste_ctx* c) { return c->stream; }
}  // namespace celeste

namespace {

int ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (bytes <= b.cap) return CELESTE_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(CELESTE_E_NOMEM, "device allocation of %zu bytes failed", bytes);
  }
  b.cap = bytes;
  return CELESTE_OK;
}

// Pinned host buffer of at least `bytes` (contents not kept on growth).
int ensure_host(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (bytes <= b.cap) return CELESTE_OK;
  const size_t cap = std::max(bytes, b.cap + b.cap / 2);
  if (b.p) (void)hipHostFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  if (hipHostMalloc(&b.p, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(CELESTE_E_NOMEM, "pinned host allocation of %zu bytes failed", cap);
  }
  b.cap = cap;
  return CELESTE_OK;
}

template <class T>
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

bool finite(double x) { return std::isfinite(x); }

// Cholesky of a symmetric 4x4; false if not positive definite.
bool chol4(const double A[4][4], double L[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 4; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 4; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  return true;
}

int make_prior(const celeste_prior* p, PriorDev* d) {
  if (!p) return fail(CELESTE_E_INVALID, "prior is NULL");
  if (!(p->p_star > 0.0 && p->p_star < 1.0)) return fail(CELESTE_E_INVALID, "prior p_star must lie in (0,1)");
  std::memset(d, 0, sizeof(*d));
  d->p_star = p->p_star;
  for (int t = 0; t < 2; ++t) {
    if (!finite(p->r_mean[t]) || !(p->r_var[t] > 0.0) || !finite(p->r_var[t]))
      return fail(CELESTE_E_INVALID, "prior r_mean/r_var[%d] invalid", t);
    d->r_mean[t] = p->r_mean[t];
    d->r_var[t] = p->r_var[t];
    for (int j = 0; j < 4; ++j) {
      if (!finite(p->c_mean[t][j])) return fail(CELESTE_E_INVALID, "prior c_mean not finite");
      d->c_mean[t][j] = p->c_mean[t][j];
      d->c_diag[t][j] = p->c_cov[t][j][j];
      for (int k = 0; k < 4; ++k)
        if (!finite(p->c_cov[t][j][k]) || p->c_cov[t][j][k] != p->c_cov[t][k][j])
          return fail(CELESTE_E_INVALID, "prior c_cov[%d] must be finite and symmetric", t);
    }
    double L[4][4];
    if (!chol4(p->c_cov[t], L)) return fail(CELESTE_E_INVALID, "prior c_cov[%d] not positive definite", t);
    double ld = 0.0;
    for (int j = 0; j < 4; ++j) ld += 2.0 * std::log(L[j][j]);
    d->c_logdet[t] = ld;
    // inverse from the Cholesky factor: solve L L^T X = I
    for (int c = 0; c < 4; ++c) {
      double y[4], x[4];
      for (int i = 0; i < 4; ++i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
      }
      for (int i = 3; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < 4; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
      }
      for (int i = 0; i < 4; ++i) d->c_inv[t][i][c] = x[i];
    }
  }
  return CELESTE_OK;
}

int make_profiles(const celeste_profiles* p, ProfDev* d) {
  if (!p) return fail(CELESTE_E_INVALID, "profiles is NULL");
  if (p->n_exp < 1 || p->n_exp > CELESTE_MAX_PROTO || p->n_dev < 1 || p->n_dev > CELESTE_MAX_PROTO)
    return fail(CELESTE_E_INVALID, "profile component counts must be in 1..%d", CELESTE_MAX_PROTO);
  std::memset(d, 0, sizeof(*d));
  d->n_exp = p->n_exp;
  d->n_dev = p->n_dev;
  for (int j = 0; j < p->n_exp; ++j) {
    if (!(p->exp_amp[j] >= 0.0) || !finite(p->exp_amp[j]) || !(p->exp_var[j] > 0.0) || !finite(p->exp_var[j]))
      return fail(CELESTE_E_INVALID, "exp profile component %d invalid", j);
    d->amp[j] = p->exp_amp[j];
    d->var[j] = p->exp_var[j];
  }
  for (int j = 0; j < p->n_dev; ++j) {
    if (!(p->dev_amp[j] >= 0.0) || !finite(p->dev_amp[j]) || !(p->dev_var[j] > 0.0) || !finite(p->dev_var[j]))
      return fail(CELESTE_E_INVALID, "dev profile component %d invalid", j);
    d->amp[p->n_exp + j] = p->dev_amp[j];
    d->var[p->n_exp + j] = p->dev_var[j];
  }
  return CELESTE_OK;
}

int check_image(const celeste_image& im, int64_t idx) {
  if (im.band < 0 || im.band > 4) return fail(CELESTE_E_INVALID, "image %lld: band %d not in 0..4", (long long)idx, im.band);
  if (im.h < 1 || im.w < 1 || im.pitch < im.w)
    return fail(CELESTE_E_INVALID, "image %lld: bad shape h=%d w=%d pitch=%d", (long long)idx, im.h, im.w, im.pitch);
  if ((int64_t)im.h * im.w > (int64_t)1 << 30) return fail(CELESTE_E_INVALID, "image %lld: patch too large", (long long)idx);
  if (im.n_psf < 1 || im.n_psf > CELESTE_MAX_PSF)
    return fail(CELESTE_E_INVALID, "image %lld: n_psf %d not in 1..%d", (long long)idx, im.n_psf, CELESTE_MAX_PSF);
  if (im.nbr_pitch != 0 && im.nbr_pitch < im.w)
    return fail(CELESTE_E_INVALID, "image %lld: nbr_pitch must be 0 or >= w", (long long)idx);
  if (!im.pixels) return fail(CELESTE_E_INVALID, "image %lld: pixels is NULL", (long long)idx);
  if (!(im.sky > 0.0) || !finite(im.sky) || !(im.calib > 0.0) || !finite(im.calib))
    return fail(CELESTE_E_INVALID, "image %lld: sky and calib must be positive and finite", (long long)idx);
  for (int k = 0; k < 2; ++k)
    if (!finite(im.origin[k])) return fail(CELESTE_E_INVALID, "image %lld: origin not finite", (long long)idx);
  for (int k = 0; k < 6; ++k)
    if (!finite(im.wcs[k])) return fail(CELESTE_E_INVALID, "image %lld: wcs not finite", (long long)idx);
  if (std::fabs(im.wcs[0] * im.wcs[3] - im.wcs[1] * im.wcs[2]) < 1e-12)
    return fail(CELESTE_E_INVALID, "image %lld: singular WCS matrix", (long long)idx);
  for (int k = 0; k < im.n_psf; ++k) {
    const double* p = im.psf[k];
    for (int j = 0; j < 6; ++j)
      if (!finite(p[j])) return fail(CELESTE_E_INVALID, "image %lld: psf not finite", (long long)idx);
    if (!(p[0] >= 0.0) || !(p[3] > 0.0) || !(p[5] > 0.0) || !(p[3] * p[5] - p[4] * p[4] > 0.0))
      return fail(CELESTE_E_INVALID, "image %lld: psf component %d needs weight >= 0 and a PD covariance",
                  (long long)idx, k);
  }
  return CELESTE_OK;
}

int check_theta(const double* th, int64_t s) {
  for (int i = 0; i < NP; ++i)
    if (!finite(th[i])) return fail(CELESTE_E_INVALID, "theta[%lld][%d] not finite", (long long)s, i);
  if (!(th[2] > 0.0 && th[2] < 1.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: a must lie in (0,1)", (long long)s);
  if (!(th[3] >= 0.0 && th[3] <= 1.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: e_dev must lie in [0,1]", (long long)s);
  if (!(th[4] > 0.0 && th[4] <= 1.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: e_axis must lie in (0,1]", (long long)s);
  if (!(th[6] > 0.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: e_scale must be > 0", (long long)s);
  for (int i : {9, 10})
    if (!(th[i] > 0.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: r2 must be > 0", (long long)s);
  for (int i = 19; i < NP; ++i)
    if (!(th[i] > 0.0)) return fail(CELESTE_E_INVALID, "theta[%lld]: c2 must be > 0", (long long)s);
  return CELESTE_OK;
}

// Host-side packed metadata; the arrays live in the context's pinned staging buffers (valid
// until the context packs the next batch).
// Host storage of the packed metadata from the process heap (the no-allocation entry point),
// instead of the context's pinned buffers.
struct HostPack {
  std::vector<ImgDev> imgs;
  std::vector<WorkItem> items;
  std::vector<SrcDev> srcs;
};

struct Packed {
  ImgDev* imgs = nullptr;
  WorkItem* items = nullptr;
  SrcDev* srcs = nullptr;
  PriorDev prior;
  ProfDev prof;
  int tstride = 0;
  int n_src = 0, n_img = 0, n_items = 0;
};

// fn(begin, end) over [0, n) in contiguous slices on up to 16 host threads (serial when small).
template <class F>
void parallel_for(int64_t n, F fn) {
  const int64_t per_thread_min = 8192;
  int nt = (int)std::min<int64_t>(16, std::max<int64_t>(1, n / per_thread_min));
  nt = std::min<int>(nt, std::max(1u, std::thread::hardware_concurrency()));
  if (nt <= 1) {
    fn((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(fn, n * t / nt, n * (t + 1) / nt);
  for (auto& x : th) x.join();
}

int items_of(const celeste_image& im, int chunk) {
  // bands of whole 8-row tile rows holding about `chunk` pixels
  const int band = std::max(TILE, (chunk / std::max(1, im.w)) / TILE * TILE);
  return (im.h + band - 1) / band;
}

int validate_and_pack(celeste_ctx* ctx, const celeste_batch* b, Packed* P, HostPack* hp = nullptr) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  if (!b) return fail(CELESTE_E_INVALID, "batch is NULL");
  if (b->n_sources < 1) return fail(CELESTE_E_INVALID, "n_sources must be >= 1");
  if (b->mem_kind != CELESTE_MEM_HOST && b->mem_kind != CELESTE_MEM_DEVICE)
    return fail(CELESTE_E_INVALID, "mem_kind must be CELESTE_MEM_HOST or CELESTE_MEM_DEVICE");
  if (!b->image_offsets || !b->images) return fail(CELESTE_E_INVALID, "image_offsets/images is NULL");
  if (b->image_offsets[0] != 0) return fail(CELESTE_E_INVALID, "image_offsets[0] must be 0");
  for (int s = 0; s < b->n_sources; ++s) {
    if (b->image_offsets[s + 1] < b->image_offsets[s])
      return fail(CELESTE_E_INVALID, "image_offsets must be non-decreasing");
    if (b->image_offsets[s + 1] == b->image_offsets[s])
      return fail(CELESTE_E_INVALID, "source %d has no images", s);
  }
  const int64_t n_img = b->image_offsets[b->n_sources];
  if (n_img > (int64_t)1 << 30) return fail(CELESTE_E_INVALID, "too many images");
  CHK(make_prior(b->prior, &P->prior));
  CHK(make_profiles(b->profiles, &P->prof));
  // image checks in parallel; the message comes from re-checking the first bad image here
  const int nslot = 16;
  std::vector<int64_t> first_bad(nslot, INT64_MAX);
  std::vector<int> slot_psf(nslot, 1);
  {
    parallel_for(n_img, [&](int64_t i0, int64_t i1) {
      const int slot = (int)((i0 * nslot) / std::max<int64_t>(1, n_img));
      int64_t bad = INT64_MAX;
      int mp = 1;
      for (int64_t i = i0; i < i1; ++i) {
        if (check_image(b->images[i], i) != CELESTE_OK) {
          bad = i;
          break;
        }
        mp = std::max(mp, b->images[i].n_psf);
      }
      first_bad[slot] = std::min(first_bad[slot], bad);
      slot_psf[slot] = std::max(slot_psf[slot], mp);
    });
  }
  const int64_t bad = *std::min_element(first_bad.begin(), first_bad.end());
  if (bad != INT64_MAX) return check_image(b->images[bad], bad);
  const int max_psf = *std::max_element(slot_psf.begin(), slot_psf.end());
  P->tstride = table_stride(max_psf, P->prof.n_exp, P->prof.n_dev);
  P->n_src = b->n_sources;
  P->n_img = (int)n_img;
  if (hp) {
    hp->imgs.resize((size_t)n_img);
    hp->srcs.resize((size_t)b->n_sources);
    P->imgs = hp->imgs.data();
    P->srcs = hp->srcs.data();
  } else {
    CHK(ensure_host(ctx->h_imgs, sizeof(ImgDev) * n_img));
    CHK(ensure_host(ctx->h_srcs, sizeof(SrcDev) * b->n_sources));
    P->imgs = as<ImgDev>(ctx->h_imgs);
    P->srcs = as<SrcDev>(ctx->h_srcs);
  }
  const int chunk = std::max(64, ctx->chunk_px);
  // work-item offsets per image (items in image order, so per source contiguous)
  std::vector<int64_t> first_item(n_img + 1, 0);
  for (int64_t i = 0; i < n_img; ++i) first_item[i + 1] = first_item[i] + items_of(b->images[i], chunk);
  if (first_item[n_img] > (int64_t)INT32_MAX / 2) return fail(CELESTE_E_INVALID, "too many work items");
  if (hp) {
    hp->items.resize((size_t)first_item[n_img]);
    P->items = hp->items.data();
  } else {
    CHK(ensure_host(ctx->h_items, sizeof(WorkItem) * first_item[n_img]));
    P->items = as<WorkItem>(ctx->h_items);
  }
  std::vector<int> src_of(n_img);
  for (int s = 0; s < b->n_sources; ++s)
    for (int64_t i = b->image_offsets[s]; i < b->image_offsets[s + 1]; ++i) src_of[i] = s;
  parallel_for(n_img, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      const celeste_image& im = b->images[i];
      const int s = src_of[i];
      ImgDev& d = P->imgs[i];
      std::memset(&d, 0, sizeof(d));
      d.pix = im.pixels;
      d.nbr_mean = im.nbr_mean;
      d.nbr_var = im.nbr_var;
      d.h = im.h;
      d.w = im.w;
      d.pitch = im.pitch;
      d.nbr_pitch = im.nbr_pitch ? im.nbr_pitch : im.pitch;
      d.band = im.band;
      d.n_psf = im.n_psf;
      d.src = s;
      d.origin[0] = im.origin[0];
      d.origin[1] = im.origin[1];
      for (int k = 0; k < 6; ++k) d.wcs[k] = im.wcs[k];
      d.sky = im.sky;
      d.calib = im.calib;
      for (int k = 0; k < CELESTE_MAX_PSF; ++k)
        for (int j = 0; j < 6; ++j) d.psf[k][j] = k < im.n_psf ? im.psf[k][j] : 0.0;
      d.item_begin = (int)first_item[i];
      d.item_end = (int)first_item[i + 1];
      const int band = std::max(TILE, (chunk / std::max(1, im.w)) / TILE * TILE);
      int64_t it = first_item[i];
      for (int r = 0; r < im.h; r += band) P->items[it++] = WorkItem{(int)i, s, r, std::min(im.h, r + band)};
    }
  });
  for (int s = 0; s < b->n_sources; ++s) {
    SrcDev sd;
    sd.img_begin = (int)b->image_offsets[s];
    sd.img_end = (int)b->image_offsets[s + 1];
    sd.item_begin = (int)first_item[sd.img_begin];
    sd.item_end = (int)first_item[sd.img_end];
    sd.npix = 0;
    for (int64_t i = sd.img_begin; i < sd.img_end; ++i) sd.npix += (int64_t)b->images[i].h * b->images[i].w;
    P->srcs[s] = sd;
  }
  P->n_items = (int)first_item[n_img];
  return CELESTE_OK;
}

// Pixel subsample: the work items are rebuilt over the kept 8-row blocks only.  kept_rows
// receives the first row of every kept block (image by image, in row order); an item takes
// up to a band's worth of one image's consecutive list entries (the blocks need not be
// adjacent), and its [row_begin, row_end) indexes kept_rows.  The item ranges of the images
// and sources and the sources' pixel counts follow.  keep / keep_off: host arrays.
int subsample_items(celeste_ctx* ctx, const celeste_batch* b, Packed* P, const uint8_t* keep,
                    const int64_t* keep_off, std::vector<int>& kept_rows) {
  if (keep_off[0] != 0) return fail(CELESTE_E_INVALID, "keep_off[0] must be 0");
  for (int i = 0; i < P->n_img; ++i)
    if (keep_off[i + 1] - keep_off[i] != (b->images[i].h + 7) / 8)
      return fail(CELESTE_E_INVALID, "image %d: keep_off must give (h + 7) / 8 blocks", i);
  const int chunk = std::max(64, ctx->chunk_px);
  std::vector<WorkItem> items;
  std::vector<int64_t> kept_px(P->n_img, 0);
  kept_rows.clear();
  for (int i = 0; i < P->n_img; ++i) {
    const celeste_image& im = b->images[i];
    const uint8_t* k = keep + keep_off[i];
    const int nb = (im.h + 7) / 8;
    const int per_item = std::max(TILE, (chunk / std::max(1, im.w)) / TILE * TILE) / TILE;   // blocks
    ImgDev& d = P->imgs[i];
    const size_t first = kept_rows.size();
    for (int j = 0; j < nb; ++j)
      if (k[j]) {
        kept_rows.push_back(TILE * j);
        kept_px[i] += (int64_t)(std::min(im.h, TILE * (j + 1)) - TILE * j) * im.w;
      }
    if (kept_rows.size() > (size_t)INT32_MAX / 2) return fail(CELESTE_E_INVALID, "too many kept blocks");
    d.item_begin = (int)items.size();
    for (size_t e = first; e < kept_rows.size(); e += per_item)
      items.push_back(WorkItem{i, d.src, (int)e, (int)std::min(kept_rows.size(), e + per_item)});
    if (items.size() > (size_t)INT32_MAX / 2) return fail(CELESTE_E_INVALID, "too many work items");
    d.item_end = (int)items.size();
  }
  CHK(ensure_host(ctx->h_items, sizeof(WorkItem) * std::max<size_t>(1, items.size())));
  P->items = as<WorkItem>(ctx->h_items);
  if (!items.empty()) std::memcpy(P->items, items.data(), sizeof(WorkItem) * items.size());
  for (int s = 0; s < P->n_src; ++s) {
    SrcDev& sd = P->srcs[s];
    sd.item_begin = P->imgs[sd.img_begin].item_begin;
    sd.item_end = P->imgs[sd.img_end - 1].item_end;
    sd.npix = 0;
    for (int i = sd.img_begin; i < sd.img_end; ++i) sd.npix += kept_px[i];
  }
  P->n_items = (int)items.size();
  return CELESTE_OK;
}

// Copies host pixel arrays into one device staging buffer and repoints the images.
int stage_host_pixels(celeste_ctx* ctx, const celeste_batch* b, Packed* P, hipStream_t st) {
  size_t total = 0;
  for (int i = 0; i < P->n_img; ++i) {
    const celeste_image& im = b->images[i];
    const size_t n = (size_t)im.h * im.w;
    total += n * (1 + (im.nbr_mean ? 1 : 0) + (im.nbr_var ? 1 : 0));
  }
  std::vector<float> host(total);
  size_t off = 0;
  std::vector<size_t> offs(3 * P->n_img, (size_t)-1);
  for (int i = 0; i < P->n_img; ++i) {
    const celeste_image& im = b->images[i];
    const float* srcs[3] = {im.pixels, im.nbr_mean, im.nbr_var};
    for (int k = 0; k < 3; ++k) {
      if (!srcs[k]) continue;
      offs[3 * i + k] = off;
      const size_t rp = k == 0 ? (size_t)im.pitch : (size_t)(im.nbr_pitch ? im.nbr_pitch : im.pitch);
      for (int r = 0; r < im.h; ++r) std::memcpy(&host[off + (size_t)r * im.w], srcs[k] + (size_t)r * rp, sizeof(float) * im.w);
      off += (size_t)im.h * im.w;
    }
  }
  CHK(ensure(ctx->staging, total * sizeof(float)));
  HIPCHK(hipMemcpyAsync(ctx->staging.p, host.data(), total * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  float* base = as<float>(ctx->staging);
  for (int i = 0; i < P->n_img; ++i) {
    ImgDev& d = P->imgs[i];
    d.pitch = d.w;
    d.nbr_pitch = d.w;
    d.pix = base + offs[3 * i];
    d.nbr_mean = offs[3 * i + 1] != (size_t)-1 ? base + offs[3 * i + 1] : nullptr;
    d.nbr_var = offs[3 * i + 2] != (size_t)-1 ? base + offs[3 * i + 2] : nullptr;
  }
  return CELESTE_OK;
}

// Device buffers of one evaluation: packed metadata, setup tables, per-item partial sums,
// per-image constants, the pixel-check flag and the log n! table.
struct EvalBufs {
  ImgDev* imgs = nullptr;
  WorkItem* items = nullptr;
  SrcDev* srcs = nullptr;
  double* img_const = nullptr;
  float* tables = nullptr;
  double* partials = nullptr;
  int* flag = nullptr;
  double* lfact = nullptr;
  bool lfact_ready = false;   // the table holds its values (else it is filled before use)
};

// The context's own buffers, grown to the batch.
int ctx_bufs(celeste_ctx* ctx, const Packed* P, EvalBufs* B) {
  CHK(ensure(ctx->imgs, sizeof(ImgDev) * P->n_img));
  CHK(ensure(ctx->items, sizeof(WorkItem) * P->n_items));
  CHK(ensure(ctx->srcs, sizeof(SrcDev) * P->n_src));
  CHK(ensure(ctx->img_const, sizeof(double) * P->n_img));
  CHK(ensure(ctx->tables, sizeof(float) * (size_t)P->tstride * P->n_img));
  CHK(ensure(ctx->partials, sizeof(double) * (size_t)NACC * P->n_items));
  CHK(ensure(ctx->flag, sizeof(int) * 4));
  if (!ctx->lfact_ready) CHK(ensure(ctx->lfact, sizeof(double) * LFACT_N));
  B->imgs = as<ImgDev>(ctx->imgs);
  B->items = as<WorkItem>(ctx->items);
  B->srcs = as<SrcDev>(ctx->srcs);
  B->img_const = as<double>(ctx->img_const);
  B->tables = as<float>(ctx->tables);
  B->partials = as<double>(ctx->partials);
  B->flag = as<int>(ctx->flag);
  B->lfact = as<double>(ctx->lfact);
  B->lfact_ready = ctx->lfact_ready;
  return CELESTE_OK;
}

// Metadata upload + pixel validation + per-image constants (the last two only when the
// call reads pixels) into the buffers B.  Synchronous.  Host batches are staged in the
// context's staging buffer first.
int prepare_in(celeste_ctx* ctx, const celeste_batch* b, Packed* P, EvalBufs* B, hipStream_t st, bool pixels) {
  if (b->mem_kind == CELESTE_MEM_HOST) CHK(stage_host_pixels(ctx, b, P, st));
  HIPCHK(hipMemcpyAsync(B->imgs, P->imgs, sizeof(ImgDev) * P->n_img, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(B->items, P->items, sizeof(WorkItem) * P->n_items, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(B->srcs, P->srcs, sizeof(SrcDev) * P->n_src, hipMemcpyHostToDevice, st));
  if (!pixels) {
    HIPCHK(hipStreamSynchronize(st));
    return CELESTE_OK;
  }
  if (!B->lfact_ready) {
    HIPCHK(launch_lfact(B->lfact, st));
    B->lfact_ready = true;   // complete before first use: the check below synchronises the stream
  }
  HIPCHK(launch_zero_int(B->flag, 4, st));
  HIPCHK(launch_check_const(B->imgs, P->n_img, B->lfact, B->img_const, B->flag, st));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, B->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) return fail(CELESTE_E_INVALID, "pixel or neighbour arrays hold negative or non-finite values");
  return CELESTE_OK;
}

// prepare_in on the context's own buffers.
int prepare(celeste_ctx* ctx, const celeste_batch* b, Packed* P, hipStream_t st, bool pixels = true) {
  EvalBufs B;
  CHK(ctx_bufs(ctx, P, &B));
  const int rc = prepare_in(ctx, b, P, &B, st, pixels);
  ctx->lfact_ready = ctx->lfact_ready || B.lfact_ready;
  return rc;
}

hipStream_t pick(celeste_ctx* ctx, void* stream) { return stream ? (hipStream_t)stream : ctx->stream; }

unsigned long long* ctr_full(celeste_ctx* c) { return as<unsigned long long>(c->ctr); }
unsigned long long* ctr_value(celeste_ctx* c) { return as<unsigned long long>(c->ctr) + 1; }
unsigned long long* ctr_grad(celeste_ctx* c) { return as<unsigned long long>(c->ctr) + 2; }
// counters [3, 9) belong to the trust-region subproblem (FitParams::tr_ctr)
unsigned long long* ctr_trial(celeste_ctx* c) { return as<unsigned long long>(c->ctr) + 9; }
unsigned long long* ctr_taken(celeste_ctx* c) { return as<unsigned long long>(c->ctr) + 10; }
constexpr int N_CTR = 11;

// HIP events between the kernel phases of one iteration (profile mode).
struct PhaseTimer {
  bool on = false;
  hipEvent_t ev[9] = {};
  int init(bool enable) {
    on = enable;
    if (!on) return CELESTE_OK;
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    return CELESTE_OK;
  }
  ~PhaseTimer() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int k, hipStream_t st) {
    if (on) (void)hipEventRecord(ev[k], st);
  }
  float span(int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms;
  }
};

int eval_impl(celeste_ctx* ctx, const celeste_batch* b, const double* theta, double* elbo, double* grad,
              double* hess, void* stream, const uint8_t* keep, const int64_t* keep_off, double keep_prob,
              bool noalloc = false);
int scratch_init(int device);

}  // namespace

// =============================================================================== ABI

extern "C" {

const char* celeste_last_error(void) { return g_err.c_str(); }

void celeste_fit_opts_default(celeste_fit_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iter = 50;
  o->init_mode = CELESTE_INIT_AS_GIVEN;
  o->pred_rtol = 1e-8;
  o->curv_tol = 1e-8;
  o->delta0 = 1.0;
  o->delta_max = 100.0;
  o->delta_min = 1e-10;
  o->eta = 0.1;
  o->u_box = 3.0;
  o->poll_every = 4;
}

int celeste_ctx_create(int hip_device, celeste_ctx** out) {
  if (!out) return fail(CELESTE_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(CELESTE_E_INVALID, "device %d not in 0..%d", hip_device, n - 1);
  HIPCHK(hipSetDevice(hip_device));
  celeste_ctx* c = new (std::nothrow) celeste_ctx();
  if (!c) return fail(CELESTE_E_NOMEM, "context allocation failed");
  c->device = hip_device;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
      c->n_cu < 1)
    c->n_cu = 256;
  if (scratch_init(hip_device) != CELESTE_OK) {   // device address of the no-allocation scratch
    delete c;
    return CELESTE_E_DEVICE;
  }
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(CELESTE_E_DEVICE, "stream creation failed");
  }
  if (ensure(c->ctr, N_CTR * sizeof(unsigned long long)) != CELESTE_OK ||
      hipMemset(c->ctr.p, 0, N_CTR * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipStreamDestroy(c->stream);
    if (c->ctr.p) (void)hipFree(c->ctr.p);
    delete c;
    return fail(CELESTE_E_DEVICE, "counter allocation failed");
  }
  {
    // Exact-zero threshold: where the device's exp2 returns exactly 0 below 2^-126 (results
    // that would be subnormal are flushed), a component whose log2 density is below -127 on a
    // whole tile contributes exactly 0 and the threshold is -127; otherwise -160 (below the
    // smallest subnormal).
    const float in[4] = {-126.5f, -127.0f, -135.0f, -149.5f};
    float res[4] = {1.f, 1.f, 1.f, 1.f};
    DevBuf pb;
    if (ensure(pb, sizeof(in) * 2) == CELESTE_OK) {
      float* d = as<float>(pb);
      if (hipMemcpy(d, in, sizeof(in), hipMemcpyHostToDevice) == hipSuccess &&
          launch_exp2_probe(d, d + 4, 4, c->stream) == hipSuccess &&
          hipMemcpyAsync(res, d + 4, sizeof(res), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
          hipStreamSynchronize(c->stream) == hipSuccess)
        c->exp2_flushes = res[0] == 0.f && res[1] == 0.f && res[2] == 0.f && res[3] == 0.f;
      c->e_zero = c->exp2_flushes ? -127.f : -160.f;
      (void)hipFree(pb.p);
    }
  }
  *out = c;
  return CELESTE_OK;
}

int celeste_ctx_get_stats(celeste_ctx* c, celeste_stats* out, int reset) {
  if (!c || !out) return fail(CELESTE_E_INVALID, "context and out must not be NULL");
  HIPCHK(hipSetDevice(c->device));
  unsigned long long h[N_CTR] = {};
  HIPCHK(hipMemcpy(h, c->ctr.p, sizeof(h), hipMemcpyDeviceToHost));
  c->stats.full_px = (int64_t)(h[0] + h[9]);
  c->stats.trial_full_px = (int64_t)h[9];
  c->stats.taken_px = (int64_t)h[10];
  c->stats.value_px = (int64_t)h[1];
  c->stats.grad_px = (int64_t)h[2];
  c->stats.tr_interior = (int64_t)h[3];
  c->stats.tr_boundary = (int64_t)h[4];
  c->stats.tr_eigen = (int64_t)h[5];
  c->stats.tr_sweeps = (int64_t)h[6];
  c->stats.tr_sweep_cap = (int64_t)h[7];
  c->stats.tr_newton_steps = (int64_t)h[8];
  *out = c->stats;
  if (reset) {
    HIPCHK(hipMemset(c->ctr.p, 0, sizeof(h)));
    c->stats = celeste_stats{};
  }
  return CELESTE_OK;
}

void celeste_ctx_destroy(celeste_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->imgs, &c->items, &c->srcs, &c->tables, &c->partials, &c->img_const, &c->staging,
                    &c->theta, &c->o_elbo, &c->o_grad, &c->o_hess, &c->flag, &c->st_buf, &c->ctr, &c->sur,
                    &c->tile_off, &c->tile_img, &c->img_field, &c->nbr_off, &c->tables2, &c->fsky,
                    &c->kept, &c->lr_in, &c->lr_cov, &c->lr_status, &c->lr_eval,
                    &c->lfact, &c->lb_buf, &c->imgs_s, &c->items_s, &c->srcs_s, &c->partials_s, &c->qbuf};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (DevBuf* b : {&c->h_imgs, &c->h_items, &c->h_srcs})
    if (b->p) (void)hipHostFree(b->p);
  (void)hipStreamDestroy(c->stream);
  delete c;
}

int celeste_ctx_set_option(celeste_ctx* c, int option, int64_t value) {
  if (!c) return fail(CELESTE_E_INVALID, "context is NULL");
  switch (option) {
    case CELESTE_OPT_CHUNK_PX:
      if (value < 64 || value > (1 << 24)) return fail(CELESTE_E_INVALID, "chunk_px must be in 64..2^24");
      c->chunk_px = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_BLOCK:
      if (value != 128 && value != 256) return fail(CELESTE_E_INVALID, "block must be 128 or 256");
      c->block = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_USE_GRAPH:
      c->use_graph = value ? 1 : 0;
      return CELESTE_OK;
    case CELESTE_OPT_PROFILE:
      c->profile = value ? 1 : 0;
      return CELESTE_OK;
    case CELESTE_OPT_VARIANT:
      if (value < 0 || value > 7) return fail(CELESTE_E_INVALID, "variant must be in 0..7");
      c->variant = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_TILE_W:
    case CELESTE_OPT_VALUE_TILE_W: {
      int l = -1;
      for (int k = 3; k <= 6; ++k)
        if (value == (1 << k)) l = k;
      if (l < 0) return fail(CELESTE_E_INVALID, "tile width must be 8, 16, 32 or 64");
      (option == CELESTE_OPT_TILE_W ? c->tile_log2 : c->vtile_log2) = l;
      return CELESTE_OK;
    }
    case CELESTE_OPT_VALUE_BLOCK:
      if (value != 128 && value != 256) return fail(CELESTE_E_INVALID, "value block must be 128 or 256");
      c->vblock = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_PERSISTENT:
      if (value < -1 || value > 16)
        return fail(CELESTE_E_INVALID, "persistent blocks per compute unit must be -1..16");
      c->persistent = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_FP64_SUMS:
      if (value != 0 && value != 1) return fail(CELESTE_E_INVALID, "FP64 sums must be 0 or 1");
      c->fp64_sums = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_TRIAL_DERIVATIVES:
      if (value != 0 && value != 1) return fail(CELESTE_E_INVALID, "trial derivatives must be 0 or 1");
      c->trial_derivs = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_TR_CHOLESKY:
      if (value != 0 && value != 1) return fail(CELESTE_E_INVALID, "trust-region Cholesky path must be 0 or 1");
      c->tr_chol = (int)value;
      return CELESTE_OK;
    case CELESTE_OPT_EXACT_ZERO:
      if (value != 0 && value != 1 && value != 127 && value != 160)
        return fail(CELESTE_E_INVALID, "exact-zero threshold must be 0, 1, 127 or 160");
      if (value == 127 && !c->exp2_flushes)
        return fail(CELESTE_E_UNSUPPORTED, "this device's exp2 does not flush results below 2^-126");
      if (value == 1)
        c->e_zero = -INFINITY;   // every skip test (log2 density >= threshold) passes: nothing is skipped
      else
        c->e_zero = value == 160 || (value == 0 && !c->exp2_flushes) ? -160.f : -127.f;
      return CELESTE_OK;
    default:
      return fail(CELESTE_E_INVALID, "unknown option %d", option);
  }
}

size_t celeste_struct_size(int which) {
  switch (which) {
    case 0: return sizeof(celeste_image);
    case 1: return sizeof(celeste_prior);
    case 2: return sizeof(celeste_profiles);
    case 3: return sizeof(celeste_batch);
    case 4: return sizeof(celeste_fit_opts);
    case 5: return sizeof(celeste_fit_result);
    case 6: return sizeof(celeste_stats);
    case 7: return sizeof(celeste_tune_result);
    case 8: return sizeof(celeste_lbfgs_opts);
    default: return 0;
  }
}

int celeste_elbo_eval(celeste_ctx* ctx, const celeste_batch* b, const double* theta, double* elbo, double* grad,
                      double* hess, void* stream) {
  return eval_impl(ctx, b, theta, elbo, grad, hess, stream, nullptr, nullptr, 1.0);
}

int celeste_elbo_eval_noalloc(celeste_ctx* ctx, const celeste_batch* b, const double* theta, double* elbo,
                              double* grad, double* hess, void* stream) {
  return eval_impl(ctx, b, theta, elbo, grad, hess, stream, nullptr, nullptr, 1.0, true);
}

int celeste_elbo_eval_sampled(celeste_ctx* ctx, const celeste_batch* b, const double* theta, const uint8_t* keep,
                              const int64_t* keep_off, double keep_prob, double* elbo, double* grad, double* hess,
                              void* stream) {
  if (!keep || !keep_off) return fail(CELESTE_E_INVALID, "keep and keep_off must not be NULL");
  if (!(keep_prob > 0.0 && keep_prob <= 1.0)) return fail(CELESTE_E_INVALID, "keep_prob must be in (0, 1]");
  return eval_impl(ctx, b, theta, elbo, grad, hess, stream, keep, keep_off, keep_prob);
}

int celeste_lr_covariance_from_hessian(celeste_ctx* ctx, int64_t n, int mem_kind, const double* theta,
                                       const double* u0, double u_box, const double* grad, const double* hess,
                                       double* cov, int32_t* status, void* stream) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  if (n < 0 || n > (int64_t)INT32_MAX / 2) return fail(CELESTE_E_INVALID, "n out of range");
  if (mem_kind != CELESTE_MEM_HOST && mem_kind != CELESTE_MEM_DEVICE)
    return fail(CELESTE_E_INVALID, "mem_kind must be CELESTE_MEM_HOST or CELESTE_MEM_DEVICE");
  if (!theta || !u0 || !grad || !hess || !cov || !status) return fail(CELESTE_E_INVALID, "NULL argument");
  if (!(u_box > 0.0) || !std::isfinite(u_box)) return fail(CELESTE_E_INVALID, "u_box must be finite and > 0");
  if (n == 0) return CELESTE_OK;
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = pick(ctx, stream);
  const size_t S = (size_t)n;
  const double *d_th = theta, *d_u0 = u0, *d_g = grad, *d_h = hess;
  double* d_cov = cov;
  if (mem_kind == CELESTE_MEM_HOST) {
    CHK(ensure(ctx->lr_in, sizeof(double) * S * (NP + 2 + NP + NP * NP)));
    double* base = as<double>(ctx->lr_in);
    double *th = base, *uu = th + S * NP, *gg = uu + S * 2, *hh = gg + S * NP;
    HIPCHK(hipMemcpyAsync(th, theta, sizeof(double) * S * NP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(uu, u0, sizeof(double) * S * 2, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(gg, grad, sizeof(double) * S * NP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(hh, hess, sizeof(double) * S * NP * NP, hipMemcpyHostToDevice, st));
    d_th = th;
    d_u0 = uu;
    d_g = gg;
    d_h = hh;
    CHK(ensure(ctx->lr_cov, sizeof(double) * S * NP * NP));
    d_cov = as<double>(ctx->lr_cov);
  }
  CHK(ensure(ctx->lr_status, sizeof(int) * S));
  PhaseTimer T;
  CHK(T.init(ctx->profile != 0));
  T.mark(0, st);
  HIPCHK(launch_lr_cov(d_th, d_u0, u_box, d_g, d_h, (int)S, d_cov, as<int>(ctx->lr_status), st));
  T.mark(1, st);
  if (mem_kind == CELESTE_MEM_HOST)
    HIPCHK(hipMemcpyAsync(cov, d_cov, sizeof(double) * S * NP * NP, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(status, ctx->lr_status.p, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  ctx->stats.lr_launches += 1;
  if (T.on) ctx->stats.ms_lr += T.span(0, 1);
  return CELESTE_OK;
}

int celeste_lr_covariance(celeste_ctx* ctx, const celeste_batch* b, const double* theta, const double* u0,
                          double u_box, double* cov, int32_t* status, void* stream) {
  if (!ctx || !b) return fail(CELESTE_E_INVALID, "context or batch is NULL");
  if (!theta || !u0 || !cov || !status) return fail(CELESTE_E_INVALID, "NULL argument");
  if (b->n_sources < 1) return fail(CELESTE_E_INVALID, "n_sources must be >= 1");
  if (!(u_box > 0.0) || !std::isfinite(u_box)) return fail(CELESTE_E_INVALID, "u_box must be finite and > 0");
  const size_t S = (size_t)b->n_sources;
  if (b->mem_kind == CELESTE_MEM_HOST) {
    std::vector<double> e(S), g(S * NP), h(S * NP * NP);
    CHK(eval_impl(ctx, b, theta, e.data(), g.data(), h.data(), stream, nullptr, nullptr, 1.0));
    return celeste_lr_covariance_from_hessian(ctx, (int64_t)S, CELESTE_MEM_HOST, theta, u0, u_box, g.data(),
                                              h.data(), cov, status, stream);
  }
  CHK(ensure(ctx->lr_eval, sizeof(double) * S * (1 + NP + NP * NP)));
  double* e = as<double>(ctx->lr_eval);
  double* g = e + S;
  double* h = g + S * NP;
  CHK(eval_impl(ctx, b, theta, e, g, h, stream, nullptr, nullptr, 1.0));
  return celeste_lr_covariance_from_hessian(ctx, (int64_t)S, CELESTE_MEM_DEVICE, theta, u0, u_box, g, h, cov, status,
                                            stream);
}

}  // extern "C"

namespace {

int scratch_bufs(celeste_ctx* ctx, const Packed* P, int per_item, EvalBufs* B);
void scratch_lfact_filled(int device);

int eval_impl(celeste_ctx* ctx, const celeste_batch* b, const double* theta, double* elbo, double* grad,
              double* hess, void* stream, const uint8_t* keep, const int64_t* keep_off, double keep_prob,
              bool noalloc) {
  Packed P;
  HostPack hp;
  CHK(validate_and_pack(ctx, b, &P, noalloc ? &hp : nullptr));
  if (!theta || !elbo) return fail(CELESTE_E_INVALID, "theta and elbo must not be NULL");
  if (hess && !grad) return fail(CELESTE_E_INVALID, "hess requires grad");
  if (noalloc && b->mem_kind != CELESTE_MEM_DEVICE)
    return fail(CELESTE_E_INVALID, "the no-allocation evaluation takes device batches only (mem_kind DEVICE)");
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = pick(ctx, stream);
  const size_t S = P.n_src;
  std::vector<double> th_host;
  const double* th_dev = theta;
  if (b->mem_kind == CELESTE_MEM_HOST) {
    for (size_t s = 0; s < S; ++s) CHK(check_theta(theta + s * NP, (int64_t)s));
    CHK(ensure(ctx->theta, sizeof(double) * NP * S));
    HIPCHK(hipMemcpyAsync(ctx->theta.p, theta, sizeof(double) * NP * S, hipMemcpyHostToDevice, st));
    th_dev = as<double>(ctx->theta);
  } else {
    th_host.resize(NP * S);
    HIPCHK(hipMemcpyAsync(th_host.data(), theta, sizeof(double) * NP * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t s = 0; s < S; ++s) CHK(check_theta(th_host.data() + s * NP, (int64_t)s));
  }
  double px_weight = 1.0;
  std::vector<int> kept_rows;
  if (keep) {
    CHK(subsample_items(ctx, b, &P, keep, keep_off, kept_rows));
    px_weight = 1.0 / keep_prob;
  }
  EvalBufs B;
  if (noalloc) {
    CHK(scratch_bufs(ctx, &P, grad ? (hess ? NACC : NGRAD) : 1, &B));
    const int rc = prepare_in(ctx, b, &P, &B, st, true);
    if (B.lfact_ready) scratch_lfact_filled(ctx->device);
    CHK(rc);
  } else {
    CHK(ctx_bufs(ctx, &P, &B));
    const int rc = prepare_in(ctx, b, &P, &B, st, true);
    ctx->lfact_ready = ctx->lfact_ready || B.lfact_ready;
    CHK(rc);
  }
  const int* kept = nullptr;
  if (keep) {
    CHK(ensure(ctx->kept, sizeof(int) * std::max<size_t>(1, kept_rows.size())));
    if (!kept_rows.empty())
      HIPCHK(hipMemcpyAsync(ctx->kept.p, kept_rows.data(), sizeof(int) * kept_rows.size(), hipMemcpyHostToDevice, st));
    kept = as<int>(ctx->kept);
  }
  double *d_elbo = elbo, *d_grad = grad, *d_hess = hess;
  if (b->mem_kind == CELESTE_MEM_HOST) {
    CHK(ensure(ctx->o_elbo, sizeof(double) * S));
    d_elbo = as<double>(ctx->o_elbo);
    if (grad) {
      CHK(ensure(ctx->o_grad, sizeof(double) * NP * S));
      d_grad = as<double>(ctx->o_grad);
    }
    if (hess) {
      CHK(ensure(ctx->o_hess, sizeof(double) * NP * NP * S));
      d_hess = as<double>(ctx->o_hess);
    }
  }
  PhaseTimer T;
  CHK(T.init(ctx->profile != 0 && !noalloc));   // events are not created on the no-allocation path
  T.mark(0, st);
  HIPCHK(launch_setup(B.imgs, P.n_img, th_dev, nullptr, P.prof, B.tables, P.tstride, st));
  T.mark(1, st);
  if (grad && hess) {
    HIPCHK(launch_eval_full(B.items, P.n_items, B.imgs, B.tables, P.tstride, P.prof.n_exp, P.prof.n_dev, nullptr,
                            B.partials, ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st, kept));
    T.mark(2, st);
    HIPCHK(launch_reduce_full(B.srcs, P.n_src, B.imgs, B.partials, B.img_const, th_dev, P.prior, nullptr, d_elbo,
                              d_grad, d_hess, ctr_full(ctx), st, px_weight));
    ctx->stats.full_launches += 1;
  } else if (grad) {
    HIPCHK(launch_eval_grad(B.items, P.n_items, B.imgs, B.tables, P.tstride, P.prof.n_exp, P.prof.n_dev, nullptr,
                            B.partials, ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st, kept));
    T.mark(2, st);
    HIPCHK(launch_reduce_grad(B.srcs, P.n_src, B.imgs, B.partials, B.img_const, th_dev, P.prior, nullptr, d_elbo,
                              d_grad, ctr_grad(ctx), st, px_weight));
    ctx->stats.grad_launches += 1;
  } else {
    HIPCHK(launch_eval_value(B.items, P.n_items, B.imgs, B.tables, P.tstride, P.prof.n_exp, P.prof.n_dev, nullptr,
                             B.partials, ctx->vblock, ctx->variant, ctx->vtile_log2, st, kept));
    T.mark(2, st);
    HIPCHK(launch_reduce_value(B.srcs, P.n_src, B.imgs, B.partials, B.img_const, th_dev, P.prior, nullptr, d_elbo,
                               ctr_value(ctx), st, px_weight));
    ctx->stats.value_launches += 1;
  }
  T.mark(3, st);
  if (b->mem_kind == CELESTE_MEM_HOST) {
    HIPCHK(hipMemcpyAsync(elbo, d_elbo, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    if (grad) HIPCHK(hipMemcpyAsync(grad, d_grad, sizeof(double) * NP * S, hipMemcpyDeviceToHost, st));
    if (hess) HIPCHK(hipMemcpyAsync(hess, d_hess, sizeof(double) * NP * NP * S, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (T.on) {
    ctx->stats.ms_setup += T.span(0, 1);
    (hess ? ctx->stats.ms_full : grad ? ctx->stats.ms_grad : ctx->stats.ms_value) += T.span(1, 2);
    (hess ? ctx->stats.ms_reduce_full : grad ? ctx->stats.ms_reduce_grad : ctx->stats.ms_reduce_value) += T.span(2, 3);
  }
  return CELESTE_OK;
}

}  // namespace

// =============================================================================== no-allocation scratch

// Device memory of celeste_elbo_eval_noalloc: one array on every GPU the library runs on,
// resident from the code object's load until the process ends, shared by every such call on
// that GPU (it keeps the last call's contents, and calls that overlap on one GPU race).  In
// host code the array's name is a host-side stand-in, not a device address: host code uses
// only the per-device address that hipGetSymbolAddress returns (scratch_init).
static __device__ __align__(256) unsigned char scratch[CELESTE_NOALLOC_SCRATCH_BYTES];

namespace {

struct ScratchSlot {
  unsigned char* ptr = nullptr;   // device address of the scratch array on this GPU
  bool lfact_ready = false;       // its log n! region holds the table
};
std::mutex g_scratch_mu;
std::unordered_map<int, ScratchSlot> g_scratch;

// Once per device, with that device current (context creation): the device address of the
// scratch array on it.
int scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ScratchSlot& sl = g_scratch[device];
  if (sl.ptr) return CELESTE_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(CELESTE_E_DEVICE, "address of the scratch array on device %d: %s", device, hipGetErrorString(e));
  }
  sl.ptr = static_cast<unsigned char*>(ptr);
  return CELESTE_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// The buffers of one evaluation carved from the device's scratch array: the log n! table
// first (filled once per device, never written by anything else), then the call's own
// regions.  E_NOMEM when the batch does not fit.
int scratch_bufs(celeste_ctx* ctx, const Packed* P, int per_item, EvalBufs* B) {
  ScratchSlot sl;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(ctx->device);
    if (it == g_scratch.end() || !it->second.ptr)
      return fail(CELESTE_E_DEVICE, "no scratch address for device %d", ctx->device);
    sl = it->second;
  }
  size_t off = 0;
  auto carve = [&off](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t o_lfact = carve(sizeof(double) * LFACT_N);
  const size_t o_flag = carve(sizeof(int) * 4);
  const size_t o_imgs = carve(sizeof(ImgDev) * P->n_img);
  const size_t o_items = carve(sizeof(WorkItem) * P->n_items);
  const size_t o_srcs = carve(sizeof(SrcDev) * P->n_src);
  const size_t o_const = carve(sizeof(double) * P->n_img);
  const size_t o_tables = carve(sizeof(float) * (size_t)P->tstride * P->n_img);
  const size_t o_part = carve(sizeof(double) * (size_t)per_item * P->n_items);
  if (off > CELESTE_NOALLOC_SCRATCH_BYTES)
    return fail(CELESTE_E_NOMEM,
                "the batch (%d sources, %d images, %d work items) needs %zu bytes of device scratch; "
                "celeste_elbo_eval_noalloc holds at most %zu: split the batch or use celeste_elbo_eval",
                P->n_src, P->n_img, P->n_items, off, (size_t)CELESTE_NOALLOC_SCRATCH_BYTES);
  unsigned char* base = sl.ptr;
  B->lfact = reinterpret_cast<double*>(base + o_lfact);
  B->flag = reinterpret_cast<int*>(base + o_flag);
  B->imgs = reinterpret_cast<ImgDev*>(base + o_imgs);
  B->items = reinterpret_cast<WorkItem*>(base + o_items);
  B->srcs = reinterpret_cast<SrcDev*>(base + o_srcs);
  B->img_const = reinterpret_cast<double*>(base + o_const);
  B->tables = reinterpret_cast<float*>(base + o_tables);
  B->partials = reinterpret_cast<double*>(base + o_part);
  B->lfact_ready = sl.lfact_ready;
  return CELESTE_OK;
}

void scratch_lfact_filled(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  g_scratch[device].lfact_ready = true;
}

}  // namespace

// =============================================================================== fits

namespace {

struct FitBufs {
  FitDev d;
};

int alloc_fit(celeste_ctx* ctx, int S, FitDev* f) {
  const size_t nd = (size_t)S * (NP * 6 + 3 * NP * NP + 2 + 7);
  const size_t ni = (size_t)S * 11 + 1;
  CHK(ensure(ctx->st_buf, nd * sizeof(double) + ni * sizeof(int) + 256));
  double* d = as<double>(ctx->st_buf);
  auto take = [&](size_t n) {
    double* r = d;
    d += n;
    return r;
  };
  f->theta = take((size_t)S * NP);
  f->psi = take((size_t)S * NP);
  f->theta_trial = take((size_t)S * NP);
  f->g = take((size_t)S * NP);
  f->p = take((size_t)S * NP);
  f->H = take((size_t)S * NP * NP);
  f->V = take((size_t)S * NP * NP);
  f->g_trial = take((size_t)S * NP);
  f->H_trial = take((size_t)S * NP * NP);
  f->u0 = take((size_t)S * 2);
  f->f = take(S);
  f->f_full = take(S);
  f->f_trial = take(S);
  f->pred = take(S);
  f->delta = take(S);
  f->pnorm = take(S);
  take(S);
  int* ip = reinterpret_cast<int*>(d);
  f->iter = ip;
  f->status = ip + S;
  f->active = ip + 2 * S;
  f->need_full = ip + 3 * S;
  f->n_full = ip + 4 * S;
  f->flags = ip + 5 * S;
  f->samp = ip + 6 * S;
  f->sw = ip + 7 * S;
  f->fa = ip + 8 * S;
  f->fb = ip + 9 * S;
  f->n_acc = ip + 10 * S;
  f->n_active = ip + 11 * S;
  return CELESTE_OK;
}

int check_opts(const celeste_fit_opts* o) {
  if (!o) return fail(CELESTE_E_INVALID, "opts is NULL");
  if (o->max_iter < 1 || o->max_iter > 100000) return fail(CELESTE_E_INVALID, "max_iter must be in 1..100000");
  if (o->init_mode != CELESTE_INIT_AS_GIVEN && o->init_mode != CELESTE_INIT_PLAIN &&
      o->init_mode != CELESTE_INIT_SURROGATE)
    return fail(CELESTE_E_INVALID, "init_mode %d not known", o->init_mode);
  if (!(o->pred_rtol >= 0.0) || !(o->curv_tol >= 0.0) || !(o->delta0 > 0.0) || !(o->delta_max >= o->delta0) ||
      !(o->delta_min >= 0.0) || !(o->eta >= 0.0 && o->eta < 1.0) || !(o->u_box > 0.0))
    return fail(CELESTE_E_INVALID, "fit options out of range");
  return CELESTE_OK;
}

// Enqueues one trust-region iteration over all sources (each kernel skips sources
// whose flag is clear).
// Persistent-grid size of the value+gradient+Hessian kernel for a fit over P: the compute units
// times the chosen blocks per compute unit, or (persistent < 0) times the blocks the launched kernel
// instance keeps resident on one.
int fit_grid(celeste_ctx* ctx, const Packed& P) {
  int bpc = ctx->persistent;
  if (bpc < 0) {
    HIPCHK(eval_full_blocks_per_cu(ctx->block, full_variant(ctx), P.prof.n_exp, P.prof.n_dev, &bpc));
    bpc = std::max(1, bpc);
  }
  ctx->pgrid = ctx->n_cu * bpc;
  ctx->stats.fit_grid_blocks = ctx->pgrid;
  return CELESTE_OK;
}

// The device work queue of a fit over P's work items (persistent mode).
int fit_queue(celeste_ctx* ctx, const Packed& P, WorkQueue* q) {
  CHK(ensure(ctx->qbuf, sizeof(int) * ((size_t)P.n_items + 64)));
  int* b = as<int>(ctx->qbuf);
  q->hdr = b;
  q->items = b + 64;
  q->srcs = as<SrcDev>(ctx->srcs);
  return CELESTE_OK;
}

int enqueue_iteration(celeste_ctx* ctx, const Packed& P, const FitDev& F, const FitParams& fp, hipStream_t st,
                      PhaseTimer* T, const WorkQueue* Q = nullptr) {
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  const WorkItem* items = as<WorkItem>(ctx->items);
  const SrcDev* srcs = as<SrcDev>(ctx->srcs);
  float* tables = as<float>(ctx->tables);
  double* parts = as<double>(ctx->partials);
  const double* ic = as<double>(ctx->img_const);
  T->mark(0, st);
  if (Q) HIPCHK(launch_build_queue(*Q, P.n_src, F.need_full, st));
  HIPCHK(launch_setup(imgs, P.n_img, F.theta, F.need_full, P.prof, tables, P.tstride, st));
  T->mark(1, st);
  HIPCHK(launch_eval_full(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.need_full, parts,
                          ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st, nullptr, Q, ctx->pgrid));
  T->mark(2, st);
  HIPCHK(launch_reduce_full(srcs, P.n_src, imgs, parts, ic, F.theta, P.prior, F.need_full, F.f_full, F.g, F.H,
                            ctr_full(ctx), st));
  T->mark(3, st);
  HIPCHK(launch_zero_int(F.n_active, 1, st));
  HIPCHK(launch_tr_step(F, P.n_src, fp, st));
  T->mark(4, st);
  HIPCHK(launch_setup(imgs, P.n_img, F.theta_trial, F.active, P.prof, tables, P.tstride, st));
  T->mark(5, st);
  HIPCHK(launch_eval_value(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.active, parts,
                           ctx->vblock, ctx->variant, ctx->vtile_log2, st));
  T->mark(6, st);
  HIPCHK(launch_reduce_value(srcs, P.n_src, imgs, parts, ic, F.theta_trial, P.prior, F.active, F.f_trial,
                             ctr_value(ctx), st));
  T->mark(7, st);
  HIPCHK(launch_accept(F, P.n_src, fp, st));
  T->mark(8, st);
  return CELESTE_OK;
}

// The value+gradient+Hessian pass at the current point of the sources flagged need_full (with
// trial derivatives: once, before the first iteration).
int enqueue_current_derivs(celeste_ctx* ctx, const Packed& P, const FitDev& F, hipStream_t st, PhaseTimer* T,
                           const WorkQueue* Q) {
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  double* parts = as<double>(ctx->partials);
  T->mark(0, st);
  if (Q) HIPCHK(launch_build_queue(*Q, P.n_src, F.need_full, st));
  HIPCHK(launch_setup(imgs, P.n_img, F.theta, F.need_full, P.prof, as<float>(ctx->tables), P.tstride, st));
  T->mark(1, st);
  HIPCHK(launch_eval_full(as<WorkItem>(ctx->items), P.n_items, imgs, as<float>(ctx->tables), P.tstride,
                          P.prof.n_exp, P.prof.n_dev, F.need_full, parts, ctx->block, full_variant(ctx),
                          ctx->tile_log2, ctx->e_zero, st, nullptr, Q, ctx->pgrid));
  T->mark(2, st);
  HIPCHK(launch_reduce_full(as<SrcDev>(ctx->srcs), P.n_src, imgs, parts, as<double>(ctx->img_const), F.theta,
                            P.prior, F.need_full, F.f_full, F.g, F.H, ctr_full(ctx), st));
  T->mark(3, st);
  return CELESTE_OK;
}

// One trust-region iteration with trial derivatives (section III-B): the subproblem at the current
// point, the ELBO with its gradient and Hessian at the trial point, the ratio test, and an accepted
// step taking over the trial point's gradient and Hessian.
int enqueue_iteration_td(celeste_ctx* ctx, const Packed& P, const FitDev& F, const FitParams& fp, hipStream_t st,
                         PhaseTimer* T, const WorkQueue* Q) {
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  double* parts = as<double>(ctx->partials);
  T->mark(0, st);
  HIPCHK(launch_zero_int(F.n_active, 1, st));
  HIPCHK(launch_tr_step(F, P.n_src, fp, st));
  T->mark(1, st);
  if (Q) HIPCHK(launch_build_queue(*Q, P.n_src, F.active, st));
  HIPCHK(launch_setup(imgs, P.n_img, F.theta_trial, F.active, P.prof, as<float>(ctx->tables), P.tstride, st));
  T->mark(2, st);
  HIPCHK(launch_eval_full(as<WorkItem>(ctx->items), P.n_items, imgs, as<float>(ctx->tables), P.tstride,
                          P.prof.n_exp, P.prof.n_dev, F.active, parts, ctx->block, full_variant(ctx),
                          ctx->tile_log2, ctx->e_zero, st, nullptr, Q, ctx->pgrid));
  T->mark(3, st);
  HIPCHK(launch_reduce_full(as<SrcDev>(ctx->srcs), P.n_src, imgs, parts, as<double>(ctx->img_const),
                            F.theta_trial, P.prior, F.active, F.f_trial, F.g_trial, F.H_trial, ctr_trial(ctx), st));
  T->mark(4, st);
  HIPCHK(launch_accept(F, P.n_src, fp, st));
  HIPCHK(launch_take_trial(F, P.n_src, st));
  T->mark(5, st);
  return CELESTE_OK;
}

void accumulate_phases_td(celeste_ctx* ctx, PhaseTimer& T) {
  if (!T.on) return;
  celeste_stats& s = ctx->stats;
  s.ms_tr += T.span(0, 1);
  s.ms_setup += T.span(1, 2);
  s.ms_full += T.span(2, 3);
  s.ms_reduce_full += T.span(3, 4);
  s.ms_accept += T.span(4, 5);
}

void accumulate_phases(celeste_ctx* ctx, PhaseTimer& T) {
  if (!T.on) return;
  celeste_stats& s = ctx->stats;
  s.ms_setup += T.span(0, 1) + T.span(4, 5);
  s.ms_full += T.span(1, 2);
  s.ms_reduce_full += T.span(2, 3);
  s.ms_tr += T.span(3, 4);
  s.ms_value += T.span(5, 6);
  s.ms_reduce_value += T.span(6, 7);
  s.ms_accept += T.span(7, 8);
}

// Host wall clock of the fits' stages (profile mode only): stage k ends at a call; the stream
// is drained first.
struct StageClock {
  bool on;
  std::chrono::steady_clock::time_point t_last = std::chrono::steady_clock::now();
  explicit StageClock(bool on_) : on(on_) {}
  void operator()(double& acc, hipStream_t s) {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    const auto now = std::chrono::steady_clock::now();
    acc += std::chrono::duration<double, std::milli>(now - t_last).count();
    t_last = now;
  }
};

// The common start of the trust-region and L-BFGS fits: validation, packing, metadata upload
// and pixel check, the fit state (F), and the start (plain, surrogate with fallback, or as
// given) with its ELBO in F.f; a source whose start is not finite is not fitted.  th receives
// the host copy of theta_inout.
int fit_begin(celeste_ctx* ctx, const celeste_batch* b, const double* theta_inout, int init_mode,
              const FitParams& fp, hipStream_t st, StageClock& stage, Packed* Pp, FitDev* Fp,
              std::vector<double>* thp) {
  Packed& P = *Pp;
  FitDev& F = *Fp;
  std::vector<double>& th = *thp;
  HIPCHK(hipSetDevice(ctx->device));
  const int S = P.n_src;
  th.resize(NP * (size_t)S);
  if (b->mem_kind == CELESTE_MEM_HOST)
    std::memcpy(th.data(), theta_inout, sizeof(double) * th.size());
  else {
    HIPCHK(hipMemcpyAsync(th.data(), theta_inout, sizeof(double) * th.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (init_mode == CELESTE_INIT_SURROGATE && !ctx->net)
    return fail(CELESTE_E_INVALID, "CELESTE_INIT_SURROGATE needs a network (celeste_ctx_set_surrogate)");
  for (int s = 0; s < S; ++s) {
    if (init_mode != CELESTE_INIT_AS_GIVEN) {
      if (!finite(th[(size_t)s * NP]) || !finite(th[(size_t)s * NP + 1]))
        return fail(CELESTE_E_INVALID, "theta[%d]: position must be finite", s);
    } else {
      CHK(check_theta(th.data() + (size_t)s * NP, s));
    }
  }
  stage(ctx->stats.ms_host_pack, st);
  CHK(prepare(ctx, b, &P, st));
  stage(ctx->stats.ms_prepare, st);
  CHK(alloc_fit(ctx, S, &F));
  HIPCHK(hipMemcpyAsync(F.theta, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, st));
  HIPCHK(launch_zero_int(F.flags, S, st));
  const ImgDev* imgs0 = as<ImgDev>(ctx->imgs);
  if (init_mode == CELESTE_INIT_SURROGATE) {
    // network start (from the catalog positions in F.theta) into theta_trial, plain start into theta,
    // both evaluated; the better one is kept
    CHK(ensure(ctx->sur, sizeof(float) * NP * (size_t)S));
    CHK(surrogate_predict(ctx->net, as<SrcDev>(ctx->srcs), S, imgs0, F.theta, as<float>(ctx->sur), st));
    HIPCHK(launch_psi_to_theta(as<float>(ctx->sur), F.theta, F.theta_trial, S, fp.u_box, st));
    stage(ctx->stats.ms_net, st);
    HIPCHK(launch_plain_init(as<SrcDev>(ctx->srcs), S, imgs0, P.prior, F.theta, st));
    for (int k = 0; k < 2; ++k) {
      double* tk = k == 0 ? F.theta : F.theta_trial;
      HIPCHK(launch_setup(imgs0, P.n_img, tk, nullptr, P.prof, as<float>(ctx->tables), P.tstride, st));
      HIPCHK(launch_eval_value(as<WorkItem>(ctx->items), P.n_items, imgs0, as<float>(ctx->tables), P.tstride,
                               P.prof.n_exp, P.prof.n_dev, nullptr, as<double>(ctx->partials), ctx->vblock, ctx->variant,
                             ctx->vtile_log2, st));
      HIPCHK(launch_reduce_value(as<SrcDev>(ctx->srcs), S, imgs0, as<double>(ctx->partials),
                                 as<double>(ctx->img_const), tk, P.prior, nullptr, k == 0 ? F.f : F.f_trial,
                                 ctr_value(ctx), st));
      ctx->stats.value_launches += 1;
    }
    HIPCHK(launch_choose_start(F, S, st));
  } else if (init_mode == CELESTE_INIT_PLAIN) {
    HIPCHK(launch_plain_init(as<SrcDev>(ctx->srcs), S, imgs0, P.prior, F.theta, st));
  }
  HIPCHK(launch_fit_init(F, S, fp, st));
  if (init_mode != CELESTE_INIT_SURROGATE) {
    // the start's ELBO (the surrogate path has it from choosing between the two starts: both lie
    // inside the boxes, where the transform round trip of the fit set-up moves a parameter by
    // rounding, or by at most 1e-9 of its box where a start sits on the box edge)
    const ImgDev* imgs = as<ImgDev>(ctx->imgs);
    HIPCHK(launch_setup(imgs, P.n_img, F.theta, nullptr, P.prof, as<float>(ctx->tables), P.tstride, st));
    HIPCHK(launch_eval_value(as<WorkItem>(ctx->items), P.n_items, imgs, as<float>(ctx->tables), P.tstride,
                             P.prof.n_exp, P.prof.n_dev, nullptr, as<double>(ctx->partials), ctx->vblock,
                             ctx->variant, ctx->vtile_log2, st));
    HIPCHK(launch_reduce_value(as<SrcDev>(ctx->srcs), S, imgs, as<double>(ctx->partials),
                               as<double>(ctx->img_const), F.theta, P.prior, nullptr, F.f, ctr_value(ctx), st));
    ctx->stats.value_launches += 1;
  }
  HIPCHK(launch_fit_start(F, S, st));
  return CELESTE_OK;
}

// Per-source results of a fit from its device state; theta_inout receives the parameters.
int fit_results(celeste_ctx* ctx, const celeste_batch* b, const FitDev& F, int S, std::vector<double>& th,
                double* theta_inout, celeste_fit_result* res, hipStream_t st, StageClock& stage) {
  std::vector<double> fv(S), pred(S), delta(S);
  std::vector<int> iter(S), status(S), nfull(S), flags(S), nacc(S);
  HIPCHK(hipMemcpyAsync(th.data(), F.theta, sizeof(double) * th.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(fv.data(), F.f, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pred.data(), F.pred, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(delta.data(), F.delta, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(iter.data(), F.iter, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(status.data(), F.status, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nfull.data(), F.n_full, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(flags.data(), F.flags, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(nacc.data(), F.n_acc, sizeof(int) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (b->mem_kind == CELESTE_MEM_HOST)
    std::memcpy(theta_inout, th.data(), sizeof(double) * th.size());
  else {
    HIPCHK(hipMemcpyAsync(theta_inout, F.theta, sizeof(double) * th.size(), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  stage(ctx->stats.ms_results, st);
  for (int s = 0; s < S; ++s) {
    res[s].elbo = fv[s];
    res[s].pred_gain = pred[s];
    res[s].delta = delta[s];
    res[s].iters = iter[s];
    res[s].status = status[s];
    res[s].n_full_evals = nfull[s];
    res[s].n_accepted = nacc[s];
    res[s].reserved = 0;
    res[s].flags = flags[s];
  }
  return CELESTE_OK;
}

// Replays (graph) or enqueues (eager) `iteration` until no source is active or max_loops loop
// steps; the host reads the device's active count every `poll` steps.
// count(stats) records the launches of one executed step (replayed or enqueued).
template <class Iter, class Count>
int run_loop(celeste_ctx* ctx, hipStream_t st, int max_loops, int poll, bool use_graph, const int* n_active_dev,
             PhaseTimer& T, Iter iteration, Count count, void (*account)(celeste_ctx*, PhaseTimer&)) {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph) {
    PhaseTimer none;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = iteration(&none);
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (rc != CELESTE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HIPCHK(e2);
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  int rc = CELESTE_OK;
  int n_active = 1;
  for (int it = 0; it < max_loops && n_active > 0; ++it) {
    if (exec) {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        rc = fail(CELESTE_E_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    } else {
      rc = iteration(&T);
      if (rc != CELESTE_OK) break;
    }
    ctx->stats.iterations += 1;
    count(ctx->stats);
    if ((it + 1) % poll == 0 || it + 1 == max_loops) {
      hipError_t e = hipMemcpyAsync(&n_active, n_active_dev, sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        rc = fail(CELESTE_E_DEVICE, "active-count readback: %s", hipGetErrorString(e));
        break;
      }
      account(ctx, T);
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  return rc;
}

int run_fit(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_fit_opts* o,
            celeste_fit_result* res, hipStream_t st, bool batched, double* start_elbo = nullptr,
            bool start_only = false) {
  StageClock stage(ctx->profile != 0);
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  if (start_only) {
    if (!o) return fail(CELESTE_E_INVALID, "opts is NULL");
    celeste_fit_opts o2 = *o;
    o2.max_iter = 1;
    CHK(check_opts(&o2));
  } else {
    CHK(check_opts(o));
  }
  if (!theta_inout || (!res && !start_only)) return fail(CELESTE_E_INVALID, "theta_inout and results must not be NULL");
  const int S = P.n_src;
  FitParams fp{};
  fp.max_iter = o->max_iter;
  fp.pred_rtol = o->pred_rtol;
  fp.curv_tol = o->curv_tol;
  fp.delta0 = o->delta0;
  fp.delta_max = o->delta_max;
  fp.delta_min = o->delta_min;
  fp.eta = o->eta;
  fp.u_box = o->u_box;
  fp.tr_chol = ctx->tr_chol;
  fp.trial_derivs = ctx->trial_derivs;
  fp.tr_ctr = as<unsigned long long>(ctx->ctr) + 3;
  FitDev F;
  std::vector<double> th;
  CHK(fit_begin(ctx, b, theta_inout, o->init_mode, fp, st, stage, &P, &F, &th));
  // the batch's per-source metadata exists from here on (fit_begin's upload may reallocate it)
  fp.srcs = as<SrcDev>(ctx->srcs);
  fp.taken_px = ctr_taken(ctx);
  if (start_only) {
    if (b->mem_kind == CELESTE_MEM_HOST) {
      HIPCHK(hipMemcpyAsync(theta_inout, F.theta, sizeof(double) * th.size(), hipMemcpyDeviceToHost, st));
      if (start_elbo) HIPCHK(hipMemcpyAsync(start_elbo, F.f, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    } else {
      HIPCHK(hipMemcpyAsync(theta_inout, F.theta, sizeof(double) * th.size(), hipMemcpyDeviceToDevice, st));
      if (start_elbo) HIPCHK(hipMemcpyAsync(start_elbo, F.f, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return CELESTE_OK;
  }
  stage(ctx->stats.ms_start, st);
  PhaseTimer T;
  CHK(T.init(ctx->profile != 0));
  const int poll = (batched && !T.on) ? std::max(1, o->poll_every) : 1;
  const bool graph = batched && ctx->use_graph && !T.on;
  WorkQueue Q;
  ctx->stats.fit_grid_blocks = 0;
  if (ctx->persistent) {
    CHK(fit_queue(ctx, P, &Q));
    CHK(fit_grid(ctx, P));
  }
  const WorkQueue* Qp = ctx->persistent ? &Q : nullptr;
  if (fp.trial_derivs) {
    // the start's gradient and Hessian, then iterations that evaluate them at every trial point
    CHK(enqueue_current_derivs(ctx, P, F, st, &T, Qp));
    ctx->stats.full_launches += 1;
    if (T.on) {
      HIPCHK(hipStreamSynchronize(st));
      ctx->stats.ms_setup += T.span(0, 1);
      ctx->stats.ms_full += T.span(1, 2);
      ctx->stats.ms_reduce_full += T.span(2, 3);
    }
    CHK(run_loop(ctx, st, o->max_iter + 1, poll, graph, F.n_active, T,
                 [&](PhaseTimer* t) { return enqueue_iteration_td(ctx, P, F, fp, st, t, Qp); },
                 [](celeste_stats& c) { c.full_launches += 1; }, accumulate_phases_td));
  } else {
    CHK(run_loop(ctx, st, o->max_iter + 1, poll, graph, F.n_active, T,
                 [&](PhaseTimer* t) { return enqueue_iteration(ctx, P, F, fp, st, t, Qp); },
                 [](celeste_stats& c) {
                   c.full_launches += 1;
                   c.value_launches += 1;
                 },
                 accumulate_phases));
  }
  stage(ctx->stats.ms_loop, st);
  return fit_results(ctx, b, F, S, th, theta_inout, res, st, stage);
}

// Trust-region fit whose early phase fits a pixel-subsampled estimate of the ELBO (8-row
// blocks kept by `keep`, weighted 1 / keep_prob): each source moves to the full ELBO when its
// model's predicted gain on the estimate falls to switch_rtol max(1, |L|), and then runs the
// fit's own stopping rule.  One iteration evaluates, per source, on whichever objective it is in.
int run_fit_sampled(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_fit_opts* o,
                    const uint8_t* keep, const int64_t* keep_off, double keep_prob, double switch_rtol,
                    celeste_fit_result* res, hipStream_t st) {
  StageClock stage(ctx->profile != 0);
  if (!keep || !keep_off) return fail(CELESTE_E_INVALID, "keep and keep_off must not be NULL");
  if (!(keep_prob > 0.0 && keep_prob <= 1.0)) return fail(CELESTE_E_INVALID, "keep_prob must be in (0, 1]");
  if (!(switch_rtol > 0.0)) return fail(CELESTE_E_INVALID, "switch_rtol must be > 0");
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_opts(o));
  if (!theta_inout || !res) return fail(CELESTE_E_INVALID, "theta_inout and results must not be NULL");
  if (keep_off[0] != 0) return fail(CELESTE_E_INVALID, "keep_off[0] must be 0");
  for (int i = 0; i < P.n_img; ++i)
    if (keep_off[i + 1] - keep_off[i] != (b->images[i].h + 7) / 8)
      return fail(CELESTE_E_INVALID, "image %d: keep_off must give (h + 7) / 8 blocks", i);
  const int S = P.n_src;
  FitParams fp{};
  fp.max_iter = o->max_iter;
  fp.pred_rtol = o->pred_rtol;
  fp.curv_tol = o->curv_tol;
  fp.delta0 = o->delta0;
  fp.delta_max = o->delta_max;
  fp.delta_min = o->delta_min;
  fp.eta = o->eta;
  fp.u_box = o->u_box;
  fp.switch_rtol = switch_rtol;
  fp.tr_chol = ctx->tr_chol;
  fp.tr_ctr = as<unsigned long long>(ctx->ctr) + 3;
  FitDev F;
  std::vector<double> th;
  CHK(fit_begin(ctx, b, theta_inout, o->init_mode, fp, st, stage, &P, &F, &th));
  // the subsampled pack: the dense image records (pixels already staged) with work items over
  // the kept blocks only
  HostPack hs;
  hs.imgs.assign(P.imgs, P.imgs + P.n_img);
  hs.srcs.assign(P.srcs, P.srcs + P.n_src);
  Packed Ps = P;
  Ps.imgs = hs.imgs.data();
  Ps.srcs = hs.srcs.data();
  std::vector<int> kept_rows;
  CHK(subsample_items(ctx, b, &Ps, keep, keep_off, kept_rows));
  CHK(ensure(ctx->imgs_s, sizeof(ImgDev) * Ps.n_img));
  CHK(ensure(ctx->items_s, sizeof(WorkItem) * std::max(1, Ps.n_items)));
  CHK(ensure(ctx->srcs_s, sizeof(SrcDev) * Ps.n_src));
  CHK(ensure(ctx->partials_s, sizeof(double) * (size_t)NACC * std::max(1, Ps.n_items)));
  CHK(ensure(ctx->kept, sizeof(int) * std::max<size_t>(1, kept_rows.size())));
  HIPCHK(hipMemcpyAsync(ctx->imgs_s.p, Ps.imgs, sizeof(ImgDev) * Ps.n_img, hipMemcpyHostToDevice, st));
  if (Ps.n_items > 0)
    HIPCHK(hipMemcpyAsync(ctx->items_s.p, Ps.items, sizeof(WorkItem) * Ps.n_items, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->srcs_s.p, Ps.srcs, sizeof(SrcDev) * Ps.n_src, hipMemcpyHostToDevice, st));
  if (!kept_rows.empty())
    HIPCHK(hipMemcpyAsync(ctx->kept.p, kept_rows.data(), sizeof(int) * kept_rows.size(), hipMemcpyHostToDevice, st));
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  const WorkItem* items = as<WorkItem>(ctx->items);
  const SrcDev* srcs = as<SrcDev>(ctx->srcs);
  const ImgDev* imgs_s = as<ImgDev>(ctx->imgs_s);
  const WorkItem* items_s = as<WorkItem>(ctx->items_s);
  const SrcDev* srcs_s = as<SrcDev>(ctx->srcs_s);
  const int* kept = as<int>(ctx->kept);
  float* tables = as<float>(ctx->tables);
  double* parts = as<double>(ctx->partials);
  double* parts_s = as<double>(ctx->partials_s);
  const double* ic = as<double>(ctx->img_const);
  const double w = 1.0 / keep_prob;
  // every fitted source starts on the subsampled objective: its value there at the start
  HIPCHK(launch_fill_int(F.samp, S, 1, st));
  HIPCHK(launch_split(F.active, F.samp, F.fa, F.fb, S, st));
  HIPCHK(launch_setup(imgs, P.n_img, F.theta, F.fb, P.prof, tables, P.tstride, st));
  HIPCHK(launch_eval_value(items_s, Ps.n_items, imgs_s, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.fb, parts_s,
                           ctx->vblock, ctx->variant, ctx->vtile_log2, st, kept));
  HIPCHK(launch_reduce_value(srcs_s, S, imgs_s, parts_s, ic, F.theta, P.prior, F.fb, F.f, ctr_value(ctx), st, w));
  stage(ctx->stats.ms_start, st);
  PhaseTimer T;
  CHK(T.init(ctx->profile != 0));
  auto iteration = [&](PhaseTimer* t) -> int {
    t->mark(0, st);
    HIPCHK(launch_split(F.need_full, F.samp, F.fa, F.fb, S, st));
    HIPCHK(launch_setup(imgs, P.n_img, F.theta, F.need_full, P.prof, tables, P.tstride, st));
    t->mark(1, st);
    HIPCHK(launch_eval_full(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.fa, parts,
                            ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st));
    HIPCHK(launch_eval_full(items_s, Ps.n_items, imgs_s, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.fb, parts_s,
                            ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st, kept));
    t->mark(2, st);
    HIPCHK(launch_reduce_full(srcs, S, imgs, parts, ic, F.theta, P.prior, F.fa, F.f_full, F.g, F.H, ctr_full(ctx), st));
    HIPCHK(launch_reduce_full(srcs_s, S, imgs_s, parts_s, ic, F.theta, P.prior, F.fb, F.f_full, F.g, F.H,
                              ctr_full(ctx), st, w));
    t->mark(3, st);
    HIPCHK(launch_zero_int(F.n_active, 1, st));
    HIPCHK(launch_tr_step(F, S, fp, st));
    t->mark(4, st);
    HIPCHK(launch_split(F.active, F.samp, F.fa, F.fb, S, st));
    HIPCHK(launch_setup(imgs, P.n_img, F.theta_trial, F.active, P.prof, tables, P.tstride, st));
    t->mark(5, st);
    HIPCHK(launch_eval_value(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.fa, parts,
                             ctx->vblock, ctx->variant, ctx->vtile_log2, st));
    HIPCHK(launch_eval_value(items_s, Ps.n_items, imgs_s, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.fb, parts_s,
                             ctx->vblock, ctx->variant, ctx->vtile_log2, st, kept));
    t->mark(6, st);
    HIPCHK(launch_reduce_value(srcs, S, imgs, parts, ic, F.theta_trial, P.prior, F.fa, F.f_trial, ctr_value(ctx), st));
    HIPCHK(launch_reduce_value(srcs_s, S, imgs_s, parts_s, ic, F.theta_trial, P.prior, F.fb, F.f_trial,
                               ctr_value(ctx), st, w));
    t->mark(7, st);
    HIPCHK(launch_accept(F, S, fp, st));
    t->mark(8, st);
    return CELESTE_OK;
  };
  const int poll = T.on ? 1 : std::max(1, o->poll_every);
  // the switches are loop steps that are not iterations: room for one per source
  CHK(run_loop(ctx, st, o->max_iter + 2, poll, ctx->use_graph && !T.on, F.n_active, T, iteration,
               [](celeste_stats& c) {
                 c.full_launches += 1;
                 c.value_launches += 1;
               },
               accumulate_phases));
  stage(ctx->stats.ms_loop, st);
  return fit_results(ctx, b, F, S, th, theta_inout, res, st, stage);
}

int check_lbfgs_opts(const celeste_lbfgs_opts* o) {
  if (!o) return fail(CELESTE_E_INVALID, "opts is NULL");
  if (o->max_iter < 1 || o->max_iter > 1000000) return fail(CELESTE_E_INVALID, "max_iter must be in 1..1e6");
  if (o->memory < 1 || o->memory > LBFGS_MAX_MEMORY) return fail(CELESTE_E_INVALID, "memory must be in 1..32");
  if (o->max_backtracks < 1 || o->max_backtracks > 60) return fail(CELESTE_E_INVALID, "max_backtracks must be in 1..60");
  if (o->init_mode != CELESTE_INIT_AS_GIVEN && o->init_mode != CELESTE_INIT_PLAIN &&
      o->init_mode != CELESTE_INIT_SURROGATE)
    return fail(CELESTE_E_INVALID, "unknown init_mode %d", o->init_mode);
  if (o->max_loops < 0) return fail(CELESTE_E_INVALID, "max_loops must be >= 0");
  if (!(o->pred_rtol > 0.0) || !(o->armijo_c1 > 0.0 && o->armijo_c1 < 0.5) || !(o->u_box > 0.0))
    return fail(CELESTE_E_INVALID, "pred_rtol and u_box must be > 0 and armijo_c1 in (0, 1/2)");
  return CELESTE_OK;
}

void accumulate_lbfgs_phases(celeste_ctx* ctx, PhaseTimer& T) {
  if (!T.on) return;
  celeste_stats& s = ctx->stats;
  s.ms_setup += T.span(0, 1) + T.span(4, 5);
  s.ms_grad += T.span(1, 2);
  s.ms_reduce_grad += T.span(2, 3);
  s.ms_lbfgs += T.span(3, 4) + T.span(7, 8);
  s.ms_value += T.span(5, 6);
  s.ms_reduce_value += T.span(6, 7);
}

int run_lbfgs(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_lbfgs_opts* o,
              celeste_fit_result* res, hipStream_t st) {
  StageClock stage(ctx->profile != 0);
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_lbfgs_opts(o));
  if (!theta_inout || !res) return fail(CELESTE_E_INVALID, "theta_inout and results must not be NULL");
  const int S = P.n_src;
  FitParams fp{};
  fp.max_iter = o->max_iter;
  fp.delta0 = 1.0;
  fp.u_box = o->u_box;
  FitDev F;
  std::vector<double> th;
  CHK(fit_begin(ctx, b, theta_inout, o->init_mode, fp, st, stage, &P, &F, &th));
  // L-BFGS state: pairs, rho, gradients and scalars, then the integer counters
  const int m = o->memory;
  const size_t nd = (size_t)S * (2 * (size_t)m * NP + m + NP + 1);
  const size_t ni = (size_t)S * 5;
  CHK(ensure(ctx->lb_buf, nd * sizeof(double) + ni * sizeof(int) + 256));
  LbfgsDev X;
  {
    double* d = as<double>(ctx->lb_buf);
    auto take = [&d](size_t n) {
      double* r = d;
      d += n;
      return r;
    };
    X.S = take((size_t)S * m * NP);
    X.Y = take((size_t)S * m * NP);
    X.rho = take((size_t)S * m);
    X.gpsi = take((size_t)S * NP);
    X.gp = take(S);
    int* ip = reinterpret_cast<int*>(d);
    X.n_pairs = ip;
    X.head = ip + S;
    X.ls = ip + 2 * S;
    X.n_val = ip + 3 * S;
    X.in_ls = ip + 4 * S;
  }
  LbfgsParams lp;
  lp.max_iter = o->max_iter;
  lp.memory = m;
  lp.max_backtracks = o->max_backtracks;
  lp.pred_rtol = o->pred_rtol;
  lp.c1 = o->armijo_c1;
  lp.u_box = o->u_box;
  HIPCHK(launch_lbfgs_init(X, S, st));
  stage(ctx->stats.ms_start, st);
  PhaseTimer T;
  CHK(T.init(ctx->profile != 0));
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  const WorkItem* items = as<WorkItem>(ctx->items);
  const SrcDev* srcs = as<SrcDev>(ctx->srcs);
  float* tables = as<float>(ctx->tables);
  double* parts = as<double>(ctx->partials);
  const double* ic = as<double>(ctx->img_const);
  auto iteration = [&](PhaseTimer* t) -> int {
    t->mark(0, st);
    HIPCHK(launch_setup(imgs, P.n_img, F.theta, F.need_full, P.prof, tables, P.tstride, st));
    t->mark(1, st);
    HIPCHK(launch_eval_grad(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, F.need_full,
                            parts, ctx->block, full_variant(ctx), ctx->tile_log2, ctx->e_zero, st));
    t->mark(2, st);
    HIPCHK(launch_reduce_grad(srcs, P.n_src, imgs, parts, ic, F.theta, P.prior, F.need_full, F.f_full, F.g,
                              ctr_grad(ctx), st));
    t->mark(3, st);
    HIPCHK(launch_zero_int(F.n_active, 1, st));
    HIPCHK(launch_lbfgs_dir(F, X, P.n_src, lp, st));
    t->mark(4, st);
    HIPCHK(launch_setup(imgs, P.n_img, F.theta_trial, X.in_ls, P.prof, tables, P.tstride, st));
    t->mark(5, st);
    HIPCHK(launch_eval_value(items, P.n_items, imgs, tables, P.tstride, P.prof.n_exp, P.prof.n_dev, X.in_ls, parts,
                             ctx->vblock, ctx->variant, ctx->vtile_log2, st));
    t->mark(6, st);
    HIPCHK(launch_reduce_value(srcs, P.n_src, imgs, parts, ic, F.theta_trial, P.prior, X.in_ls, F.f_trial,
                               ctr_value(ctx), st));
    t->mark(7, st);
    HIPCHK(launch_lbfgs_accept(F, X, P.n_src, lp, st));
    t->mark(8, st);
    return CELESTE_OK;
  };
  const int max_loops = o->max_loops > 0 ? o->max_loops : 4 * o->max_iter + 64;
  const int poll = T.on ? 1 : std::max(1, o->poll_every);
  CHK(run_loop(ctx, st, max_loops, poll, ctx->use_graph && !T.on, F.n_active, T, iteration,
               [](celeste_stats& c) {
                 c.grad_launches += 1;
                 c.value_launches += 1;
               },
               accumulate_lbfgs_phases));
  stage(ctx->stats.ms_loop, st);
  return fit_results(ctx, b, F, S, th, theta_inout, res, st, stage);
}

}  // namespace

extern "C" {

int celeste_newton_fit(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_fit_opts* opts,
                       celeste_fit_result* result) {
  if (!b) return fail(CELESTE_E_INVALID, "batch is NULL");
  if (b->n_sources != 1) return fail(CELESTE_E_INVALID, "celeste_newton_fit takes exactly one source");
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  return run_fit(ctx, b, theta_inout, opts, result, ctx->stream, false);
}

int celeste_batch_fit(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_fit_opts* opts,
                      celeste_fit_result* results, void* stream) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  return run_fit(ctx, b, theta_inout, opts, results, pick(ctx, stream), true);
}

int celeste_batch_fit_sampled(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout,
                              const celeste_fit_opts* opts, const uint8_t* keep, const int64_t* keep_off,
                              double keep_prob, double switch_rtol, celeste_fit_result* results, void* stream) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  return run_fit_sampled(ctx, b, theta_inout, opts, keep, keep_off, keep_prob, switch_rtol, results,
                         pick(ctx, stream));
}

void celeste_lbfgs_opts_default(celeste_lbfgs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iter = 1000;
  o->memory = 10;
  o->max_backtracks = 30;
  o->init_mode = CELESTE_INIT_PLAIN;
  o->poll_every = 4;
  o->max_loops = 0;
  o->pred_rtol = 1e-8;
  o->armijo_c1 = 1e-4;
  o->u_box = 3.0;
}

int celeste_lbfgs_fit(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_lbfgs_opts* opts,
                      celeste_fit_result* results, void* stream) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  return run_lbfgs(ctx, b, theta_inout, opts, results, pick(ctx, stream));
}

}  // extern "C"

// =============================================================================== surrogate glue

namespace {

struct HostBox {
  double lo, hi;
  int kind;   // 0 identity, 1 scaled logistic, 2 exp
};

HostBox host_box(int i, const double* u0, double u_box) {
  if (i == 0 || i == 1) return {u0[i] - u_box, u0[i] + u_box, 1};
  if (i == 2 || i == 3) return {1e-4, 1.0 - 1e-4, 1};
  if (i == 4) return {0.01, 0.99, 1};
  if (i == 6) return {0.2, 15.0, 1};
  if (i == 9 || i == 10 || i >= 19) return {0.0, 0.0, 2};
  return {0.0, 0.0, 0};
}

}  // namespace

extern "C" {

int celeste_ctx_set_surrogate(celeste_ctx* ctx, celeste_net* net) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  ctx->net = net;
  return CELESTE_OK;
}

int celeste_make_patches(celeste_ctx* ctx, const celeste_batch* b, const double* theta, void* out) {
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  if (!theta || !out) return fail(CELESTE_E_INVALID, "theta and out must not be NULL");
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const double* th = theta;
  if (b->mem_kind == CELESTE_MEM_HOST) {
    CHK(ensure(ctx->theta, sizeof(double) * NP * P.n_src));
    HIPCHK(hipMemcpyAsync(ctx->theta.p, theta, sizeof(double) * NP * P.n_src, hipMemcpyHostToDevice, st));
    th = as<double>(ctx->theta);
  }
  CHK(prepare(ctx, b, &P, st));
  HIPCHK(launch_patches(as<SrcDev>(ctx->srcs), P.n_src, as<ImgDev>(ctx->imgs), th, out, st));
  HIPCHK(hipStreamSynchronize(st));
  return CELESTE_OK;
}

int celeste_theta_to_psi(const double* theta, const double* u0, int64_t n, double u_box, double* psi) {
  if (!theta || !u0 || !psi || n < 0 || !(u_box > 0.0)) return fail(CELESTE_E_INVALID, "bad argument");
  for (int64_t s = 0; s < n; ++s)
    for (int i = 0; i < NP; ++i) {
      const HostBox bx = host_box(i, u0 + 2 * s, u_box);
      const double t = theta[s * NP + i];
      double v = t;
      if (bx.kind == 2) {
        v = std::log(t);
      } else if (bx.kind == 1) {
        const double span = bx.hi - bx.lo;
        const double x = std::min(std::max(t, bx.lo + 1e-9 * span), bx.hi - 1e-9 * span);
        const double f = (x - bx.lo) / span;
        v = std::log(f) - std::log1p(-f);
      }
      psi[s * NP + i] = v;
    }
  return CELESTE_OK;
}

int celeste_psi_to_theta(const double* psi, const double* u0, int64_t n, double u_box, double* theta) {
  if (!theta || !u0 || !psi || n < 0 || !(u_box > 0.0)) return fail(CELESTE_E_INVALID, "bad argument");
  for (int64_t s = 0; s < n; ++s)
    for (int i = 0; i < NP; ++i) {
      const HostBox bx = host_box(i, u0 + 2 * s, u_box);
      const double p = psi[s * NP + i];
      double v = p;
      if (bx.kind == 2) v = std::exp(p);
      else if (bx.kind == 1) v = bx.lo + (bx.hi - bx.lo) / (1.0 + std::exp(-p));
      theta[s * NP + i] = v;
    }
  return CELESTE_OK;
}

}  // extern "C"

// =============================================================================== crowded fields

namespace {

// Bounding boxes [x0, x1) x [y0, y1) of each source's patches (union over its images, in
// image-frame coordinates), for the colouring.
struct Box {
  int64_t x0, x1, y0, y1;
};
constexpr int64_t CELL = 128;   // grid cell of the colouring (>= the usual patch side)

bool overlap(const Box& a, const Box& b) { return a.x0 < b.x1 && b.x0 < a.x1 && a.y0 < b.y1 && b.y0 < a.y1; }

int64_t cell_key(int64_t cx, int64_t cy) { return (cx << 32) ^ (cy & 0xffffffffLL); }

int source_boxes(const celeste_batch* b, std::vector<Box>* out) {
  const int S = b->n_sources;
  if (b->image_offsets[0] != 0) return fail(CELESTE_E_INVALID, "image_offsets[0] must be 0");
  out->resize(S);
  for (int s = 0; s < S; ++s) {
    if (b->image_offsets[s + 1] <= b->image_offsets[s]) return fail(CELESTE_E_INVALID, "source %d has no images", s);
    Box bx{INT64_MAX, INT64_MIN, INT64_MAX, INT64_MIN};
    for (int64_t i = b->image_offsets[s]; i < b->image_offsets[s + 1]; ++i) {
      const celeste_image& im = b->images[i];
      const double ox = im.origin[0], oy = im.origin[1];
      if (!std::isfinite(ox) || !std::isfinite(oy) || std::fabs(ox) > 1e9 || std::fabs(oy) > 1e9 || im.h < 1 ||
          im.w < 1)
        return fail(CELESTE_E_INVALID, "image %lld: bad origin or shape", (long long)i);
      // non-negative cell coordinates: shift by 2^31 before the grid division
      const int64_t x0 = (int64_t)std::floor(ox) + ((int64_t)1 << 31), y0 = (int64_t)std::floor(oy) + ((int64_t)1 << 31);
      bx.x0 = std::min(bx.x0, x0);
      bx.y0 = std::min(bx.y0, y0);
      bx.x1 = std::max(bx.x1, x0 + im.w + (ox != std::floor(ox) ? 1 : 0));
      bx.y1 = std::max(bx.y1, y0 + im.h + (oy != std::floor(oy) ? 1 : 0));
    }
    (*out)[s] = bx;
  }
  return CELESTE_OK;
}

// No two images of the batch on the same field may overlap (single writer per field pixel).
int check_disjoint(const celeste_batch* b, const celeste_fields* f) {
  const int64_t n = b->image_offsets[b->n_sources];
  std::unordered_map<int64_t, std::vector<int64_t>> grid;
  for (int64_t i = 0; i < n; ++i) {
    const celeste_image& a = b->images[i];
    const int64_t ax = (int64_t)a.origin[0], ay = (int64_t)a.origin[1];
    const int64_t fkey = (int64_t)f->img_field[i] << 40;
    for (int64_t cy = ay / CELL; cy <= (ay + a.h - 1) / CELL; ++cy)
      for (int64_t cx = ax / CELL; cx <= (ax + a.w - 1) / CELL; ++cx) {
        auto& v = grid[fkey ^ (cx << 20) ^ cy];
        for (int64_t j : v) {
          const celeste_image& c = b->images[j];
          const int64_t bx = (int64_t)c.origin[0], by = (int64_t)c.origin[1];
          if (f->img_field[j] == f->img_field[i] && ax < bx + c.w && bx < ax + a.w && ay < by + c.h && by < ay + a.h)
            return fail(CELESTE_E_INVALID, "images %lld and %lld overlap in field %d", (long long)j, (long long)i,
                        f->img_field[i]);
        }
        v.push_back(i);
      }
  }
  return CELESTE_OK;
}

int check_fields(const celeste_batch* b, const Packed& P, const celeste_fields* f) {
  if (!f || !f->img_field || !f->mean || !f->var) return fail(CELESTE_E_INVALID, "fields and its arrays must not be NULL");
  if (b->mem_kind != CELESTE_MEM_DEVICE) return fail(CELESTE_E_INVALID, "crowded fields need CELESTE_MEM_DEVICE");
  if (f->n_fields < 1 || f->height < 1 || f->width < 1 || f->reserved != 0)
    return fail(CELESTE_E_INVALID, "bad field dimensions");
  for (int i = 0; i < P.n_img; ++i) {
    const celeste_image& im = b->images[i];
    const int fi = f->img_field[i];
    if (fi < 0 || fi >= f->n_fields) return fail(CELESTE_E_INVALID, "image %d: field index out of range", i);
    const double ox = im.origin[0], oy = im.origin[1];
    if (ox != std::floor(ox) || oy != std::floor(oy)) return fail(CELESTE_E_INVALID, "image %d: origin not integer", i);
    if (ox < 0 || oy < 0 || ox + im.w > f->width || oy + im.h > f->height)
      return fail(CELESTE_E_INVALID, "image %d: patch outside its field", i);
  }
  return CELESTE_OK;
}

int upload_theta(celeste_ctx* ctx, const celeste_batch* b, const Packed& P, const double* theta, const double** out,
                 hipStream_t st) {
  if (!theta) return fail(CELESTE_E_INVALID, "theta is NULL");
  std::vector<double> h(NP * (size_t)P.n_src);
  HIPCHK(hipMemcpyAsync(h.data(), theta, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int s = 0; s < P.n_src; ++s) CHK(check_theta(h.data() + (size_t)s * NP, s));
  *out = theta;
  (void)ctx;
  (void)b;
  return CELESTE_OK;
}

}  // namespace

extern "C" {

int celeste_render_fields(celeste_ctx* ctx, const celeste_batch* b, const double* theta, const celeste_fields* f) {
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_fields(b, P, f));
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const double* th = nullptr;
  CHK(upload_theta(ctx, b, P, theta, &th, st));
  CHK(prepare(ctx, b, &P, st, false));
  // tile -> images index (counting sort, images in source order within a tile)
  const int tx = (f->width + 31) / 32, ty = (f->height + 31) / 32;
  const int tpf = tx * ty;
  const int64_t n_tiles64 = (int64_t)tpf * f->n_fields;
  if (n_tiles64 > INT32_MAX / 2) return fail(CELESTE_E_INVALID, "too many tiles");
  const int n_tiles = (int)n_tiles64;
  std::vector<int> cnt(n_tiles + 1, 0);
  for (int i = 0; i < P.n_img; ++i) {
    const celeste_image& im = b->images[i];
    const int c0 = (int)im.origin[0], r0 = (int)im.origin[1];
    const int base = f->img_field[i] * tpf;
    for (int yy = r0 / 32; yy <= (r0 + im.h - 1) / 32; ++yy)
      for (int xx = c0 / 32; xx <= (c0 + im.w - 1) / 32; ++xx) cnt[base + yy * tx + xx + 1] += 1;
  }
  for (int t = 0; t < n_tiles; ++t) cnt[t + 1] += cnt[t];
  std::vector<int> pos(cnt.begin(), cnt.end() - 1), lst((size_t)cnt[n_tiles]);
  for (int i = 0; i < P.n_img; ++i) {
    const celeste_image& im = b->images[i];
    const int c0 = (int)im.origin[0], r0 = (int)im.origin[1];
    const int base = f->img_field[i] * tpf;
    for (int yy = r0 / 32; yy <= (r0 + im.h - 1) / 32; ++yy)
      for (int xx = c0 / 32; xx <= (c0 + im.w - 1) / 32; ++xx) lst[pos[base + yy * tx + xx]++] = i;
  }
  CHK(ensure(ctx->tile_off, sizeof(int) * cnt.size()));
  CHK(ensure(ctx->tile_img, sizeof(int) * std::max<size_t>(1, lst.size())));
  HIPCHK(hipMemcpyAsync(ctx->tile_off.p, cnt.data(), sizeof(int) * cnt.size(), hipMemcpyHostToDevice, st));
  if (!lst.empty())
    HIPCHK(hipMemcpyAsync(ctx->tile_img.p, lst.data(), sizeof(int) * lst.size(), hipMemcpyHostToDevice, st));
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  HIPCHK(launch_setup(imgs, P.n_img, th, nullptr, P.prof, as<float>(ctx->tables), P.tstride, st));
  HIPCHK(launch_render(as<int>(ctx->tile_off), as<int>(ctx->tile_img), n_tiles, imgs, as<float>(ctx->tables),
                       P.tstride, P.prof.n_exp, P.prof.n_dev, f->height, f->width, tx, tpf, f->mean, f->var, st));
  HIPCHK(hipStreamSynchronize(st));
  return CELESTE_OK;
}

int celeste_neighbour_arrays(celeste_ctx* ctx, const celeste_batch* b, const double* theta, const celeste_fields* f,
                             const int64_t* nbr_off, float* nbr_mean, float* nbr_var) {
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_fields(b, P, f));
  if (!nbr_off || !nbr_mean || !nbr_var) return fail(CELESTE_E_INVALID, "neighbour arrays must not be NULL");
  for (int i = 0; i < P.n_img; ++i)
    if (nbr_off[i] < 0) return fail(CELESTE_E_INVALID, "negative neighbour offset");
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const double* th = nullptr;
  CHK(upload_theta(ctx, b, P, theta, &th, st));
  CHK(prepare(ctx, b, &P, st, false));
  CHK(ensure(ctx->img_field, sizeof(int) * P.n_img));
  CHK(ensure(ctx->nbr_off, sizeof(long long) * P.n_img));
  HIPCHK(hipMemcpyAsync(ctx->img_field.p, f->img_field, sizeof(int) * P.n_img, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->nbr_off.p, nbr_off, sizeof(long long) * P.n_img, hipMemcpyHostToDevice, st));
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  HIPCHK(launch_setup(imgs, P.n_img, th, nullptr, P.prof, as<float>(ctx->tables), P.tstride, st));
  HIPCHK(launch_neighbours(imgs, P.n_img, as<int>(ctx->img_field), as<float>(ctx->tables), P.tstride, P.prof.n_exp,
                           P.prof.n_dev, f->height, f->width, f->mean, f->var, as<long long>(ctx->nbr_off), nbr_mean,
                           nbr_var, st));
  HIPCHK(hipStreamSynchronize(st));
  return CELESTE_OK;
}

int celeste_colour_sources(const celeste_batch* b, int32_t* colour, int32_t* n_colours) {
  if (!b || !b->image_offsets || !b->images) return fail(CELESTE_E_INVALID, "batch is NULL or incomplete");
  if (!colour || !n_colours) return fail(CELESTE_E_INVALID, "colour and n_colours must not be NULL");
  if (b->n_sources < 1) return fail(CELESTE_E_INVALID, "n_sources must be >= 1");
  std::vector<Box> box;
  CHK(source_boxes(b, &box));
  const int S = b->n_sources;
  std::unordered_map<int64_t, std::vector<int>> grid;
  std::vector<int> stamp;   // stamp[c] == s: colour c is taken by a neighbour of s
  int nc = 0;
  for (int s = 0; s < S; ++s) {
    const Box& a = box[s];
    for (int64_t cy = a.y0 / CELL; cy <= (a.y1 - 1) / CELL; ++cy)
      for (int64_t cx = a.x0 / CELL; cx <= (a.x1 - 1) / CELL; ++cx) {
        auto it = grid.find(cell_key(cx, cy));
        if (it == grid.end()) continue;
        for (int t : it->second)
          if (overlap(a, box[t])) stamp[colour[t]] = s;
      }
    int c = 0;
    while (c < nc && stamp[c] == s) ++c;
    if (c == nc) {
      ++nc;
      stamp.push_back(-1);
    }
    colour[s] = c;
    for (int64_t cy = a.y0 / CELL; cy <= (a.y1 - 1) / CELL; ++cy)
      for (int64_t cx = a.x0 / CELL; cx <= (a.x1 - 1) / CELL; ++cx) grid[cell_key(cx, cy)].push_back(s);
  }
  *n_colours = nc;
  return CELESTE_OK;
}

int celeste_update_fields(celeste_ctx* ctx, const celeste_batch* b, const double* theta_old, const double* theta_new,
                          const celeste_fields* f) {
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_fields(b, P, f));
  CHK(check_disjoint(b, f));
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const double *th_old = nullptr, *th_new = nullptr;
  CHK(upload_theta(ctx, b, P, theta_old, &th_old, st));
  CHK(upload_theta(ctx, b, P, theta_new, &th_new, st));
  CHK(prepare(ctx, b, &P, st, false));
  CHK(ensure(ctx->tables2, sizeof(float) * (size_t)P.tstride * P.n_img));
  CHK(ensure(ctx->img_field, sizeof(int) * P.n_img));
  HIPCHK(hipMemcpyAsync(ctx->img_field.p, f->img_field, sizeof(int) * P.n_img, hipMemcpyHostToDevice, st));
  const ImgDev* imgs = as<ImgDev>(ctx->imgs);
  HIPCHK(launch_setup(imgs, P.n_img, th_old, nullptr, P.prof, as<float>(ctx->tables), P.tstride, st));
  HIPCHK(launch_setup(imgs, P.n_img, th_new, nullptr, P.prof, as<float>(ctx->tables2), P.tstride, st));
  HIPCHK(launch_update_fields(imgs, P.n_img, as<int>(ctx->img_field), as<float>(ctx->tables),
                              as<float>(ctx->tables2), P.tstride, P.prof.n_exp, P.prof.n_dev, f->height, f->width,
                              f->mean, f->var, st));
  HIPCHK(hipStreamSynchronize(st));
  return CELESTE_OK;
}

int celeste_field_elbo(celeste_ctx* ctx, const celeste_batch* b, const double* theta, const celeste_fields* f,
                       const float* field_pixels, const double* field_sky, double* elbo_out) {
  Packed P;
  CHK(validate_and_pack(ctx, b, &P));
  CHK(check_fields(b, P, f));
  if (!field_pixels || !field_sky || !elbo_out)
    return fail(CELESTE_E_INVALID, "field_pixels, field_sky and elbo_out must not be NULL");
  for (int k = 0; k < f->n_fields; ++k)
    if (!(field_sky[k] > 0.0) || !std::isfinite(field_sky[k]))
      return fail(CELESTE_E_INVALID, "field %d: sky must be finite and > 0", k);
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const double* th = nullptr;
  CHK(upload_theta(ctx, b, P, theta, &th, st));
  const int S = P.n_src;
  const int64_t n = (int64_t)f->n_fields * f->height * f->width;
  const int per_block = 8192;
  const int64_t nb64 = (n + per_block - 1) / per_block;
  if (nb64 > INT32_MAX / 2) return fail(CELESTE_E_INVALID, "fields too large");
  const int nb = (int)nb64;
  CHK(ensure(ctx->fsky, sizeof(double) * f->n_fields));
  CHK(ensure(ctx->o_elbo, sizeof(double) * S));
  CHK(ensure(ctx->partials, sizeof(double) * (size_t)nb));
  HIPCHK(hipMemcpyAsync(ctx->fsky.p, field_sky, sizeof(double) * f->n_fields, hipMemcpyHostToDevice, st));
  HIPCHK(launch_prior_term(th, S, P.prior, as<double>(ctx->o_elbo), st));
  HIPCHK(launch_field_terms(field_pixels, f->mean, f->var, as<double>(ctx->fsky), f->height, f->width, f->n_fields,
                            per_block, nb, as<double>(ctx->partials), st));
  std::vector<double> pri(S), part(nb);
  HIPCHK(hipMemcpyAsync(pri.data(), ctx->o_elbo.p, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(part.data(), ctx->partials.p, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double tot = 0.0;
  for (double v : part) tot += v;
  for (double v : pri) tot += v;
  *elbo_out = tot;
  return CELESTE_OK;
}

int celeste_start(celeste_ctx* ctx, const celeste_batch* b, double* theta_inout, const celeste_fit_opts* opts,
                  double* elbo_out) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  return run_fit(ctx, b, theta_inout, opts, nullptr, ctx->stream, true, elbo_out, true);
}

}  // extern "C"

// =============================================================================== autotuner

namespace {

std::string tune_key(celeste_ctx* ctx, const Packed& P, const celeste_batch* b) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) std::memset(&prop, 0, sizeof(prop));
  int max_psf = 1;
  double px = 0.0;
  for (int i = 0; i < P.n_img; ++i) {
    max_psf = std::max(max_psf, b->images[i].n_psf);
    px += (double)b->images[i].h * b->images[i].w;
  }
  const int cls = (int)std::lround(std::log2(std::max(1.0, px / std::max(1, P.n_img))));
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s|%s|cu%d|exp%d|dev%d|psf%d|px2^%d", prop.name, prop.gcnArchName,
                prop.multiProcessorCount, P.prof.n_exp, P.prof.n_dev, max_psf, cls);
  std::string k(buf);
  for (char& c : k)
    if (c == ' ' || c == '\t' || c == '\n') c = '_';
  return k;
}

// 1 if the cache holds the key (fills r), 0 if not or the file does not exist yet.
int tune_cache_read(const char* path, const std::string& key, celeste_tune_result* r) {
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  char line[1024];
  int found = 0;
  while (std::fgets(line, sizeof(line), f)) {
    char k[600];
    celeste_tune_result t{};
    if (std::sscanf(line, "%599s %d %d %d %d %d %d %lf %lf", k, &t.chunk_px, &t.block, &t.variant, &t.tile_w,
                    &t.value_block, &t.value_tile_w, &t.full_ms, &t.value_ms) == 9 &&
        key == k) {
      *r = t;   // the last matching line wins
      found = 1;
    }
  }
  std::fclose(f);
  return found;
}

int tune_cache_append(const char* path, const std::string& key, const celeste_tune_result& r) {
  FILE* f = std::fopen(path, "a");
  if (!f) return fail(CELESTE_E_INVALID, "autotune cache %s: cannot open for appending", path);
  std::fprintf(f, "%s %d %d %d %d %d %d %.6f %.6f\n", key.c_str(), r.chunk_px, r.block, r.variant, r.tile_w,
               r.value_block, r.value_tile_w, r.full_ms, r.value_ms);
  std::fclose(f);
  return CELESTE_OK;
}

int log2_tile(int w) {
  for (int k = 3; k <= 6; ++k)
    if (w == (1 << k)) return k;
  return -1;
}

// Minimum over `reps` timed launches (after one untimed) of a launch sequence, in ms.
template <class F>
int time_min(hipStream_t st, int reps, F launch, double* best) {
  hipEvent_t a = nullptr, z = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&z));
  int rc = CELESTE_OK;
  *best = 1e300;
  for (int r = 0; r <= reps && rc == CELESTE_OK; ++r) {
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(z, st);
    if (e == hipSuccess) e = hipEventSynchronize(z);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, z);
    if (e != hipSuccess) rc = fail(CELESTE_E_DEVICE, "autotune launch: %s", hipGetErrorString(e));
    else if (r > 0) *best = std::min(*best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  return rc;
}

int autotune(celeste_ctx* ctx, const celeste_batch* b, const double* theta, int64_t sample_px,
             const char* cache_path, celeste_tune_result* out) {
  if (!ctx) return fail(CELESTE_E_INVALID, "context is NULL");
  if (!theta) return fail(CELESTE_E_INVALID, "theta is NULL");
  Packed P0;
  CHK(validate_and_pack(ctx, b, &P0));
  HIPCHK(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  const std::string key = tune_key(ctx, P0, b);
  celeste_tune_result r{};
  if (cache_path && tune_cache_read(cache_path, key, &r)) {
    const int tl = log2_tile(r.tile_w), vl = log2_tile(r.value_tile_w);
    if (tl < 0 || vl < 0 || (r.block != 128 && r.block != 256) || (r.value_block != 128 && r.value_block != 256) ||
        r.variant < 0 || r.variant > 7 || r.chunk_px < 64 || r.chunk_px > (1 << 24))
      return fail(CELESTE_E_INVALID, "autotune cache %s: bad entry for %s", cache_path, key.c_str());
    ctx->chunk_px = r.chunk_px;
    ctx->block = r.block;
    ctx->variant = r.variant;
    ctx->tile_log2 = tl;
    ctx->vblock = r.value_block;
    ctx->vtile_log2 = vl;
    r.from_cache = 1;
    if (out) *out = r;
    return CELESTE_OK;
  }
  // theta on the host, for the sample
  const int S = b->n_sources;
  std::vector<double> th((size_t)S * NP);
  if (b->mem_kind == CELESTE_MEM_HOST)
    std::memcpy(th.data(), theta, sizeof(double) * th.size());
  else {
    HIPCHK(hipMemcpyAsync(th.data(), theta, sizeof(double) * th.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int s = 0; s < S; ++s) CHK(check_theta(th.data() + (size_t)s * NP, s));
  // every k-th source, about sample_px pixels
  if (sample_px <= 0) sample_px = 60000000;
  int64_t total = 0;
  for (int64_t i = 0; i < b->image_offsets[S]; ++i) total += (int64_t)b->images[i].h * b->images[i].w;
  const int64_t stride = std::max<int64_t>(1, total / std::max<int64_t>(1, sample_px));
  std::vector<int64_t> offs{0};
  std::vector<celeste_image> imgs;
  std::vector<double> ths;
  for (int64_t s = 0; s < S; s += stride) {
    for (int64_t i = b->image_offsets[s]; i < b->image_offsets[s + 1]; ++i) {
      imgs.push_back(b->images[i]);
      r.sample_px += (int64_t)b->images[i].h * b->images[i].w;
    }
    offs.push_back((int64_t)imgs.size());
    ths.insert(ths.end(), th.begin() + s * NP, th.begin() + (s + 1) * NP);
  }
  r.sample_sources = (int64_t)offs.size() - 1;
  celeste_batch sub = *b;
  sub.n_sources = (int32_t)r.sample_sources;
  sub.image_offsets = offs.data();
  sub.images = imgs.data();
  CHK(ensure(ctx->theta, sizeof(double) * ths.size()));
  HIPCHK(hipMemcpyAsync(ctx->theta.p, ths.data(), sizeof(double) * ths.size(), hipMemcpyHostToDevice, st));
  const double* th_dev = as<double>(ctx->theta);

  // every return before the end leaves the context's work-item size as it was
  struct ChunkGuard {
    celeste_ctx* c;
    int saved;
    ~ChunkGuard() { c->chunk_px = saved; }
  } guard{ctx, ctx->chunk_px};
  const int chunks[] = {4096, 8192, 16384};
  const int variants[] = {2, 3, 6, 7};
  struct Cand {
    double ms;
    int chunk, block, variant, tl;
    bool is_default() const { return chunk == 4096 && block == 256 && variant == 3 && tl == 3; }
  };
  std::vector<Cand> cands;
  int rc = CELESTE_OK;
  for (int chunk : chunks) {
    ctx->chunk_px = chunk;
    Packed P;
    rc = validate_and_pack(ctx, &sub, &P);
    if (rc == CELESTE_OK) rc = prepare(ctx, &sub, &P, st);
    if (rc != CELESTE_OK) break;
    const ImgDev* di = as<ImgDev>(ctx->imgs);
    float* tables = as<float>(ctx->tables);
    HIPCHK(launch_setup(di, P.n_img, th_dev, nullptr, P.prof, tables, P.tstride, st));
    for (int block : {128, 256})
      for (int variant : variants)
        for (int tl = 3; tl <= 6 && rc == CELESTE_OK; ++tl) {
          double ms = 0.0;
          rc = time_min(st, 3, [&]() {
            return launch_eval_full(as<WorkItem>(ctx->items), P.n_items, di, tables, P.tstride, P.prof.n_exp,
                                    P.prof.n_dev, nullptr, as<double>(ctx->partials), block,
                                    variant | (ctx->fp64_sums ? 8 : 0), tl, ctx->e_zero, st);
          }, &ms);
          r.n_candidates += 1;
          double& unit_best = (variant & 4) ? r.matrix_full_ms : r.vector_full_ms;
          if (rc == CELESTE_OK && (unit_best == 0.0 || ms < unit_best)) unit_best = ms;
          if (rc == CELESTE_OK) cands.push_back(Cand{ms, chunk, block, variant, tl});
        }
    if (rc != CELESTE_OK) break;
  }
  if (rc != CELESTE_OK) return rc;
  if (cands.empty()) return fail(CELESTE_E_DEVICE, "autotune: no candidate could be timed");
  // the four fastest and the default again, nine launches each, in one pass: candidates within a
  // few per cent of each other are ordered by more than one noisy minimum, and the default is
  // timed beside them, so the pick is never slower than the default by the pass's own timings
  std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  {
    std::vector<Cand> fin(cands.begin(), cands.begin() + std::min<size_t>(4, cands.size()));
    bool has_default = false;
    for (const Cand& c : fin) has_default = has_default || c.is_default();
    if (!has_default)
      for (const Cand& c : cands)
        if (c.is_default()) fin.push_back(c);
    cands.swap(fin);
  }
  std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.chunk < y.chunk; });
  {
    int prepared = 0;
    Packed P;
    for (Cand& c : cands) {
      if (c.chunk != prepared) {
        ctx->chunk_px = c.chunk;
        CHK(validate_and_pack(ctx, &sub, &P));
        CHK(prepare(ctx, &sub, &P, st));
        HIPCHK(launch_setup(as<ImgDev>(ctx->imgs), P.n_img, th_dev, nullptr, P.prof, as<float>(ctx->tables),
                            P.tstride, st));
        prepared = c.chunk;
      }
      const ImgDev* di = as<ImgDev>(ctx->imgs);
      float* tables = as<float>(ctx->tables);
      CHK(time_min(st, 9, [&]() {
        return launch_eval_full(as<WorkItem>(ctx->items), P.n_items, di, tables, P.tstride, P.prof.n_exp,
                                P.prof.n_dev, nullptr, as<double>(ctx->partials), c.block,
                                c.variant | (ctx->fp64_sums ? 8 : 0), c.tl, ctx->e_zero, st);
      }, &c.ms));
      if (c.is_default()) r.default_full_ms = c.ms;
    }
  }
  {
    // fastest of the pass; on a tie the default stays
    const Cand* pick = nullptr;
    for (const Cand& c : cands)
      if (!pick || c.ms < pick->ms || (c.ms == pick->ms && c.is_default())) pick = &c;
    r.full_ms = pick->ms;
    r.chunk_px = pick->chunk;
    r.block = pick->block;
    r.variant = pick->variant;
    r.tile_w = 1 << pick->tl;
  }
  // value kernel on the chosen work items
  ctx->chunk_px = r.chunk_px;
  {
    Packed P;
    CHK(validate_and_pack(ctx, &sub, &P));
    CHK(prepare(ctx, &sub, &P, st));
    const ImgDev* di = as<ImgDev>(ctx->imgs);
    float* tables = as<float>(ctx->tables);
    HIPCHK(launch_setup(di, P.n_img, th_dev, nullptr, P.prof, tables, P.tstride, st));
    double vbest = 1e300;
    for (int vblock : {128, 256})
      for (int tl = 3; tl <= 6; ++tl) {
        double ms = 0.0;
        CHK(time_min(st, 3, [&]() {
          return launch_eval_value(as<WorkItem>(ctx->items), P.n_items, di, tables, P.tstride, P.prof.n_exp,
                                   P.prof.n_dev, nullptr, as<double>(ctx->partials), vblock, r.variant, tl, st);
        }, &ms));
        r.n_candidates += 1;
        if (vblock == 256 && tl == 3 && r.chunk_px == 4096) r.default_value_ms = ms;
        if (ms < vbest) {
          vbest = ms;
          r.value_ms = ms;
          r.value_block = vblock;
          r.value_tile_w = 1 << tl;
        }
      }
  }
  if (r.chunk_px != 4096) {
    // the default's value-kernel time on its own work items
    ctx->chunk_px = 4096;
    Packed P;
    CHK(validate_and_pack(ctx, &sub, &P));
    CHK(prepare(ctx, &sub, &P, st));
    const ImgDev* di = as<ImgDev>(ctx->imgs);
    float* tables = as<float>(ctx->tables);
    HIPCHK(launch_setup(di, P.n_img, th_dev, nullptr, P.prof, tables, P.tstride, st));
    CHK(time_min(st, 3, [&]() {
      return launch_eval_value(as<WorkItem>(ctx->items), P.n_items, di, tables, P.tstride, P.prof.n_exp,
                               P.prof.n_dev, nullptr, as<double>(ctx->partials), 256, 3, 3, st);
    }, &r.default_value_ms));
  }
  guard.saved = r.chunk_px;  // the guard leaves the chosen size on the context
  ctx->block = r.block;
  ctx->variant = r.variant;
  ctx->tile_log2 = log2_tile(r.tile_w);
  ctx->vblock = r.value_block;
  ctx->vtile_log2 = log2_tile(r.value_tile_w);
  if (cache_path) CHK(tune_cache_append(cache_path, key, r));
  if (out) *out = r;
  return CELESTE_OK;
}

}  // namespace

extern "C" int celeste_autotune(celeste_ctx* ctx, const celeste_batch* batch, const double* theta, int64_t sample_px,
                                const char* cache_path, celeste_tune_result* out) {
  return autotune(ctx, batch, theta, sample_px, cache_path, out);
}
