// Internal device-side layouts of libceleste (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/celeste.h"

namespace celeste {

constexpr int NP = 27;       // natural parameters per source
constexpr int NZ = 11;       // per-image z-space: a, m_s, v_s, m_g, v_g, p_x, p_y, e_dev, e_axis, e_angle, e_scale
constexpr int NACC = 1 + NZ + NZ * (NZ + 1) / 2;   // value, gradient, upper-triangle Hessian = 78

// Per-image device metadata, packed from celeste_image by the host.
struct ImgDev {
  const float* pix;
  const float* nbr_mean;
  const float* nbr_var;
  int32_t h, w, pitch, band;
  int32_t n_psf, src;
  int32_t item_begin, item_end;   // work items covering this image
  int32_t nbr_pitch, pad_;        // row stride of the neighbour arrays
  double origin[2];
  double wcs[6];
  double sky, calib;
  double psf[CELESTE_MAX_PSF][6];
};

// One unit of pixel work: a band of rows [row_begin, row_end) of one image, all columns.
// The pixel kernels walk a band in 8x8 tiles, one tile per wavefront step.
struct WorkItem {
  int32_t img, src, row_begin, row_end;
};
constexpr int TILE = 8;

// Source -> images / work items (CSR, contiguous).
struct SrcDev {
  int32_t img_begin, img_end, item_begin, item_end;
  int64_t npix;                   // pixels over all the source's images
};

// Prior with the colour covariance inverse and log-determinant precomputed (FP64).
struct PriorDev {
  double p_star;
  double r_mean[2], r_var[2];
  double c_mean[2][4];
  double c_inv[2][4][4];
  double c_logdet[2];
  double c_diag[2][4];       // diagonal of the colour covariance (plain start)
};

struct ProfDev {
  int32_t n_exp, n_dev;
  double amp[2 * CELESTE_MAX_PROTO];   // exp components first, then dev
  double var[2 * CELESTE_MAX_PROTO];
};

// Per-image setup table (FP32, written by the setup kernel, read with wave-uniform loads).
namespace tab {
// header
constexpr int PSX = 0, PSY = 1, CALIB = 2, SKY = 3, CS = 4, CG = 5, MU_S = 6, MU_G = 7;
constexpr int KS = 8, KG = 9, KSG = 10, KA_S = 11, KA_G = 12, KA_SG = 13, KV_S = 14, KV_G = 15;
constexpr int EDEV = 16;
constexpr int KS_AA = 17, KS_AM = 18, KS_AV = 19, KS_MM = 20, KS_MV = 21, KS_VV = 22;
constexpr int KG_AA = 23, KG_AM = 24, KG_AV = 25, KG_MM = 26, KG_MV = 27, KG_VV = 28;
constexpr int KSG_AA = 29, KSG_AM = 30, KSG_AV = 31;
constexpr int NPSF = 32;                 // stored as float
// shape-derivative contraction coefficients
constexpr int W1 = 64;                   // [3 eta][3]: (W_xx/2, W_xy, W_yy/2) of dW/deta
constexpr int W4 = 73;                   // [6 pairs][5]: B4 contraction
constexpr int W2 = 103;                  // [6 pairs][3]: (W_xx/2, W_xy, W_yy/2) of d2W/deta deta'
constexpr int STAR = 128;                // [CELESTE_MAX_PSF][16]
constexpr int STAR_REC = 16;
constexpr int GAL = 192;                 // [n_psf][n_exp + n_dev][GAL_REC]
constexpr int GAL_REC = 24;
// galaxy record fields
constexpr int R_C0 = 0, R_QXX = 1, R_QXY = 2, R_QYY = 3, R_PXX = 4, R_PXY = 5, R_PYY = 6, R_NU = 7;
constexpr int R_3PXX = 8, R_3PYY = 9, R_2PXY = 10, R_6PXX = 11, R_6PYY = 12, R_3PXY = 13, R_4PXY = 14;
constexpr int R_K4A = 15, R_K4B = 16, R_K4C = 17, R_K4D = 18, R_K4E = 19;
// star record fields: c0, qxx, qxy, qyy, Pxx, Pxy, Pyy, xi_x, xi_y
constexpr int S_XIX = 7, S_XIY = 8;
// bound of the galaxy components of one PSF component: each has log2 density at most
// S_GC0 + S_GMU |d|^2 at offset d from the PSF component's centre (S_GMU < 0)
constexpr int S_GC0 = 9, S_GMU = 10;
}  // namespace tab

inline int table_stride(int max_psf, int n_exp, int n_dev) {
  int n = tab::GAL + max_psf * (n_exp + n_dev) * tab::GAL_REC;
  return (n + 15) & ~15;
}

// ---------------------------------------------------------------- device work queue
// The work items of the sources whose flag is set, in source and item order, rebuilt on the
// device before each phase of a fit iteration; persistent pixel kernels draw the list's entries
// in turn from a shared counter, so their grids cover only the work of sources still being
// fitted and uneven items balance across the blocks (the value+gradient+Hessian kernel; the
// value kernel's items are too cheap to repay the draw).
struct WorkQueue {
  int* items;       // capacity n_items: work-item indices
  int* hdr;         // [0]: entries, [1]: next entry to draw
  const SrcDev* srcs;
};
hipError_t launch_build_queue(WorkQueue q, int n_src, const int* flag, hipStream_t st);
// The calling block's next work item, or -1 once the list is drawn (the same value on every
// thread; the leading barrier keeps the block's shared buffers of the previous item intact
// until every thread has finished with them).
__device__ __forceinline__ int queue_next(const WorkQueue& q) {
  __shared__ int pos;
  __syncthreads();
  if (threadIdx.x == 0) pos = atomicAdd(q.hdr + 1, 1);
  __syncthreads();
  const int w = pos;
  return w < q.hdr[0] ? q.items[w] : -1;
}

// ---------------------------------------------------------------- launch wrappers
hipError_t launch_setup(const ImgDev* imgs, int n_img, const double* theta, const int* src_flag,
                        ProfDev prof, float* tables, int tstride, hipStream_t st);
// log n! table for the theta-independent pixel constants (LFACT_N doubles), and the pass that
// checks every pixel / neighbour value (bad |= 1 on a negative or non-finite one) and writes
// each image's constant sum x log E_bg - E_bg - log x!.
constexpr int LFACT_N = 1 << 16;
hipError_t launch_lfact(double* table, hipStream_t st);
hipError_t launch_check_const(const ImgDev* imgs, int n_img, const double* lfact, double* img_const, int* bad,
                              hipStream_t st);
// tw_log2: log2 of the pixel-tile width (3..6; tiles hold 64 pixels).  kept: nullptr for
// dense work items; for a pixel subsample, the first rows of the kept 8-row blocks, and each
// item's [row_begin, row_end) indexes this list instead of rows.
// e_zero: a component whose log2 density is below e_zero on every lane of a tile is exactly 0
// there and is skipped (see launch_exp2_probe).
// queue: NULL = one block per work item (blocks of unflagged sources exit at once); else a
// persistent grid of min(n_items, persistent_grid) blocks drawing the flagged sources' items from
// the queue (src_flag is then not read).
hipError_t launch_eval_full(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables,
                            int tstride, int n_exp, int n_dev, const int* src_flag, double* partials,
                            int block, int variant, int tw_log2, float e_zero, hipStream_t st,
                            const int* kept = nullptr, const WorkQueue* queue = nullptr,
                            int persistent_grid = 0);
// Blocks of the value+gradient+Hessian kernel instance for (block, variant, n_exp, n_dev) that one
// compute unit keeps resident (register and LDS budget of the instance).
hipError_t eval_full_blocks_per_cu(int block, int variant, int n_exp, int n_dev, int* blocks);
// Value and z-gradient only: one partial of NGRAD = 1 + NZ doubles per work item (value, 11
// gradient entries); arguments as launch_eval_full (variant: bit 1 only).
constexpr int NGRAD = 1 + NZ;
hipError_t launch_eval_grad(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables,
                            int tstride, int n_exp, int n_dev, const int* src_flag, double* partials,
                            int block, int variant, int tw_log2, float e_zero, hipStream_t st,
                            const int* kept = nullptr);
// out[i] = the pixel kernels' exp2(in[i]) on the device (i < n).
hipError_t launch_exp2_probe(const float* in, float* out, int n, hipStream_t st);
hipError_t launch_eval_value(const WorkItem* items, int n_items, const ImgDev* imgs, const float* tables,
                             int tstride, int n_exp, int n_dev, const int* src_flag, double* partials,
                             int block, int variant, int tw_log2, hipStream_t st,
                             const int* kept = nullptr);
// px_weight scales every image's pixel partials (not its theta-free constant): 1/p for a
// pixel subsample whose work items cover only the kept rows.
hipError_t launch_reduce_full(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                              const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                              double* elbo, double* grad, double* hess, unsigned long long* px_ctr,
                              hipStream_t st, double px_weight = 1.0);
// Value and natural gradient per source from gradient partials (NGRAD per work item).
hipError_t launch_reduce_grad(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                              const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                              double* elbo, double* grad, unsigned long long* px_ctr, hipStream_t st,
                              double px_weight = 1.0);
hipError_t launch_reduce_value(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* partials,
                               const double* img_const, const double* theta, PriorDev prior, const int* src_flag,
                               double* elbo, unsigned long long* px_ctr, hipStream_t st,
                               double px_weight = 1.0);

hipError_t launch_render(const int* tile_off, const int* tile_img, int n_tiles, const ImgDev* imgs,
                         const float* tables, int tstride, int n_exp, int n_dev, int H, int W, int tiles_x,
                         int tiles_per_field, float* mean, float* var, hipStream_t st);
hipError_t launch_neighbours(const ImgDev* imgs, int n_img, const int* img_field, const float* tables, int tstride,
                             int n_exp, int n_dev, int H, int W, const float* mean, const float* var,
                             const long long* nbr_off, float* nbr_mean, float* nbr_var, hipStream_t st);

hipError_t launch_update_fields(const ImgDev* imgs, int n_img, const int* img_field, const float* t_old,
                                const float* t_new, int tstride, int n_exp, int n_dev, int H, int W, float* mean,
                                float* var, hipStream_t st);
hipError_t launch_field_terms(const float* x, const float* mean, const float* var, const double* sky, int H, int W,
                              int n_fields, int per_block, int n_blocks, double* partials, hipStream_t st);
hipError_t launch_prior_term(const double* theta, int n_src, PriorDev prior, double* out, hipStream_t st);

// ---------------------------------------------------------------- trust-region state
struct FitDev {
  double* theta;        // S x 27 current (natural)
  double* psi;          // S x 27 current (unconstrained)
  double* u0;           // S x 2 box centre
  double* theta_trial;  // S x 27
  double* g;            // S x 27 natural gradient at current
  double* H;            // S x 729 natural Hessian at current
  double* V;            // S x 729 eigenvectors of the previous trust-region model (warm start)
  double* g_trial;      // S x 27 natural gradient at the trial point (trial derivatives)
  double* H_trial;      // S x 729 natural Hessian at the trial point (trial derivatives)
  double* p;            // S x 27 step (psi)
  double* f;            // S current ELBO (from the evaluation at which the current point was accepted)
  double* f_full;       // S ELBO from the full pass
  double* f_trial;      // S
  double* pred;         // S
  double* delta;        // S
  double* pnorm;        // S
  int* iter;            // S
  int* status;          // S
  int* active;          // S  1 while the source is being fitted
  int* need_full;       // S  1 when g/H must be computed at theta (with trial derivatives: from an
                        //    accepted step until k_take_trial hands over the trial point's g/H)
  int* n_full;          // S value+gradient+Hessian evaluations
  int* n_acc;           // S accepted steps
  int* flags;           // S  CELESTE_FLAG_* bits
  int* samp;            // S  1 while the source fits the pixel-subsampled objective (early phase)
  int* sw;              // S  1 in the iteration that moves the source from the subsampled to the full
                        //    objective (its trial point is its current point, to re-evaluate the ELBO)
  int* fa;              // S  gating flags of the current phase on the full objective ...
  int* fb;              // S  ... and on the subsampled one (launch_split)
  int* n_active;        // 1 counter
};

struct FitParams {
  int max_iter;
  double pred_rtol, curv_tol, delta0, delta_max, delta_min, eta, u_box;
  double switch_rtol;   // subsampled phase: move to the full objective when pred <= switch_rtol max(1, |L|)
  int tr_chol;          // solve the subproblem by Cholesky factorisations where B is positive definite
  int trial_derivs;     // the gradient and Hessian are evaluated at every trial point (k_accept counts
                        // each trial evaluation; launch_take_trial moves them to an accepted point)
  const SrcDev* srcs;   // with trial_derivs: the sources (pixel counts) ...
  unsigned long long* taken_px;   // ... and the pixels of accepted steps whose trial derivatives are taken
  unsigned long long* tr_ctr;   // subproblems solved: [0] interior step, [1] boundary step by Cholesky,
                                // [2] by the eigendecomposition; [3] Jacobi sweeps, [4] solves that
                                // reached the 40-sweep cap, [5] Newton steps on the multiplier
};

hipError_t launch_fit_init(FitDev st, int n_src, FitParams fp, hipStream_t s);
hipError_t launch_psi_to_theta(const float* psi, const double* theta_cat, double* theta_out, int n_src,
                               double u_box, hipStream_t s);
hipError_t launch_choose_start(FitDev st, int n_src, hipStream_t s);

// ---------------------------------------------------------------- L-BFGS state
// Beyond the fit state, whose fields keep their meaning with need_full = "needs a gradient",
// delta = the current step length and n_full = gradient evaluations.
constexpr int LBFGS_MAX_MEMORY = 32;
struct LbfgsDev {
  double* gpsi;     // S x 27 psi-gradient of -L at the current point
  double* S;        // S x memory x 27 curvature pairs: steps
  double* Y;        // S x memory x 27 curvature pairs: gradient changes
  double* rho;      // S x memory: 1 / s'y
  double* gp;       // S: g'p of the current direction
  int* n_pairs;     // S: stored pairs
  int* head;        // S: ring slot of the next pair
  int* ls;          // S: halvings in the current line search
  int* n_val;       // S: trial value evaluations
  int* in_ls;       // S: 1 while a trial point awaits its value
};

struct LbfgsParams {
  int max_iter, memory, max_backtracks;
  double pred_rtol, c1, u_box;
};

hipError_t launch_lbfgs_init(LbfgsDev X, int n_src, hipStream_t s);
// One wavefront per source with a new gradient: curvature pair, two-loop direction, stopping
// rule, first trial point.  n_active must be zeroed before launch_lbfgs_accept counts into it.
hipError_t launch_lbfgs_dir(FitDev F, LbfgsDev X, int n_src, LbfgsParams lp, hipStream_t s);
// One thread per source: sufficient-decrease test of the trial point, step or halving; counts the
// sources still being fitted into F.n_active.
hipError_t launch_lbfgs_accept(FitDev F, LbfgsDev X, int n_src, LbfgsParams lp, hipStream_t s);

// context accessors used by the network code, and the shared error slot
int ctx_device(const celeste_ctx* c);
hipStream_t ctx_stream(const celeste_ctx* c);
void set_error(const char* msg);
int surrogate_predict(celeste_net* net, const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* theta_cat,
                      float* psi_out, hipStream_t st);
hipError_t launch_patches(const SrcDev* srcs, int n_src, const ImgDev* imgs, const double* theta, void* out,
                          hipStream_t st);
hipError_t launch_plain_init(const SrcDev* srcs, int n_src, const ImgDev* imgs, PriorDev prior, double* theta,
                             hipStream_t s);
hipError_t launch_tr_step(FitDev st, int n_src, FitParams fp, hipStream_t s);
hipError_t launch_accept(FitDev st, int n_src, FitParams fp, hipStream_t s);
// Trial derivatives: sources whose step was just accepted take the gradient and Hessian of their
// trial point (g_trial, H_trial) and clear need_full.
hipError_t launch_take_trial(FitDev st, int n_src, hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
hipError_t launch_fill_int(int* p, int n, int value, hipStream_t s);
// fa[s] = flag[s] && !samp[s], fb[s] = flag[s] && samp[s] for every source
hipError_t launch_split(const int* flag, const int* samp, int* fa, int* fb, int n_src, hipStream_t s);
// Linear-response covariance per source from the natural gradient and Hessian at theta (u0:
// S x 2 position-box centres of the fit's coordinates); cov S x 27 x 27, status S.
hipError_t launch_lr_cov(const double* theta, const double* u0, double u_box, const double* grad, const double* hess,
                         int n_src, double* cov, int* status, hipStream_t s);

}  // namespace celeste
