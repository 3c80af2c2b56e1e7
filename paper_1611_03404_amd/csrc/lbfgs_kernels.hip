// Limited-memory BFGS on the device: the optimiser of the earlier Celeste (section III-B: it
// needed thousands of iterations on some sources, and trust-region Newton with the exact
// Hessian replaced it), kept to compare the two on the same data.  The same unconstrained
// coordinates psi as the trust-region fit; f = -ELBO is minimised.
//
// One loop step per source: if it accepted a step (need_full), the value+gradient pass has
// refreshed L and the natural gradient, and k_lbfgs_dir (one wavefront, lane j = coordinate j)
// stores the curvature pair (s = a p, y = g_new - g_old) when s'y > 1e-10 |s||y|, forms the
// direction by the two-loop recursion over the ring of pairs (Nocedal & Wright, Algorithm 7.4;
// initial scaling s'y / y'y of the newest pair; the unit-length steepest-descent step when no
// pair is stored or the direction does not descend, then without pairs), applies the stopping
// rule (the model's predicted gain -g'p/2 <= pred_rtol max(1, |L|)) and sets the first trial
// point psi + p.  The trial's value comes from the value pass; k_lbfgs_accept applies the
// sufficient-decrease condition f(psi + a p) <= f(psi) + c1 a g'p and either takes the step
// (the next loop step computes its gradient) or halves a (up to max_backtracks times).
#include <math.h>

#include "celeste_internal.h"
#include "psi_map.h"

namespace celeste {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void k_lbfgs_init(LbfgsDev X, int n_src) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  X.n_pairs[s] = 0;
  X.head[s] = 0;
  X.ls[s] = 0;
  X.n_val[s] = 0;
  X.in_ls[s] = 0;
  X.gp[s] = 0.0;
}

__global__ __launch_bounds__(64) void k_lbfgs_dir(FitDev F, LbfgsDev X, LbfgsParams lp) {
  __shared__ double al[LBFGS_MAX_MEMORY];
  const int s = blockIdx.x;
  if (!F.need_full[s]) return;
  const int j = threadIdx.x;
  const bool on = j < NP;
  const size_t o = (size_t)s * NP;
  const int m = lp.memory;
  double* Sb = X.S + (size_t)s * m * NP;
  double* Yb = X.Y + (size_t)s * m * NP;
  double* rho = X.rho + (size_t)s * m;
  const double* u0 = F.u0 + 2 * s;
  // psi-gradient of f = -L at the current point
  Box bx{0.0, 0.0, 0};
  double gn = 0.0;
  if (on) {
    bx = box_of(j, u0, lp.u_box);
    double d1, d2;
    to_theta1(F.psi[o + j], bx, &d1, &d2);
    gn = -d1 * F.g[o + j];
  }
  if (j == 0) F.n_full[s] += 1;
  const double gg = wave_sum(gn * gn);
  if (!isfinite(gg)) {
    if (j == 0) {
      F.status[s] = CELESTE_NONFINITE;
      F.active[s] = 0;
      F.need_full[s] = 0;
    }
    return;
  }
  int np_ = X.n_pairs[s], head = X.head[s];
  if (F.iter[s] > 0) {
    // the pair of the step just taken
    const double sv = on ? F.delta[s] * F.p[o + j] : 0.0;
    const double yv = on ? gn - X.gpsi[o + j] : 0.0;
    const double sy = wave_sum(sv * yv), ss = wave_sum(sv * sv), yy = wave_sum(yv * yv);
    if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
      if (on) {
        Sb[(size_t)head * NP + j] = sv;
        Yb[(size_t)head * NP + j] = yv;
      }
      if (j == 0) rho[head] = 1.0 / sy;
      head = (head + 1) % m;
      np_ = min(np_ + 1, m);
    }
  }
  if (on) X.gpsi[o + j] = gn;
  __syncthreads();   // rho of the new pair is visible to every lane
  // two-loop recursion: r = H gn, newest pair first, then oldest first
  double p = 0.0, gp = 0.0;
  bool ok = false;
  if (np_ > 0) {
    double q = gn;
    for (int k = 0; k < np_; ++k) {
      const int i = (head - 1 - k + 2 * m) % m;
      const double si = on ? Sb[(size_t)i * NP + j] : 0.0, yi = on ? Yb[(size_t)i * NP + j] : 0.0;
      const double a = rho[i] * wave_sum(si * q);
      if (j == 0) al[k] = a;
      q -= a * yi;
    }
    const int inew = (head - 1 + m) % m;
    const double sn = on ? Sb[(size_t)inew * NP + j] : 0.0, yn = on ? Yb[(size_t)inew * NP + j] : 0.0;
    double r = wave_sum(sn * yn) / wave_sum(yn * yn) * q;
    __syncthreads();
    for (int k = np_ - 1; k >= 0; --k) {
      const int i = (head - 1 - k + 2 * m) % m;
      const double si = on ? Sb[(size_t)i * NP + j] : 0.0, yi = on ? Yb[(size_t)i * NP + j] : 0.0;
      const double b = rho[i] * wave_sum(yi * r);
      r += (al[k] - b) * si;
    }
    p = -r;
    gp = wave_sum(gn * p);
    ok = gp < 0.0;
  }
  if (!ok) {
    // first step, or a direction that does not descend: unit-length steepest descent, no pairs
    np_ = 0;
    head = 0;
    p = -gn / sqrt(gg);
    gp = wave_sum(gn * p);
  }
  const double pred = -0.5 * gp;
  const double L = F.f[s];
  if (j == 0) {
    X.n_pairs[s] = np_;
    X.head[s] = head;
    X.gp[s] = gp;
    F.pred[s] = pred;
    F.need_full[s] = 0;
  }
  if (pred <= lp.pred_rtol * fmax(1.0, fabs(L))) {
    if (j == 0) {
      F.status[s] = CELESTE_CONVERGED;
      F.active[s] = 0;
    }
    return;
  }
  if (F.iter[s] >= lp.max_iter) {
    if (j == 0) F.active[s] = 0;   // status stays CELESTE_MAX_ITER
    return;
  }
  if (on) {
    F.p[o + j] = p;
    double d1, d2;
    F.theta_trial[o + j] = to_theta1(F.psi[o + j] + p, bx, &d1, &d2);
  }
  if (j == 0) {
    F.delta[s] = 1.0;
    X.ls[s] = 0;
    X.in_ls[s] = 1;
  }
}

__global__ void k_lbfgs_accept(FitDev F, LbfgsDev X, int n_src, LbfgsParams lp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  if (X.in_ls[s]) {
    const size_t o = (size_t)s * NP;
    const double* u0 = F.u0 + 2 * s;
    const double ft = F.f_trial[s], f = F.f[s], a = F.delta[s];
    X.n_val[s] += 1;
    // f is the ELBO L and the search minimises -L: -ft <= -f + c1 a g'p
    if (isfinite(ft) && -ft <= -f + lp.c1 * a * X.gp[s]) {
      for (int i = 0; i < NP; ++i) {
        F.psi[o + i] += a * F.p[o + i];
        double d1, d2;
        F.theta[o + i] = to_theta1(F.psi[o + i], box_of(i, u0, lp.u_box), &d1, &d2);
      }
      F.f[s] = ft;
      F.iter[s] += 1;
      F.n_acc[s] += 1;
      F.need_full[s] = 1;
      X.in_ls[s] = 0;
    } else if (X.ls[s] >= lp.max_backtracks) {
      F.status[s] = CELESTE_LINE_SEARCH_FAILED;
      F.active[s] = 0;
      X.in_ls[s] = 0;
    } else {
      const double an = 0.5 * a;
      F.delta[s] = an;
      X.ls[s] += 1;
      for (int i = 0; i < NP; ++i) {
        double d1, d2;
        F.theta_trial[o + i] = to_theta1(F.psi[o + i] + an * F.p[o + i], box_of(i, u0, lp.u_box), &d1, &d2);
      }
    }
  }
  if (F.active[s]) atomicAdd(F.n_active, 1);
}

}  // namespace

hipError_t launch_lbfgs_init(LbfgsDev X, int n_src, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbfgs_init, dim3((n_src + 255) / 256), dim3(256), 0, s, X, n_src);
  return hipGetLastError();
}

hipError_t launch_lbfgs_dir(FitDev F, LbfgsDev X, int n_src, LbfgsParams lp, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbfgs_dir, dim3(n_src), dim3(64), 0, s, F, X, lp);
  return hipGetLastError();
}

hipError_t launch_lbfgs_accept(FitDev F, LbfgsDev X, int n_src, LbfgsParams lp, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lbfgs_accept, dim3((n_src + 255) / 256), dim3(256), 0, s, F, X, n_src, lp);
  return hipGetLastError();
}

}  // namespace celeste
