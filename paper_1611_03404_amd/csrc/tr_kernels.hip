// Trust-region Newton state machine on the device (section III-B: Newton's method
// with updates constrained by a trust region, dense hand-derived Hessian, per
// source).  One wavefront per active source solves the 27x27 FP64 subproblem
//     maximise g'p + p'Hp/2  subject to |p| <= Delta     (unconstrained coordinates)
// through a cyclic Jacobi eigendecomposition of B = -H (parallel round-robin
// ordering, 14 disjoint rotations per round applied to B in LDS by 2x2 blocks, one
// barrier after the rotation parameters and one after the update), followed by the secular
// equation |(B + sI)^{-1} g| = Delta solved by safeguarded Newton on 1/|p(s)|
// (More-Sorensen), including the hard case.  Where B is positive definite, Cholesky
// factorisations of B + lam I give the step instead (the interior Newton step, or the
// boundary step by Newton's method on lam).  A separate kernel applies the
// ratio test and updates the radius, one thread per source.
#include <math.h>

#include "celeste_internal.h"
#include "psi_map.h"

namespace celeste {

namespace {

constexpr int NPAD = 28;   // 27 padded to an even order for the round-robin schedule

// ---------------------------------------------------------------- start of a fit
__global__ void k_fit_init(FitDev st, int n_src, FitParams fp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  double* th = st.theta + (size_t)s * NP;
  double* ps = st.psi + (size_t)s * NP;
  double* u0 = st.u0 + 2 * s;
  u0[0] = th[0];
  u0[1] = th[1];
  for (int i = 0; i < NP; ++i) {
    const Box b = box_of(i, u0, fp.u_box);
    ps[i] = to_psi1(th[i], b);
    double d1, d2;
    th[i] = to_theta1(ps[i], b, &d1, &d2);
  }
  double* V = st.V + (size_t)s * NP * NP;
  for (int i = 0; i < NP * NP; ++i) V[i] = (i % (NP + 1) == 0) ? 1.0 : 0.0;
  st.delta[s] = fp.delta0;
  st.iter[s] = 0;
  st.status[s] = CELESTE_MAX_ITER;
  st.active[s] = 1;
  st.need_full[s] = 1;
  st.n_full[s] = 0;
  st.n_acc[s] = 0;
  st.pred[s] = 0.0;
  st.samp[s] = 0;
  st.sw[s] = 0;
}

// Surrogate start: theta = T(psi) with the position box centred on the catalog position.
__global__ void k_psi_to_theta(const float* __restrict__ psi, const double* __restrict__ theta_cat,
                               double* __restrict__ theta_out, int n_src, double u_box) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  const double u0[2] = {theta_cat[(size_t)s * NP], theta_cat[(size_t)s * NP + 1]};
  for (int i = 0; i < NP; ++i) {
    double d1, d2;
    theta_out[(size_t)s * NP + i] = to_theta1((double)psi[(size_t)s * NP + i], box_of(i, u0, u_box), &d1, &d2);
  }
}

// Keep the surrogate start (theta_trial, ELBO f_trial) where its ELBO is finite and higher
// than the plain start's (theta, f); otherwise flag the fallback.
__global__ void k_choose_start(FitDev st, int n_src) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  const double fs = st.f_trial[s], fp = st.f[s];
  if (isfinite(fs) && (!isfinite(fp) || fs > fp)) {
    for (int i = 0; i < NP; ++i) st.theta[(size_t)s * NP + i] = st.theta_trial[(size_t)s * NP + i];
    st.f[s] = fs;
    st.flags[s] = 0;
  } else {
    st.flags[s] = CELESTE_FLAG_FALLBACK_USED;
  }
}

// A source whose starting ELBO is not finite is not fitted.
__global__ void k_fit_start(FitDev st, int n_src) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src) return;
  if (!isfinite(st.f[s])) {
    st.status[s] = CELESTE_NONFINITE;
    st.active[s] = 0;
    st.need_full[s] = 0;
  }
}

__device__ inline void pair_of(int round, int k, int* p, int* q) {
  // circle method over NPAD players: player NPAD-1 fixed, the rest rotate
  const int m = NPAD - 1;
  if (k == 0) {
    *p = m;
    *q = round;
  } else {
    *p = (round + k) % m;
    *q = (round - k + m) % m;
  }
}

__global__ __launch_bounds__(64) void k_tr(FitDev st, FitParams fp) {
  __shared__ double B[NPAD][NPAD + 1];
  __shared__ double V[NPAD][NPAD + 1];   // eigenvectors; the Cholesky paths' factor before that
  __shared__ double g[NPAD], gt[NPAD], lam[NPAD], pt[NPAD], d1s[NP];
  // a round's rotations: (p, q) and (cos, sin) side by side so that a reader loads each pair at once
  __shared__ double2 rcs[NPAD / 2];
  __shared__ int2 rpq[NPAD / 2];
  __shared__ int done;
  const int s = blockIdx.x;
  if (!st.active[s]) return;
  const int t = threadIdx.x;
  if (t == 0 && st.need_full[s]) {
    st.n_full[s] += 1;
    st.need_full[s] = 0;
  }
  const double* ps = st.psi + (size_t)s * NP;
  const double* gn = st.g + (size_t)s * NP;
  const double* Hn = st.H + (size_t)s * NP * NP;
  const double* u0 = st.u0 + 2 * s;
  // transform to unconstrained coordinates: g = t' g_n, B = -(D H D + diag(t'' g_n))
  __shared__ double d2s[NP];
  if (t < NP) {
    double d1, d2;
    to_theta1(ps[t], box_of(t, u0, fp.u_box), &d1, &d2);
    d1s[t] = d1;
    d2s[t] = d2;
  }
  __syncthreads();
  for (int k = t; k < NPAD * NPAD; k += 64) {
    const int i = k / NPAD, j = k - i * NPAD;
    double b = 0.0;
    if (i < NP && j < NP) {
      b = -d1s[i] * Hn[i * NP + j] * d1s[j];
      if (i == j) b -= d2s[i] * gn[i];
    }
    B[i][j] = b;
  }
  if (t < NPAD) g[t] = t < NP ? d1s[t] * gn[t] : 0.0;
  __syncthreads();
  auto wsum = [](double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return __shfl(x, 0);
  };
  const double delta = st.delta[s];
  // psi step; predicted gain; whether B is positive semi-definite to the curvature tolerance
  __shared__ double pst[NPAD], y[NPAD];
  double pred = 0.0;
  bool curv_ok = true;

  // ---- Cholesky paths.  Where B is positive definite, the subproblem's solution is
  // p(lam) = (B + lam I)^{-1} g with lam = 0 if |p(0)| <= Delta (the interior Newton step), and
  // otherwise the lam > 0 with |p(lam)| = Delta (optimality conditions of Nocedal & Wright,
  // Theorem 4.1).  That lam is found by Newton's method on 1/|p(lam)| - 1/Delta from lam = 0
  // (Nocedal & Wright, Algorithm 4.3, with q = L^{-1} p): the function is concave and increasing
  // for lam >= 0, so the iterates increase to the root and B + lam I stays positive definite.
  // Each step costs one Cholesky factorisation (right-looking in LDS, one column per step, the
  // forward substitution carried along) and two triangular solves, instead of the
  // eigendecomposition.  B indefinite or nearly singular (a pivot at most 1e-12 of the largest
  // diagonal entry), or a boundary step not within 1e-9 Delta of the radius after 30 Newton
  // steps, takes the eigendecomposition below.
  int path = 2;   // 0: interior step by Cholesky, 1: boundary step by Cholesky, 2: eigendecomposition
  if (fp.tr_chol) {
    double dmax = t < NP ? B[t][t] : -INFINITY;
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
    dmax = __shfl(dmax, 0);
    // V <- the Cholesky factor L of B + lam I (lower triangle), pst <- (B + lam I)^{-1} g (V holds
    // the eigenvectors only in the eigendecomposition path, which loads them afresh)
    auto factor_solve = [&](double lam) -> bool {
      for (int k = t; k < NP * NP; k += 64) {
        const int i = k / NP, j = k - i * NP;
        V[i][j] = B[i][j] + (i == j ? lam : 0.0);
      }
      if (t < NPAD) y[t] = g[t];
      __syncthreads();
      for (int k = 0; k < NP; ++k) {
        const double piv = V[k][k];   // the same value on every lane: the decision is uniform
        if (!(piv > 1e-12 * (dmax + lam))) return false;
        const double lkk = sqrt(piv);
        // (V[k][k] is read above by every lane and written only after the barrier)
        if (t > k && t < NP) V[t][k] /= lkk;
        if (t == k) y[k] /= lkk;
        __syncthreads();
        // trailing update of the lower triangle: lane (h, j) = (t / 32, t % 32) takes column j,
        // rows j + h, j + h + 2, ... (each entry updated by one lane)
        {
          const int j = t & 31;
          if (j > k && j < NP) {
            const double ljk = V[j][k];
            for (int i = j + (t >> 5); i < NP; i += 2) V[i][j] -= V[i][k] * ljk;
          }
        }
        if (t > k && t < NP) y[t] -= V[t][k] * y[k];
        if (t == k) V[k][k] = lkk;
        __syncthreads();
      }
      // back substitution L' p = y, one unknown per step
      for (int k = NP - 1; k >= 0; --k) {
        const double yk = y[k] / V[k][k];
        if (t == k) pst[k] = yk;
        if (t < k) y[t] -= V[k][t] * yk;
        __syncthreads();
      }
      return true;
    };
    if (dmax > 0.0 && factor_solve(0.0)) {
      double pn2 = wsum(t < NP ? pst[t] * pst[t] : 0.0);
      if (pn2 <= delta * delta) {
        path = 0;
        pred = 0.5 * wsum(t < NP ? g[t] * pst[t] : 0.0);
      } else {
        double lam = 0.0;
        int it = 0;
        for (; it < 30; ++it) {
          const double pn = sqrt(pn2);
          if (fabs(pn - delta) <= 1e-9 * delta) {
            path = 1;
            break;
          }
          // q = L^{-1} p by forward substitution, lane k keeping q_k
          if (t < NPAD) y[t] = t < NP ? pst[t] : 0.0;
          __syncthreads();
          double qk = 0.0;
          for (int k = 0; k < NP; ++k) {
            const double yk = y[k] / V[k][k];
            if (t == k) qk = yk;
            if (t > k && t < NP) y[t] -= V[t][k] * yk;
            __syncthreads();
          }
          const double qn2 = wsum(qk * qk);
          lam += (pn2 / qn2) * (pn - delta) / delta;
          if (!(lam >= 0.0)) lam = 0.0;   // only by rounding: |p(0)| > Delta
          if (!factor_solve(lam)) break;
          pn2 = wsum(t < NP ? pst[t] * pst[t] : 0.0);
        }
        if (t == 0 && fp.tr_ctr) atomicAdd(fp.tr_ctr + 5, (unsigned long long)it);
        // predicted gain g'p - p'Bp/2 with (B + lam I) p = g
        if (path == 1) pred = 0.5 * (wsum(t < NP ? g[t] * pst[t] : 0.0) + lam * pn2);
      }
    }
    __syncthreads();
  }

  if (path == 2) {
  // warm start: the eigenvectors of the previous model (identity at the first iteration)
  for (int k = t; k < NPAD * NPAD; k += 64) {
    const int i = k / NPAD, j = k - i * NPAD;
    V[i][j] = (i < NP && j < NP) ? st.V[(size_t)s * NP * NP + i * NP + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  // B <- V^T B V, nearly diagonal when the model changed little since the previous iteration;
  // the Jacobi rotations below accumulate into V, so V ends as the eigenvectors of the model.
  // Lane (h, j) = (t / 32, t % 32), j < NPAD, forms column j of each product for the rows
  // NPAD/2 h .. NPAD/2 h + NPAD/2 - 1 in registers (one LDS read of its own column and broadcast
  // reads of the other operand per r; every entry summed over r in increasing order) and stores
  // them after the barrier.
  {
    constexpr int HR = NPAD / 2;
    const int cj = t & 31, r0 = (t >> 5) * HR;
    const bool cl = cj < NPAD;
    double acc[HR];
#pragma unroll
    for (int i = 0; i < HR; ++i) acc[i] = 0.0;
    if (cl)
      for (int r = 0; r < NPAD; ++r) {
        const double v = V[r][cj];
#pragma unroll
        for (int i = 0; i < HR; ++i) acc[i] += B[r0 + i][r] * v;
      }
    __syncthreads();
    if (cl)
#pragma unroll
      for (int i = 0; i < HR; ++i) B[r0 + i][cj] = acc[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < HR; ++i) acc[i] = 0.0;
    if (cl)
      for (int r = 0; r < NPAD; ++r) {
        const double b = B[r][cj];
#pragma unroll
        for (int i = 0; i < HR; ++i) acc[i] += V[r][r0 + i] * b;
      }
    __syncthreads();
    if (cl)
#pragma unroll
      for (int i = 0; i < HR; ++i) B[r0 + i][cj] = acc[i];
    __syncthreads();
  }
  // symmetrise (the Hessian is assembled symmetrically; this removes rounding asymmetry)
  for (int k = t; k < NPAD * NPAD; k += 64) {
    const int i = k / NPAD, j = k - i * NPAD;
    if (i < j) {
      const double m = 0.5 * (B[i][j] + B[j][i]);
      B[i][j] = m;
      B[j][i] = m;
    }
  }
  __syncthreads();

  // ---- cyclic Jacobi, round-robin parallel ordering
  // A lane updates the same off-diagonal 2x2 blocks of B (by pair indices a < b) and the same
  // entries of V in every round, so their indices are decoded once here.
  constexpr int NPR = NPAD / 2;                     // disjoint rotations per round
  constexpr int NBLK = NPR * (NPR - 1) / 2;         // off-diagonal 2x2 blocks of B per round
  constexpr int BPL = (NBLK + 63) / 64, VPL = (NPR * NPAD + 63) / 64;
  int blk_a[BPL], blk_b[BPL];   // blk_a < 0: no block
#pragma unroll
  for (int u = 0; u < BPL; ++u) {
    const int k = t + 64 * u;
    blk_a[u] = -1;
    blk_b[u] = -1;
    if (k >= NBLK) continue;
    int a = 0, idx = k;
    while (idx >= NPR - 1 - a) {
      idx -= NPR - 1 - a;
      ++a;
    }
    blk_a[u] = a;
    blk_b[u] = a + 1 + idx;
  }
  int v_pr[VPL], v_r[VPL];      // rotation and row of the lane's entries of V (v_pr < 0: none)
#pragma unroll
  for (int u = 0; u < VPL; ++u) {
    const int k = t + 64 * u;
    v_pr[u] = k < NPR * NPAD ? k / NPAD : -1;
    v_r[u] = k - (k / NPAD) * NPAD;
  }
  int sweeps = 0;
  for (; sweeps < 40; ++sweeps) {
    double off = 0.0, fro = 0.0;
    for (int k = t; k < NPAD * NPAD; k += 64) {
      const int i = k / NPAD, j = k - i * NPAD;
      const double v = B[i][j] * B[i][j];
      fro += v;
      if (i != j) off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      fro += __shfl_xor(fro, o);
    }
    if (off <= 1e-30 * fro || fro == 0.0) break;
    for (int round = 0; round < NPAD - 1; ++round) {
      if (t < NPR) {
        int p, q;
        pair_of(round, t, &p, &q);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        const double apq = B[p][q], app = B[p][p], aqq = B[q][q];
        double c = 1.0, sn = 0.0, tt = 0.0;
        if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
          const double th = (aqq - app) / (2.0 * apq);
          tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          sn = tt * c;
        }
        rpq[t] = make_int2(p, q);
        rcs[t] = make_double2(c, sn);
        // the pair's own 2x2 block takes the rotated eigenvalue estimates and exact zeros; no other
        // lane reads these four entries in this round
        if (tt != 0.0) {
          B[p][p] = app - tt * apq;
          B[q][q] = aqq + tt * apq;
          B[p][q] = 0.0;
          B[q][p] = 0.0;
        }
      }
      __syncthreads();
      // B <- J^T B J and V <- V J in one pass: the off-diagonal 2x2 blocks of B (pair a's rows x
      // pair b's columns, a < b), each read and written by one lane, so no entry is touched twice;
      // a block is transformed columns first, then rows, and mirrored
#pragma unroll
      for (int u = 0; u < BPL; ++u) {
        const int a = blk_a[u], b = blk_b[u];
        if (a < 0) continue;
        const int2 pq1 = rpq[a], pq2 = rpq[b];
        const double2 cs1 = rcs[a], cs2 = rcs[b];
        const int p1 = pq1.x, q1 = pq1.y, p2 = pq2.x, q2 = pq2.y;
        const double c1 = cs1.x, s1 = cs1.y, c2 = cs2.x, s2 = cs2.y;
        const double x00 = B[p1][p2], x01 = B[p1][q2], x10 = B[q1][p2], x11 = B[q1][q2];
        const double y00 = c2 * x00 - s2 * x01, y01 = s2 * x00 + c2 * x01;
        const double y10 = c2 * x10 - s2 * x11, y11 = s2 * x10 + c2 * x11;
        const double z00 = c1 * y00 - s1 * y10, z10 = s1 * y00 + c1 * y10;
        const double z01 = c1 * y01 - s1 * y11, z11 = s1 * y01 + c1 * y11;
        B[p1][p2] = z00;
        B[p1][q2] = z01;
        B[q1][p2] = z10;
        B[q1][q2] = z11;
        B[p2][p1] = z00;
        B[q2][p1] = z01;
        B[p2][q1] = z10;
        B[q2][q1] = z11;
      }
#pragma unroll
      for (int u = 0; u < VPL; ++u) {
        const int pr = v_pr[u], r = v_r[u];
        if (pr < 0) continue;
        const int2 pq = rpq[pr];
        const double2 cs = rcs[pr];
        const int p = pq.x, q = pq.y;
        const double c = cs.x, sn = cs.y;
        const double vp = V[r][p], vq = V[r][q];
        V[r][p] = c * vp - sn * vq;
        V[r][q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
  }

  if (t == 0 && fp.tr_ctr) {
    atomicAdd(fp.tr_ctr + 3, (unsigned long long)sweeps);
    if (sweeps == 40) atomicAdd(fp.tr_ctr + 4, 1ull);
  }

  // ---- eigen-coordinates of g; the eigenvectors are kept for the next iteration's start
  if (t < NP) {
    lam[t] = B[t][t];
    double a = 0.0;
    for (int r = 0; r < NP; ++r) a += V[r][t] * g[r];
    gt[t] = a;
  }
  for (int k = t; k < NP * NP; k += 64) st.V[(size_t)s * NP * NP + k] = V[k / NP][k % NP];
  __syncthreads();

  // ---- secular equation, one eigen-coordinate per lane (lanes >= NP hold neutral values);
  // every reduction is broadcast from lane 0 so all lanes take the same decisions
  {
    const bool on = t < NP;
    const double li = on ? lam[t] : 0.0, gi = on ? gt[t] : 0.0;
    auto wmin = [](double x) {
      for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
      return __shfl(x, 0);
    };
    auto wmax = [](double x) {
      for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
      return __shfl(x, 0);
    };
    const double lam0 = wmin(on ? li : INFINITY);
    // first index holding the smallest eigenvalue
    const unsigned long long at_min = __ballot(on && li == lam0);
    const int i0 = __ffsll((long long)at_min) - 1;
    const double scale = fmax(1.0, wmax(on ? fabs(li) : 0.0));
    const double gn2 = wsum(gi * gi);
    auto pnorm2 = [&](double sv) {
      const double q = on ? gi / (li + sv) : 0.0;
      return wsum(q * q);
    };
    double sv = 0.0, pti = 0.0;
    bool hard = false;
    if (!(lam0 > 1e-14 * scale && pnorm2(0.0) <= delta * delta)) {
      const double slo = fmax(0.0, -lam0);
      const bool bottom = on && fabs(li - lam0) <= 1e-12 * scale;
      const double gbot2 = wsum(bottom ? gi * gi : 0.0);
      const double qrest = (on && !bottom) ? gi / (li + slo) : 0.0;
      const double prest2 = wsum(qrest * qrest);
      if (sqrt(gbot2) <= 1e-12 * fmax(1.0, sqrt(gn2)) && prest2 <= delta * delta) {
        hard = true;
        sv = slo;
        pti = bottom ? 0.0 : qrest;
        if (t == i0) pti += sqrt(fmax(delta * delta - prest2, 0.0));
      } else {
        double lo = slo, hi = slo + sqrt(gn2) / delta + 1.0;
        sv = (slo > 0.0) ? slo + 1e-12 * scale : 0.0;
        if (pnorm2(sv) > delta * delta) {
          for (int it = 0; it < 200; ++it) {
            const double den = li + sv;
            const double q = on ? gi / den : 0.0;
            const double a2 = wsum(q * q);
            const double b3 = wsum(on ? q * q / den : 0.0);
            const double pn = sqrt(a2);
            if (fabs(pn - delta) <= 1e-13 * delta) break;
            if (pn > delta) lo = fmax(lo, sv); else hi = fmin(hi, sv);
            // Newton on 1/|p(s)| - 1/Delta, kept inside the bracket
            double nx = sv + (a2 / b3) * (pn - delta) / delta;
            if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
            if (nx == sv) break;
            sv = nx;
          }
        }
        // else: |p| <= Delta just above the pole (nearly the hard case): keep sv
      }
    }
    if (!hard) pti = on ? gi / (li + sv) : 0.0;
    if (on) pt[t] = pti;
    pred = wsum(on ? gi * pti - 0.5 * li * pti * pti : 0.0);
    curv_ok = lam0 >= -fp.curv_tol * scale;
  }
  __syncthreads();
  // the step back in psi coordinates
  if (t < NP) {
    double a = 0.0;
    for (int i = 0; i < NP; ++i) a += V[t][i] * pt[i];
    pst[t] = a;
  }
  }   // eigendecomposition

  if (t == 0) {
    if (fp.tr_ctr) atomicAdd(fp.tr_ctr + path, 1ull);
    // convergence and iteration cap; on the subsampled objective, the switch to the full one
    const double f = st.f[s];
    int d = 0;
    if (st.samp[s]) {
      if (pred <= fp.switch_rtol * fmax(1.0, fabs(f))) {
        st.samp[s] = 0;
        st.sw[s] = 1;
        d = 2;
      } else if (st.iter[s] >= fp.max_iter) {
        st.status[s] = CELESTE_MAX_ITER;
        d = 1;
      }
    } else if (pred <= fp.pred_rtol * fmax(1.0, fabs(f)) && curv_ok) {
      st.status[s] = CELESTE_CONVERGED;
      d = 1;
    } else if (st.iter[s] >= fp.max_iter) {
      st.status[s] = CELESTE_MAX_ITER;
      d = 1;
    }
    st.pred[s] = pred;
    if (d == 1) st.active[s] = 0;
    done = d;
  }
  __syncthreads();
  if (done == 2) {
    // the switch: the trial point is the current point, whose ELBO on the full objective the
    // value pass evaluates (k_accept takes it as the current value)
    if (t < NP) st.theta_trial[(size_t)s * NP + t] = st.theta[(size_t)s * NP + t];
    return;
  }
  if (done) return;
  // ---- step in psi and the trial point
  double* pp = st.p + (size_t)s * NP;
  double* tht = st.theta_trial + (size_t)s * NP;
  double pn2 = 0.0;
  if (t < NP) {
    const double a = pst[t];
    pp[t] = a;
    double d1, d2;
    tht[t] = to_theta1(ps[t] + a, box_of(t, u0, fp.u_box), &d1, &d2);
    pn2 = a * a;
  }
  for (int o = 32; o > 0; o >>= 1) pn2 += __shfl_xor(pn2, o);
  if (t == 0) st.pnorm[s] = sqrt(pn2);
}

// Ratio test, radius update and acceptance; one thread per source.
__global__ void k_accept(FitDev st, int n_src, FitParams fp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_src || !st.active[s]) return;
  if (st.sw[s]) {
    // moved to the full objective: its value at the current point, then its gradient and Hessian
    st.sw[s] = 0;
    st.f[s] = st.f_trial[s];
    st.need_full[s] = 1;
    if (!isfinite(st.f[s])) {
      st.status[s] = CELESTE_NONFINITE;
      st.active[s] = 0;
      st.need_full[s] = 0;
      return;
    }
    atomicAdd(st.n_active, 1);
    return;
  }
  if (fp.trial_derivs) st.n_full[s] += 1;   // the trial point's value+gradient+Hessian evaluation
  const double ft = st.f_trial[s], f = st.f[s], pred = st.pred[s];
  const double rho = isfinite(ft) ? (ft - f) / pred : -INFINITY;
  const double pn = st.pnorm[s];
  double delta = st.delta[s];
  if (rho < 0.25)
    delta = 0.25 * pn;
  else if (rho > 0.75 && pn >= 0.99 * delta)
    delta = fmin(2.0 * delta, fp.delta_max);
  st.delta[s] = delta;
  if (rho > fp.eta) {
    double* th = st.theta + (size_t)s * NP;
    double* ps = st.psi + (size_t)s * NP;
    const double* tt = st.theta_trial + (size_t)s * NP;
    const double* pp = st.p + (size_t)s * NP;
    for (int i = 0; i < NP; ++i) {
      ps[i] += pp[i];
      th[i] = tt[i];
    }
    st.f[s] = ft;
    st.need_full[s] = 1;
    st.n_acc[s] += 1;
    if (fp.trial_derivs && fp.taken_px) atomicAdd(fp.taken_px, (unsigned long long)fp.srcs[s].npix);
  }
  st.iter[s] += 1;
  if (delta < fp.delta_min) {
    st.status[s] = CELESTE_TR_COLLAPSED;
    st.active[s] = 0;
    st.need_full[s] = 0;
    return;
  }
  atomicAdd(st.n_active, 1);
}

// Trial derivatives: a source whose step was just accepted (need_full set by k_accept) takes the
// gradient and Hessian evaluated at its trial point, which is now its current point; one 64-thread
// block per source.
__global__ __launch_bounds__(64) void k_take_trial(FitDev st) {
  const int s = blockIdx.x;
  if (!st.need_full[s]) return;
  const int t = threadIdx.x;
  if (t < NP) st.g[(size_t)s * NP + t] = st.g_trial[(size_t)s * NP + t];
  double* H = st.H + (size_t)s * NP * NP;
  const double* Ht = st.H_trial + (size_t)s * NP * NP;
  for (int k = t; k < NP * NP; k += 64) H[k] = Ht[k];
  __syncthreads();   // every thread has read the flag before it is cleared
  if (t == 0) st.need_full[s] = 0;
}

__global__ void k_fill(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_split(const int* __restrict__ flag, const int* __restrict__ samp, int* __restrict__ fa,
                        int* __restrict__ fb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int f = flag[i] != 0, sm = samp[i] != 0;
  fa[i] = f && !sm;
  fb[i] = f && sm;
}

__global__ void k_zero(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- linear-response covariance
// Sigma = D (-H_psi)^{-1} D at a fitted theta, H_psi = D H D + diag(D' g) in the fit's
// unconstrained coordinates (D = d theta / d psi, diagonal), one wavefront per source, FP64:
// Cholesky factor L of -H_psi in LDS (right-looking, one column per step, the trailing
// update spread over the lanes), L^{-1} by forward substitution (one column per lane), and
// Sigma_psi = L^{-T} L^{-1} summed in the same order for (a, b) and (b, a), so the result is
// exactly symmetric.  status: 0, 1 when a pivot is not positive (-H_psi not positive
// definite), 2 for a non-finite input; cov is NaN where status != 0.
__global__ __launch_bounds__(64) void k_lr_cov(const double* __restrict__ theta, const double* __restrict__ u0s,
                                               double u_box, const double* __restrict__ grad,
                                               const double* __restrict__ hess, double* __restrict__ cov,
                                               int* __restrict__ status) {
  __shared__ double M[NP][NP + 1];
  __shared__ double W[NP][NP + 1];
  __shared__ double d1s[NP];
  __shared__ int bad;
  const int s = blockIdx.x, t = threadIdx.x;
  const double* th = theta + (size_t)s * NP;
  const double* g = grad + (size_t)s * NP;
  const double* H = hess + (size_t)s * NP * NP;
  if (t == 0) bad = 0;
  __syncthreads();
  double d2g = 0.0;
  if (t < NP) {
    const double u0[2] = {u0s[2 * s], u0s[2 * s + 1]};
    const Box b = box_of(t, u0, u_box);
    double d1, d2;
    to_theta1(to_psi1(th[t], b), b, &d1, &d2);
    d1s[t] = d1;
    d2g = d2 * g[t];
    if (!isfinite(th[t]) || !isfinite(g[t]) || !isfinite(u0[0]) || !isfinite(u0[1])) atomicOr(&bad, 2);
  }
  __syncthreads();
  for (int k = t; k < NP * NP; k += 64) {
    const int r = k / NP, c = k - r * NP;
    const double h = 0.5 * (H[r * NP + c] + H[c * NP + r]);
    if (!isfinite(h)) atomicOr(&bad, 2);
    M[r][c] = -(d1s[r] * h * d1s[c]);
  }
  __syncthreads();
  if (t < NP) M[t][t] -= d2g;
  __syncthreads();
  if (bad == 0) {
    for (int k = 0; k < NP; ++k) {
      const double piv = M[k][k];
      if (!(piv > 0.0) || !isfinite(piv)) {   // the same value on every lane: a uniform exit
        if (t == 0) bad = 1;
        break;
      }
      const double lkk = sqrt(piv);
      __syncthreads();
      if (t == k) M[k][k] = lkk;
      if (t > k && t < NP) M[t][k] /= lkk;
      __syncthreads();
      for (int e = t; e < NP * NP; e += 64) {
        const int i = e / NP, j = e - i * NP;
        if (j > k && i >= j) M[i][j] -= M[i][k] * M[j][k];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  double* out = cov + (size_t)s * NP * NP;
  if (bad != 0) {
    for (int k = t; k < NP * NP; k += 64) out[k] = __builtin_nan("");
    if (t == 0) status[s] = bad;
    return;
  }
  if (t < NP) {
    const int j = t;
    for (int i = 0; i < NP; ++i) {
      if (i < j) {
        W[i][j] = 0.0;
        continue;
      }
      double acc = i == j ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= M[i][k] * W[k][j];
      W[i][j] = acc / M[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < NP * NP; e += 64) {
    const int a = e / NP, b = e - a * NP;
    double acc = 0.0;
    for (int k = a > b ? a : b; k < NP; ++k) acc += W[k][a] * W[k][b];
    out[e] = acc * (d1s[a] * d1s[b]);   // the same rounding for (a, b) and (b, a)
  }
  if (t == 0) status[s] = 0;
}

}  // namespace

hipError_t launch_fit_init(FitDev st, int n_src, FitParams fp, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_init, dim3((n_src + 127) / 128), dim3(128), 0, s, st, n_src, fp);
  return hipGetLastError();
}

hipError_t launch_psi_to_theta(const float* psi, const double* theta_cat, double* theta_out, int n_src,
                               double u_box, hipStream_t s) {
  hipLaunchKernelGGL(k_psi_to_theta, dim3((n_src + 127) / 128), dim3(128), 0, s, psi, theta_cat, theta_out, n_src,
                     u_box);
  return hipGetLastError();
}

hipError_t launch_choose_start(FitDev st, int n_src, hipStream_t s) {
  hipLaunchKernelGGL(k_choose_start, dim3((n_src + 127) / 128), dim3(128), 0, s, st, n_src);
  return hipGetLastError();
}

hipError_t launch_fit_start(FitDev st, int n_src, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_start, dim3((n_src + 127) / 128), dim3(128), 0, s, st, n_src);
  return hipGetLastError();
}

hipError_t launch_tr_step(FitDev st, int n_src, FitParams fp, hipStream_t s) {
  hipLaunchKernelGGL(k_tr, dim3(n_src), dim3(64), 0, s, st, fp);
  return hipGetLastError();
}

hipError_t launch_accept(FitDev st, int n_src, FitParams fp, hipStream_t s) {
  hipLaunchKernelGGL(k_accept, dim3((n_src + 127) / 128), dim3(128), 0, s, st, n_src, fp);
  return hipGetLastError();
}

hipError_t launch_take_trial(FitDev st, int n_src, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_take_trial, dim3(n_src), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_lr_cov(const double* theta, const double* u0, double u_box, const double* grad, const double* hess,
                         int n_src, double* cov, int* status, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lr_cov, dim3(n_src), dim3(64), 0, s, theta, u0, u_box, grad, hess, cov, status);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int value, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_split(const int* flag, const int* samp, int* fa, int* fb, int n_src, hipStream_t s) {
  if (n_src <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3((n_src + 255) / 256), dim3(256), 0, s, flag, samp, fa, fb, n_src);
  return hipGetLastError();
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3((n + 127) / 128), dim3(128), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace celeste
