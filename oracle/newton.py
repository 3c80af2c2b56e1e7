"""Trust-region Newton fit of one source (oracle).

Section III-B: each source's ELBO is maximised with Newton's method whose
updates are constrained by a trust region, using the manually computed
gradient and dense Hessian; the paper reports convergence within 50
iterations.  The paper gives no constants, so this follows the textbook
trust-region algorithm (Nocedal & Wright, Alg. 4.1, the book the paper cites
for L-BFGS) with the exact subproblem solved through a symmetric
eigendecomposition and the secular equation (More-Sorensen, incl. the hard
case):

  maximise  m(p) = g'p + p'Hp/2  subject to |p| <= Delta   (in psi coordinates)
  rho = (L(psi+p) - L(psi)) / m(p)
  rho < 1/4                      -> Delta = |p| / 4
  rho > 3/4 and |p| at the bound -> Delta = min(2 Delta, Delta_max)
  rho > eta                      -> accept
  converged when m(p) <= tol * max(1, |L|) and -H is positive semidefinite
  (smallest eigenvalue >= -curv_tol * max(1, |H|)); collapsed when Delta < Delta_min.

Parity: the subproblem is pinned by its KKT conditions; fits by monotone ELBO,
the stopping rule, and agreement across starting points.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.optimize import brentq

from . import model, transforms

CONVERGED, MAX_ITER, TR_COLLAPSED, NONFINITE = 0, 1, 2, 3


@dataclass
class FitOpts:
    max_iter: int = 50
    pred_rtol: float = 1e-8
    curv_tol: float = 1e-8
    delta0: float = 1.0
    delta_max: float = 100.0
    delta_min: float = 1e-10
    eta: float = 0.1
    box: float = 3.0


@dataclass
class FitResult:
    theta: np.ndarray
    elbo: float
    iters: int
    status: int
    pred: float
    history: list = field(default_factory=list)


def tr_subproblem(g, H, delta):
    """Exact maximiser of g'p + p'Hp/2 over |p| <= delta.

    With B = -H = V diag(lam) V', the solution is p = (B + s I)^{-1} g for the smallest
    s >= max(0, -lam_min) with |p| <= delta and s (delta - |p|) = 0; in the hard case
    (g orthogonal to the bottom eigenspace) a multiple of the bottom eigenvector is added
    to reach the boundary.  Returns p, predicted gain, s, lam (ascending eigenvalues of B).
    """
    B = -0.5 * (H + H.T)
    lam, V = np.linalg.eigh(B)
    gt = V.T @ g
    scale = max(1.0, np.max(np.abs(lam)))
    lam0 = lam[0]

    def pnorm(s):
        return math.sqrt(np.sum((gt / (lam + s)) ** 2))

    s = 0.0
    if lam0 > 1e-14 * scale and pnorm(0.0) <= delta:
        pt = gt / lam
    else:
        s_lo = max(0.0, -lam0)
        # components of g in the bottom eigenspace
        bottom = np.abs(lam - lam0) <= 1e-12 * scale
        gbot = math.sqrt(np.sum(gt[bottom] ** 2))
        rest = ~bottom
        if gbot <= 1e-12 * max(1.0, np.linalg.norm(g)):
            prest = gt[rest] / (lam[rest] + s_lo) if np.any(rest) else np.zeros(0)
            nrest = math.sqrt(np.sum(prest ** 2))
            if nrest <= delta:                   # hard case
                s = s_lo
                pt = np.zeros_like(gt)
                pt[rest] = prest
                tau = math.sqrt(max(delta * delta - nrest * nrest, 0.0))
                pt[np.argmax(bottom)] += tau
                p = V @ pt
                pred = g @ p + 0.5 * p @ H @ p
                return p, pred, s, lam
        # root of |p(s)| = delta on (s_lo, hi]; just above the pole the norm may already be
        # inside (g nearly orthogonal to the bottom space): then that point is taken
        s_a = s_lo + 1e-12 * scale if s_lo > 0 else 0.0
        f = lambda t: pnorm(t) - delta
        if f(s_a) <= 0:
            s = s_a
        else:
            b = s_lo + np.linalg.norm(g) / delta + 1.0
            s = brentq(f, s_a, b, xtol=1e-15, rtol=1e-15, maxiter=500)
        pt = gt / (lam + s)
    p = V @ pt
    pred = g @ p + 0.5 * p @ H @ p
    return p, pred, s, lam


def _tr_loop(psi, u0, objective, opts, it0, delta, switch_rtol=None, record=False, hist=None):
    """The trust-region iteration from psi (f, g, H of objective(psi, want) in psi coordinates).

    Without switch_rtol: the fit proper (stopping rule of the module docstring).  With it: the
    early phase on a subsampled objective, which stops instead when its model's predicted gain
    is at most switch_rtol max(1, |f|) (status None: go on with the full objective).  Iterations
    are counted from it0 against opts.max_iter.  Returns (psi, f, iterations, status, pred, delta)."""
    f, g, H = objective(psi, "hess")
    status = MAX_ITER
    pred = float("nan")
    it = it0
    if not np.isfinite(f):
        return psi, f, it, NONFINITE, pred, delta
    while True:
        p, pred, s, lam = tr_subproblem(g, H, delta)
        if record:
            hist.append(dict(it=it, elbo=f, pred=pred, delta=delta, lam0=lam[0], sampled=switch_rtol is not None))
        if switch_rtol is not None:
            if pred <= switch_rtol * max(1.0, abs(f)):
                status = None
                break
        elif pred <= opts.pred_rtol * max(1.0, abs(f)) and lam[0] >= -opts.curv_tol * max(1.0, np.max(np.abs(lam))):
            status = CONVERGED
            break
        if it >= opts.max_iter:
            status = MAX_ITER
            break
        f_new = objective(psi + p, "value")
        rho = (f_new - f) / pred if np.isfinite(f_new) else -np.inf
        pn = np.linalg.norm(p)
        if rho < 0.25:
            delta = 0.25 * pn
        elif rho > 0.75 and pn >= 0.99 * delta:
            delta = min(2.0 * delta, opts.delta_max)
        if rho > opts.eta:
            psi = psi + p
            f, g, H = objective(psi, "hess")
        it += 1
        if delta < opts.delta_min:
            status = TR_COLLAPSED
            break
    return psi, f, it, status, pred, delta


def _objective(images, prior, profiles, u0, box):
    def objective(psi, want):
        theta, d1, d2 = transforms.to_theta(psi, u0, box)
        if want == "value":
            return model.elbo_value(theta, images, prior, profiles)
        f, gt, Ht = model.elbo(theta, images, prior, profiles)
        g, H = transforms.grad_hess_psi(gt, Ht, d1, d2)
        return f, g, H
    return objective


def fit(theta0, images, prior, profiles, opts: FitOpts = FitOpts(), record=False):
    """Maximise the ELBO of one source from theta0 by trust-region Newton in psi coordinates."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    u0 = theta0[0:2].copy()
    psi = transforms.to_psi(theta0, u0, opts.box)
    hist = []
    psi, f, it, status, pred, _ = _tr_loop(psi, u0, _objective(images, prior, profiles, u0, opts.box), opts, 0,
                                           opts.delta0, record=record, hist=hist)
    return FitResult(transforms.to_theta(psi, u0, opts.box)[0], f, it, status, pred, hist)


def fit_sampled(theta0, images, sampled_images, prior, profiles, switch_rtol, opts: FitOpts = FitOpts(),
                record=False):
    """Trust-region Newton with a subsampled early phase (the paper's closing section proposes
    subsampling pixels to speed up the optimisation).  sampled_images are the source's images
    with per-pixel weights (kept blocks 1/p, dropped blocks 0; the theta-free part of every
    pixel is kept whole, model.image_sums).  Phase 1 is the trust-region fit of that unbiased
    estimate of the ELBO, until its model's predicted gain is at most switch_rtol max(1, |L_s|)
    (no curvature condition) or the iteration cap; phase 2 continues from there on the full
    ELBO with the trust radius it reached and the fit's own stopping rule.  The switch is not an
    iteration; the cap counts both phases."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    u0 = theta0[0:2].copy()
    psi = transforms.to_psi(theta0, u0, opts.box)
    hist = []
    psi, f, it, status, pred, delta = _tr_loop(psi, u0, _objective(sampled_images, prior, profiles, u0, opts.box),
                                               opts, 0, opts.delta0, switch_rtol=switch_rtol, record=record,
                                               hist=hist)
    n_sampled = it
    if status is None:
        psi, f, it, status, pred, _ = _tr_loop(psi, u0, _objective(images, prior, profiles, u0, opts.box), opts,
                                               it, delta, record=record, hist=hist)
    r = FitResult(transforms.to_theta(psi, u0, opts.box)[0], f, it, status, pred, hist)
    r.sampled_iters = n_sampled
    return r
