"""Limited-memory BFGS fit of one source (oracle; test infrastructure only).

Section III-B reports that the earlier version of Celeste optimised each source with L-BFGS
(citing Nocedal & Wright), and that some sources then needed thousands of iterations, which
dominated the runtime; trust-region Newton with the exact Hessian replaced it.  The paper
gives no L-BFGS settings, so this follows the textbook algorithm (Nocedal & Wright, 2nd ed.,
Algorithm 7.4 for the two-loop recursion and Algorithm 7.5 for the iteration) in the same
unconstrained coordinates psi as the trust-region fit, with these readings:

  * objective: minimise f(psi) = -L(theta(psi)); gradient g = -D g_theta (D = dtheta/dpsi);
  * memory m = 10 curvature pairs (s, y); initial inverse Hessian gamma I with
    gamma = s'y / y'y of the newest pair, and for the first step the unit-length step
    p = -g / |g| (the identity scaled so the first trial moves psi by 1); a direction with
    g'p >= 0 (possible only through rounding) restarts the same way with the pairs dropped;
  * line search: backtracking from alpha = 1 with the sufficient-decrease (Armijo) condition
    f(psi + alpha p) <= f(psi) + c1 alpha g'p, c1 = 1e-4, halving alpha up to 30 times;
    a non-finite trial value counts as a failed condition;
  * a pair with s'y <= 1e-10 |s| |y| is not stored (the curvature condition is not enforced by
    a backtracking search, and BFGS needs s'y > 0);
  * stopping: the quasi-Newton model's predicted gain -g'p / 2 (= g'H g / 2 for the model
    inverse Hessian H) is at most pred_rtol max(1, |L|), the rule the trust-region fit applies to
    its own model; status MAX_ITER after max_iter iterations, LINE_SEARCH_FAILED when 30
    halvings find no sufficient decrease.

An iteration is one accepted step (one gradient evaluation); the value evaluations of the line
search are counted separately.

Parity: the two-loop recursion is pinned by the secant condition (the recursion applied to the
newest y returns the newest s) and by equality with the dense BFGS inverse-Hessian update
(Nocedal & Wright, eq. 6.17) applied to the same pairs, written out in the test; the iteration
by the exact minimisers of strictly convex quadratics and of the Rosenbrock function, and by
the trust-region oracle's optimum of the config-0 source.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import model, transforms

CONVERGED, MAX_ITER, LINE_SEARCH_FAILED, NONFINITE = 0, 1, 4, 3


@dataclass
class LbfgsOpts:
    max_iter: int = 1000
    memory: int = 10
    pred_rtol: float = 1e-8
    c1: float = 1e-4
    max_backtracks: int = 30
    box: float = 3.0


@dataclass
class LbfgsResult:
    theta: np.ndarray
    elbo: float
    iters: int
    status: int
    pred: float
    value_evals: int
    history: list = field(default_factory=list)


def two_loop(g, S, Y):
    """H g for the L-BFGS inverse-Hessian approximation defined by the pairs (S[i], Y[i]),
    oldest first, with H0 = gamma I, gamma = s'y / y'y of the newest pair (1 without pairs)
    (Nocedal & Wright, Algorithm 7.4)."""
    q = np.array(g, dtype=np.float64)
    k = len(S)
    alpha = np.zeros(k)
    rho = [1.0 / float(Y[i] @ S[i]) for i in range(k)]
    for i in range(k - 1, -1, -1):
        alpha[i] = rho[i] * float(S[i] @ q)
        q = q - alpha[i] * Y[i]
    gamma = float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1]) if k else 1.0
    r = gamma * q
    for i in range(k):
        beta = rho[i] * float(Y[i] @ r)
        r = r + (alpha[i] - beta) * S[i]
    return r


def minimise(fun, grad, x0, opts: LbfgsOpts = LbfgsOpts(), scale=1.0, record=False):
    """L-BFGS with backtracking on a generic smooth f (fun, grad of x); scale sets the
    stopping tolerance pred_rtol * max(1, scale).  Returns (x, f, iterations, status,
    predicted gain, value evaluations, history)."""
    x = np.array(x0, dtype=np.float64)
    f = float(fun(x))
    g = np.asarray(grad(x), dtype=np.float64)
    S, Y = [], []
    it = 0
    n_val = 0
    hist = []
    status = MAX_ITER
    pred = float("nan")
    if not np.isfinite(f) or not np.all(np.isfinite(g)):
        return x, f, 0, NONFINITE, pred, n_val, hist
    while True:
        p = -two_loop(g, S, Y) if S else None
        if p is None or not float(g @ p) < 0.0:
            # first step, or a direction that does not descend (rounding): restart from the
            # unit-length steepest-descent step and forget the pairs
            S, Y = [], []
            gn = float(np.linalg.norm(g))
            p = -g / gn if gn > 0 else np.zeros_like(g)
        pred = -0.5 * float(g @ p)
        if record:
            hist.append(dict(it=it, f=f, pred=pred))
        if pred <= opts.pred_rtol * max(1.0, abs(scale(f) if callable(scale) else scale)):
            status = CONVERGED
            break
        if it == opts.max_iter:
            status = MAX_ITER
            break
        gp = float(g @ p)
        alpha = 1.0
        accepted = False
        for _ in range(opts.max_backtracks + 1):
            xt = x + alpha * p
            ft = float(fun(xt))
            n_val += 1
            if np.isfinite(ft) and ft <= f + opts.c1 * alpha * gp:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            status = LINE_SEARCH_FAILED
            break
        gt = np.asarray(grad(xt), dtype=np.float64)
        s, y = xt - x, gt - g
        if float(s @ y) > 1e-10 * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
            S.append(s)
            Y.append(y)
            if len(S) > opts.memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = xt, ft, gt
        it += 1
    return x, f, it, status, pred, n_val, hist


def fit(theta0, images, prior, profiles, opts: LbfgsOpts = LbfgsOpts(), record=False):
    """Maximise the ELBO of one source from theta0 by L-BFGS in psi coordinates."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    u0 = theta0[0:2].copy()
    psi0 = transforms.to_psi(theta0, u0, opts.box)

    def th_of(psi):
        return transforms.to_theta(psi, u0, opts.box)

    def fun(psi):
        return -model.elbo_value(th_of(psi)[0], images, prior, profiles)

    def grad(psi):
        th, d1, _ = th_of(psi)
        _, g, _ = model.elbo(th, images, prior, profiles)
        return -d1 * g

    psi, f, it, status, pred, n_val, hist = minimise(fun, grad, psi0, opts, scale=lambda f_: -f_, record=record)
    return LbfgsResult(th_of(psi)[0], -f, it, status, pred, n_val, hist)
