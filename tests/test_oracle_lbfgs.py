"""Pins of the L-BFGS oracle (the earlier Celeste optimiser of section III-B), CPU only."""
import numpy as np
import pytest

import synth
from oracle import init as oinit
from oracle import lbfgs, model, newton


def _pairs(rng, n, k):
    """k curvature pairs y = A s of a random SPD matrix A (s'y > 0)."""
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(rng.uniform(0.1, 10.0, n)) @ Q.T
    S = [rng.normal(size=n) for _ in range(k)]
    return A, S, [A @ s for s in S]


def _bfgs_dense(S, Y, n):
    """Inverse-Hessian approximation by the BFGS update H <- (I - r s y') H (I - r y s') + r s s',
    r = 1 / y's, from H0 = gamma I with gamma = s'y / y'y of the newest pair."""
    H = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]) * np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / (y @ s)
        H = (np.eye(n) - r * np.outer(s, y)) @ H @ (np.eye(n) - r * np.outer(y, s)) + r * np.outer(s, s)
    return H


def test_two_loop_secant_and_dense_update():
    rng = np.random.default_rng(3)
    n = 27
    for k in (1, 4, 10):
        A, S, Y = _pairs(rng, n, k)
        # secant condition on the newest pair: H y = s
        np.testing.assert_allclose(lbfgs.two_loop(Y[-1], S, Y), S[-1], rtol=1e-9, atol=1e-12)
        # the recursion applies the same matrix as the dense BFGS updates
        H = _bfgs_dense(S, Y, n)
        for _ in range(3):
            g = rng.normal(size=n)
            np.testing.assert_allclose(lbfgs.two_loop(g, S, Y), H @ g, rtol=1e-9, atol=1e-12 * np.abs(H @ g).max())
    # no pairs: the identity
    g = rng.normal(size=n)
    np.testing.assert_array_equal(lbfgs.two_loop(g, [], []), g)


def test_minimises_quadratics_and_rosenbrock():
    rng = np.random.default_rng(4)
    n = 27
    for cond in (10.0, 1e3):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A = Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T
        b = rng.normal(size=n)
        xs = np.linalg.solve(A, b)
        fs = -0.5 * b @ xs
        x, f, it, status, pred, nv, _ = lbfgs.minimise(lambda x: 0.5 * x @ A @ x - b @ x, lambda x: A @ x - b,
                                                        np.zeros(n), lbfgs.LbfgsOpts(pred_rtol=1e-14), scale=1.0)
        assert status == lbfgs.CONVERGED and it < 400
        assert abs(f - fs) <= 1e-12 * max(1.0, abs(fs))
        np.testing.assert_allclose(x, xs, rtol=1e-4, atol=1e-5 * np.abs(xs).max())

    def rosen(x):
        return 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2

    def drosen(x):
        return np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200.0 * (x[1] - x[0] ** 2)])

    x, f, it, status, *_ = lbfgs.minimise(rosen, drosen, np.array([-1.2, 1.0]), lbfgs.LbfgsOpts(pred_rtol=1e-20))
    assert status == lbfgs.CONVERGED and f < 1e-16
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-7)


def test_status_paths():
    A = np.diag(np.arange(1.0, 6.0))
    x, f, it, status, *_ = lbfgs.minimise(lambda x: 0.5 * x @ A @ x, lambda x: A @ x, np.ones(5),
                                          lbfgs.LbfgsOpts(max_iter=2, pred_rtol=1e-30))
    assert status == lbfgs.MAX_ITER and it == 2
    # a wrong-sign gradient: no step along p decreases f -> the line search fails
    x, f, it, status, *_ = lbfgs.minimise(lambda x: 0.5 * x @ A @ x, lambda x: -(A @ x), np.ones(5))
    assert status == lbfgs.LINE_SEARCH_FAILED and it == 0
    x, f, it, status, *_ = lbfgs.minimise(lambda x: np.nan, lambda x: x, np.ones(5))
    assert status == lbfgs.NONFINITE


def test_config0_reaches_the_trust_region_optimum():
    """From the plain start L-BFGS converges to the trust-region oracle's optimum of the
    config-0 source (A22: within 1e-5 |L*| or above), in more iterations (section III-B)."""
    sb = synth.make_config(0)
    imgs = model.source_images(sb, 0)
    th0 = oinit.plain_init(sb.u_cat[0], imgs, sb.prior)
    tr = newton.fit(th0, imgs, sb.prior, sb.profiles)
    lb = lbfgs.fit(th0, imgs, sb.prior, sb.profiles, record=True)
    assert tr.status == newton.CONVERGED and lb.status == lbfgs.CONVERGED
    assert abs(lb.elbo - tr.elbo) <= 1e-5 * abs(tr.elbo) or lb.elbo >= tr.elbo
    assert lb.iters > tr.iters
    f = [h["f"] for h in lb.history]
    assert all(b <= a for a, b in zip(f, f[1:]))       # f = -L never increases over accepted steps
    assert lb.value_evals >= lb.iters
