"""Pins of the oracle's linear-response covariance (the closing section's linear response
methods): the textbook Gaussian case where it recovers the exact posterior covariance, the
defining sensitivity of a tilted optimum on the Celeste ELBO itself, the reduction to -H^{-1}
at an interior stationary point, and a coordinate held at its box edge."""
import numpy as np
import pytest

import synth
from oracle import init as oinit
from oracle import lr, model, newton, transforms


def test_textbook_gaussian_target_recovers_exact_covariance():
    """Target N(0, A^{-1}), q = prod N(m_i, v_i): the ELBO is
    -m'Am/2 - sum A_ii v_i / 2 + sum log v_i / 2 (+ const).  Mean field gives v_i = 1/A_ii,
    linear response gives the exact covariance A^{-1} (Sherman-Morrison for A = al I + w w')."""
    d, al = 4, 1.7
    w = np.array([0.9, -0.4, 1.3, 0.2])
    A = al * np.eye(d) + np.outer(w, w)
    Ainv = (np.eye(d) - np.outer(w, w) / (al + w @ w)) / al

    def elbo(x):
        m, v = x[:d], x[d:]
        return -0.5 * m @ A @ m - 0.5 * np.sum(np.diag(A) * v) + 0.5 * np.sum(np.log(v))

    x0 = np.concatenate([np.zeros(d), 1.0 / np.diag(A)])
    n, h = 2 * d, 1e-4
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            e_i, e_j = np.eye(n)[i] * h, np.eye(n)[j] * h
            H[i, j] = (elbo(x0 + e_i + e_j) - elbo(x0 + e_i - e_j) - elbo(x0 - e_i + e_j)
                       + elbo(x0 - e_i - e_j)) / (4 * h * h)
    S = lr.lr_from_hessian(H)
    assert S is not None
    assert np.allclose(S[:d, :d], Ainv, rtol=1e-6, atol=1e-7)
    # mean field under-estimates every marginal variance here
    assert np.all(1.0 / np.diag(A) < np.diag(Ainv))


def test_not_positive_definite_is_none():
    H = -np.eye(27)
    H[5, 5] = 0.3
    assert lr.lr_from_hessian(H) is None
    H = -np.eye(27)
    H[3, 4] = np.nan
    assert lr.lr_from_hessian(H) is None


def test_interior_stationary_point_reduces_to_minus_inverse():
    rng = np.random.default_rng(3)
    sb = synth.make_config(0)
    th = sb.theta_truth[0].copy()
    th[2], th[3], th[4], th[6] = 0.4, 0.6, 0.5, 2.0
    B = rng.normal(size=(27, 27))
    H = -(B @ B.T + 27 * np.eye(27))
    S = lr.lr_covariance(th, np.zeros(27), H, th[0:2] + 0.3)
    assert np.allclose(S, -np.linalg.inv(H), rtol=1e-9, atol=1e-14)


@pytest.fixture(scope="module")
def bright_fits():
    sb = synth.make_config(1, n_sources=4, bright=True)
    out = {}
    for s in (1, 3):
        imgs = model.source_images(sb, s)
        th0 = oinit.plain_init(sb.u_cat[s], imgs, sb.prior)
        res = newton.fit(th0, imgs, sb.prior, sb.profiles)
        assert res.status == newton.CONVERGED
        out[s] = (sb, imgs, th0[0:2].copy(), res.theta)
    return out


def _tilted_optimum(imgs, sb, u0, psi, g_star, i, t):
    """Stationary point of L(psi) - g_star'psi + t theta_i(psi), by Newton's method from psi.
    Subtracting g_star, the psi-gradient of L at the fit, makes the fit an exact stationary
    point without changing any second derivative (the fit stops on its predicted gain, and
    flat directions such as a shape parameter drifting towards its box edge would otherwise
    move the reference point)."""
    psi = psi.copy()
    for _ in range(40):
        th, d1, d2 = transforms.to_theta(psi, u0)
        _, g, H = model.elbo(th, imgs, sb.prior, sb.profiles)
        g = g.copy()
        g[i] += t
        gp, Hp = transforms.grad_hess_psi(g, H, d1, d2)
        step = np.linalg.solve(Hp, g_star - gp)
        psi = psi + step
        if np.max(np.abs(step)) < 1e-13:
            break
    return psi


def test_tilted_optimum_sensitivity(bright_fits):
    """Column i of Sigma_LR is d theta*/dt for the objective tilted by t theta_i (central
    difference of re-solved optima): the definition of linear response, independent of the
    formula."""
    sb, imgs, u0, th_fit = bright_fits[1]
    psi0 = transforms.to_psi(th_fit, u0)
    th0, d1, d2 = transforms.to_theta(psi0, u0)
    _, g, H = model.elbo(th0, imgs, sb.prior, sb.profiles)
    g_star = transforms.grad_hess_psi(g, H, d1, d2)[0]
    S = lr.lr_covariance(th0, g, H, u0)
    assert S is not None
    for i in (0, 2, 4, 7, 11):
        tau = 1e-5 / np.sqrt(S[i, i])
        tp = transforms.to_theta(_tilted_optimum(imgs, sb, u0, psi0, g_star, i, tau), u0)[0]
        tm = transforms.to_theta(_tilted_optimum(imgs, sb, u0, psi0, g_star, i, -tau), u0)[0]
        col = (tp - tm) / (2 * tau)
        scale = np.max(np.abs(S[:, i]))
        assert np.max(np.abs(col - S[:, i])) <= 1e-4 * scale, (i, np.max(np.abs(col - S[:, i])) / scale)


def test_coordinate_at_box_edge_has_no_variance(bright_fits):
    sb, imgs, u0, th = bright_fits[3]
    assert th[2] < 1e-4 + 1e-6          # q(star) ended at its lower edge
    _, g, H = model.elbo(th, imgs, sb.prior, sb.profiles)
    S = lr.lr_covariance(th, g, H, u0)
    assert S is not None
    assert S[2, 2] < 1e-6 * S[0, 0]      # against 2e-3 px^2 for the position
    assert np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > -1e-12 * np.max(np.abs(S)))
