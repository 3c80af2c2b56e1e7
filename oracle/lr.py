"""Linear-response covariance of a fitted source (oracle; test infrastructure only).

The paper's closing section (Conclusions and Future Work) proposes linear response methods
(Giordano et al., 2015) for the uncertainty of the variational fit: a factorised q
under-estimates posterior variance, and parameters that are point estimates (position,
galaxy shape) get no variance at all.  Linear response reads the covariance off how the
optimum moves when the objective is tilted: at a stationary point of the ELBO L in some
coordinates psi, maximising L + t theta_i moves the optimum by

    d theta*/dt = D (-H_psi)^{-1} D e_i,   D = d theta / d psi (diagonal here),

so the linear-response covariance is Sigma_LR = D (-H_psi)^{-1} D.

Coordinates: the fit is stationary in the unconstrained psi of the trust-region fit (the
boxes of u, a, e_dev, e_axis, e_scale and the logs of the variances), not always in theta:
a coordinate that ends at its box edge has a non-zero theta-gradient and a vanishing D,
and then gets (near) zero variance, as a parameter held at its bound should.  Where the
fit is interior, H_psi = D H_theta D + diag(D' g_theta) with g_theta = 0, and Sigma_LR
reduces to -H_theta^{-1}, the textbook form.

The entries of u, a, e_*, the log-brightness means r1 and the colour means c1 are the
linear-response covariances of first moments of q (or of point estimates); for those the
map from theta to the mean parameters of q is the identity.  The rows of the variance
parameters (r2, c2) are sensitivities of those parameters, not moments.

Defined only where -H_psi is positive definite (a strict local maximum in psi); otherwise
the result is None.
"""
from __future__ import annotations

import numpy as np

from . import transforms


def lr_from_hessian(H):
    """-H^{-1} for a symmetric negative-definite H; None if -H is not positive definite or
    H holds a non-finite entry."""
    H = np.asarray(H, dtype=np.float64)
    if not np.all(np.isfinite(H)):
        return None
    Hs = 0.5 * (H + H.T)
    if np.linalg.eigvalsh(-Hs).min() <= 0.0:
        return None
    return -np.linalg.inv(Hs)


def lr_covariance(theta, g_theta, H_theta, u0, box=3.0):
    """Sigma_LR (27 x 27) at a fitted theta from the ELBO's natural gradient and Hessian
    there; u0 and box give the position box of the fit's coordinates.  None where -H_psi
    is not positive definite."""
    psi = transforms.to_psi(theta, u0, box)
    _, d1, d2 = transforms.to_theta(psi, u0, box)
    _, Hp = transforms.grad_hess_psi(np.asarray(g_theta, np.float64), np.asarray(H_theta, np.float64), d1, d2)
    Sp = lr_from_hessian(Hp)
    if Sp is None:
        return None
    return d1[:, None] * Sp * d1[None, :]
