"""Unconstrained coordinates for the trust-region fit (oracle).

The paper optimises with trust-region Newton (section III-B) but does not say
in which coordinates.  Here each natural parameter theta_i is an elementwise
function of an unconstrained psi_i:

  u (x, y)         u0 - B + 2B sigmoid(psi)     box of half-width B around the start u0
  a, e_dev         lo + (hi - lo) sigmoid(psi)  on [1e-4, 1 - 1e-4]
  e_axis           same, on [0.01, 0.99]
  e_scale          same, on [0.2, 15] px
  e_angle, r1, c1  identity
  r2, c2           exp(psi)

so g_psi = t' * g_theta and H_psi = D H_theta D + diag(t'' * g_theta), D = diag(t').
Parity: pinned by finite differences of the composed map in the tests.
"""
from __future__ import annotations

import numpy as np

NP = 27
BOUNDED = {2: (1e-4, 1 - 1e-4), 3: (1e-4, 1 - 1e-4), 4: (0.01, 0.99), 6: (0.2, 15.0)}
IDENTITY = [5, 7, 8] + list(range(11, 19))
LOG = [9, 10] + list(range(19, 27))
CLIP_FRAC = 1e-9


def _bounds(u0, box):
    lo = np.full(NP, -np.inf)
    hi = np.full(NP, np.inf)
    lo[0:2] = np.asarray(u0) - box
    hi[0:2] = np.asarray(u0) + box
    for i, (a, b) in BOUNDED.items():
        lo[i], hi[i] = a, b
    return lo, hi


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def to_psi(theta, u0, box=3.0):
    """psi = T^{-1}(theta); bounded entries are first clipped into the open box."""
    theta = np.asarray(theta, dtype=np.float64)
    lo, hi = _bounds(u0, box)
    psi = theta.copy()
    logit_idx = [0, 1] + list(BOUNDED.keys())
    for i in logit_idx:
        span = hi[i] - lo[i]
        x = np.clip(theta[i], lo[i] + CLIP_FRAC * span, hi[i] - CLIP_FRAC * span)
        f = (x - lo[i]) / span
        psi[i] = np.log(f) - np.log1p(-f)
    psi[LOG] = np.log(theta[LOG])
    return psi


def to_theta(psi, u0, box=3.0):
    """theta = T(psi) with first and second derivatives (elementwise)."""
    psi = np.asarray(psi, dtype=np.float64)
    lo, hi = _bounds(u0, box)
    th = psi.copy()
    d1 = np.ones(NP)
    d2 = np.zeros(NP)
    for i in [0, 1] + list(BOUNDED.keys()):
        span = hi[i] - lo[i]
        s = _sig(psi[i])
        th[i] = lo[i] + span * s
        d1[i] = span * s * (1 - s)
        d2[i] = span * s * (1 - s) * (1 - 2 * s)
    e = np.exp(psi[LOG])
    th[LOG] = e
    d1[LOG] = e
    d2[LOG] = e
    return th, d1, d2


def grad_hess_psi(g_theta, H_theta, d1, d2):
    g = d1 * g_theta
    H = d1[:, None] * H_theta * d1[None, :] + np.diag(d2 * g_theta)
    return g, H
