"""The galaxy-group bound that lets the value+gradient+Hessian kernel skip all galaxy
components of one PSF component on a tile (CPU only).

The 14 galaxy components of PSF component k share its offset d and have covariances
C_j = nu_j W + Sigma_k (W the shape matrix in the image frame, PSD).  Since det C_j >= det Sigma_k
and lambda_max(C_j) <= nu_max lambda_max(W) + lambda_max(Sigma_k), every component's log2 density
is at most  c0 + mu |d|^2  with
    c0 = log2(w_k amp_max / (2 pi sqrt(det Sigma_k))),   mu = -log2(e) / (2 (nu_max lambda_max(W) + lambda_max(Sigma_k))).
The setup kernel writes c0 and mu rounded up to FP32 and the pixel kernel skips the group where
c0 + mu |d|^2 lies below the exact-zero threshold minus 1.  This test restates that bound from
its definition and checks it against the brute-force maximum over the components of their
exact log2 densities, for random shapes, PSFs, WCS matrices and offsets.
"""
import math

import numpy as np

import synth


def _rot(t):
    return np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])


def _lam_max(M):
    return float(np.linalg.eigvalsh(M)[-1])


def test_group_bound_dominates_every_component():
    prof = synth.load_profiles()
    amp = np.concatenate([prof["exp"][0], prof["dev"][0]])
    nu = np.concatenate([prof["exp"][1], prof["dev"][1]])
    rng = np.random.default_rng(161103404)
    worst = -np.inf
    n_checked = 0
    for trial in range(4000):
        q = rng.uniform(0.01, 1.0)
        t = rng.uniform(0, math.pi)
        s = math.exp(rng.uniform(math.log(0.2), math.log(15.0)))
        A = rng.normal(0, 0.3, (2, 2)) + np.eye(2) * rng.uniform(0.6, 1.4)
        W = A @ (s * s * _rot(t) @ np.diag([1.0, q * q]) @ _rot(t).T) @ A.T
        sx, sy = rng.uniform(0.5, 3.5, 2)
        rho = rng.uniform(-0.3, 0.3)
        Sig = np.array([[sx * sx, rho * sx * sy], [rho * sx * sy, sy * sy]])
        wk = rng.uniform(0.01, 1.0)
        lmax = nu.max() * _lam_max(W) + _lam_max(Sig)
        c0 = math.log2(wk * amp.max()) - math.log2(2 * math.pi) - 0.5 * math.log2(np.linalg.det(Sig))
        mu = -0.5 * math.log2(math.e) / lmax
        # offsets out to where the densities fall below 2^-200
        r = rng.uniform(0, 1.0, 64) ** 0.5 * math.sqrt(-200.0 / mu) if mu < 0 else np.zeros(64)
        ang = rng.uniform(0, 2 * math.pi, 64)
        d = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
        bound = c0 + mu * np.sum(d * d, axis=1)
        for j in range(amp.size):
            C = nu[j] * W + Sig
            P = np.linalg.inv(C)
            quad = np.einsum("ni,ij,nj->n", d, P, d)
            dens = (math.log2(wk * amp[j]) - math.log2(2 * math.pi) - 0.5 * math.log2(np.linalg.det(C))
                    - 0.5 * math.log2(math.e) * quad)
            worst = max(worst, float(np.max(dens - bound)))
            n_checked += dens.size
    assert n_checked == 4000 * 64 * amp.size
    # the bound holds with room for the FP32 rounding the kernel covers by a margin of 1
    assert worst <= 1e-9, worst


def test_group_bound_is_tight_at_the_centre_for_a_point_like_galaxy():
    """Where W -> 0 and one component carries the largest amplitude, the bound's constant is
    that component's log2 peak density: the bound is not loose by construction."""
    prof = synth.load_profiles()
    amp = np.concatenate([prof["exp"][0], prof["dev"][0]])
    Sig = np.array([[1.7, 0.2], [0.2, 1.2]])
    c0 = math.log2(0.6 * amp.max()) - math.log2(2 * math.pi) - 0.5 * math.log2(np.linalg.det(Sig))
    j = int(np.argmax(amp))
    peak = math.log2(0.6 * amp[j]) - math.log2(2 * math.pi) - 0.5 * math.log2(np.linalg.det(Sig))
    assert abs(c0 - peak) < 1e-12
