"""FP64 oracle of the Celeste per-source ELBO, gradient and dense Hessian.

Section III-A defines the model: pixel counts x_nm ~ Poisson(F_nm) with F a
deterministic function of the catalog and the image metadata; each source
has a Bernoulli star/galaxy indicator a, a lognormal reference-band
brightness r, multivariate-normal colours c (log ratios of adjacent bands),
a position mu and, for galaxies, shape/scale/morphology phi.  Section III-B
defines the objective: the ELBO  E_q[log p(x,z) - log q(z)]  (Eq. 1) with
the mean-field q(z) = q(r|a) q(c|a) q(a) (lognormal / multivariate normal /
Bernoulli), maximised per source with the other sources held fixed, using a
hand-derived gradient and dense Hessian.

The paper leaves the expected log-rate E_q[log F] unspecified beyond a note
that intractable integrals are approximated; here it is the second-order
delta method  E[log F] ~= log E[F] - Var[F] / (2 E[F]^2).

Everything below works in "z-space" per image: the 11 quantities one image
sees, z = (a, m_s, v_s, m_g, v_g, p_x, p_y, e_dev, e_axis, e_angle, e_scale),
where m_i, v_i are the mean and variance of log brightness of type i in the
image's band and p is the source position in the image's pixel frame.
theta -> z is linear per image, so the theta Hessian is sum_n J_n^T H_z J_n.

Derivatives are propagated with a small second-order forward-mode "jet"
(value, gradient, Hessian per pixel) and the product/chain rules, starting
from closed-form derivatives of each bivariate Gaussian with respect to its
mean and covariance (standard matrix-calculus identities for log det C and
C^{-1}).

Parity: pinned by tests against finite differences, library Poisson log-pmf,
Gauss-Hermite quadrature and Monte Carlo of the variational expectation,
mixture flux integrals and symmetry invariants.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln

NP = 27          # parameters per source
NZ = 11          # per-image z-space dimension
# parameter indices (natural coordinates)
I_U = (0, 1)
I_A = 2
I_DEV, I_AXIS, I_ANGLE, I_SCALE = 3, 4, 5, 6
I_R1 = (7, 8)    # [star, galaxy]
I_R2 = (9, 10)
I_C1 = (slice(11, 15), slice(15, 19))
I_C2 = (slice(19, 23), slice(23, 27))
# z indices
Z_A, Z_MS, Z_VS, Z_MG, Z_VG, Z_PX, Z_PY, Z_DEV, Z_AXIS, Z_ANGLE, Z_SCALE = range(NZ)

# log l_b = log l_r + S[b] . c  with c_j = log(l_{j+1} / l_j), bands u,g,r,i,z = 0..4
COLOUR_SIGNS = np.array([
    [-1.0, -1.0, 0.0, 0.0],   # u
    [0.0, -1.0, 0.0, 0.0],    # g
    [0.0, 0.0, 0.0, 0.0],     # r (reference)
    [0.0, 0.0, 1.0, 0.0],     # i
    [0.0, 0.0, 1.0, 1.0],     # z
])


# ----------------------------------------------------------------------------
# second-order jets over pixels
# ----------------------------------------------------------------------------

class Jet:
    """Per-pixel value v (n,), gradient g (n,D) and Hessian h (n,D,D)."""

    __slots__ = ("v", "g", "h")

    def __init__(self, v, g, h):
        self.v, self.g, self.h = v, g, h

    @staticmethod
    def const(value, n, D=NZ):
        return Jet(np.full(n, float(value)), np.zeros((n, D)), np.zeros((n, D, D)))

    @staticmethod
    def var(value, index, n, D=NZ):
        g = np.zeros((n, D))
        g[:, index] = 1.0
        return Jet(np.full(n, float(value)), g, np.zeros((n, D, D)))

    def __add__(self, o):
        if isinstance(o, Jet):
            return Jet(self.v + o.v, self.g + o.g, self.h + o.h)
        return Jet(self.v + o, self.g, self.h)

    __radd__ = __add__

    def __neg__(self):
        return Jet(-self.v, -self.g, -self.h)

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if isinstance(o, Jet):
            v = self.v * o.v
            g = self.g * o.v[:, None] + o.g * self.v[:, None]
            h = (self.h * o.v[:, None, None] + o.h * self.v[:, None, None]
                 + self.g[:, :, None] * o.g[:, None, :] + o.g[:, :, None] * self.g[:, None, :])
            return Jet(v, g, h)
        return Jet(self.v * o, self.g * o, self.h * o)

    __rmul__ = __mul__

    def apply(self, f, df, d2f):
        """Chain rule for a scalar function with value f, first df, second d2f (arrays)."""
        return Jet(f, self.g * df[:, None],
                   self.h * df[:, None, None] + self.g[:, :, None] * self.g[:, None, :] * d2f[:, None, None])

    def exp(self):
        e = np.exp(self.v)
        return self.apply(e, e, e)

    def square(self):
        return self * self

    def sum(self):
        return self.v.sum(), self.g.sum(axis=0), self.h.sum(axis=0)


# ----------------------------------------------------------------------------
# brightness moments (O1)
# ----------------------------------------------------------------------------

def band_moments(theta, band):
    """Mean and variance of log brightness for star and galaxy in `band`.

    Under q, log l_r ~ N(r1, r2) and each colour c_j ~ N(c1_j, c2_j) independently
    (diagonal q), and log l_b = log l_r + S_b . c (colours are log ratios of adjacent
    bands, reference band r; section III-A).  Returns (m_s, v_s, m_g, v_g).
    """
    S = COLOUR_SIGNS[band]
    m_s = theta[I_R1[0]] + S @ theta[I_C1[0]]
    v_s = theta[I_R2[0]] + (S * S) @ theta[I_C2[0]]
    m_g = theta[I_R1[1]] + S @ theta[I_C1[1]]
    v_g = theta[I_R2[1]] + (S * S) @ theta[I_C2[1]]
    return m_s, v_s, m_g, v_g


def lognormal_moments(m, v):
    """E[l] and E[l^2] for log l ~ N(m, v); inf where they overflow (a trial point that far out
    gets a non-finite ELBO, which the fits reject)."""
    with np.errstate(over="ignore"):
        return float(np.exp(m + 0.5 * v)), float(np.exp(2.0 * m + 2.0 * v))


# ----------------------------------------------------------------------------
# galaxy shape matrix and its derivatives
# ----------------------------------------------------------------------------

def _rot(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s], [s, c]])


def _drot(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[-s, -c], [c, -s]])


def shape_matrix(e_axis, e_angle, e_scale):
    """W = s^2 R(t) diag(1, q^2) R(t)^T with first and second derivatives in (q, t, s).

    Returns W (2,2), dW (3,2,2), d2W (3,3,2,2) in the order (e_axis, e_angle, e_scale).
    The half-light ellipse has major axis along angle t (radians, counter-clockwise from
    +x), minor/major ratio q and half-light radius s (px).
    """
    q, t, s = e_axis, e_angle, e_scale
    R, dR = _rot(t), _drot(t)
    d2R = -R
    D = np.diag([1.0, q * q])
    Dq = np.diag([0.0, 2.0 * q])
    Dqq = np.diag([0.0, 2.0])
    core = R @ D @ R.T
    core_q = R @ Dq @ R.T
    core_t = dR @ D @ R.T + R @ D @ dR.T
    core_qq = R @ Dqq @ R.T
    core_qt = dR @ Dq @ R.T + R @ Dq @ dR.T
    core_tt = d2R @ D @ R.T + 2.0 * dR @ D @ dR.T + R @ D @ d2R.T
    W = s * s * core
    dW = np.stack([s * s * core_q, s * s * core_t, 2.0 * s * core])
    d2W = np.empty((3, 3, 2, 2))
    d2W[0, 0] = s * s * core_qq
    d2W[0, 1] = d2W[1, 0] = s * s * core_qt
    d2W[0, 2] = d2W[2, 0] = 2.0 * s * core_q
    d2W[1, 1] = s * s * core_tt
    d2W[1, 2] = d2W[2, 1] = 2.0 * s * core_t
    d2W[2, 2] = 2.0 * core
    return W, dW, d2W


# ----------------------------------------------------------------------------
# one bivariate Gaussian and its derivatives (O3/O4 building block)
# ----------------------------------------------------------------------------

def _quad(b, M):
    """b_n' M b_n for each row of b (n,2)."""
    return M[0, 0] * b[:, 0] ** 2 + (M[0, 1] + M[1, 0]) * b[:, 0] * b[:, 1] + M[1, 1] * b[:, 1] ** 2


def gaussian_value(d, C):
    """Density N(p; mu, C) at offsets d = p - mu (n,2)."""
    P = np.linalg.inv(C)
    return np.exp(-math.log(2.0 * math.pi) - 0.5 * math.log(np.linalg.det(C)) - 0.5 * _quad(d, P))


def gaussian_with_derivs(d, C, dC=None, d2C=None):
    """Density N(p; mu, C) at offsets d = p - mu (n,2), with derivatives.

    Derivatives are taken with respect to x = (mu_x, mu_y, eta_1..eta_k) where C depends
    on eta through dC (k,2,2) and d2C (k,k,2,2).  Uses, with P = C^{-1} and b = P d:
      dlogN/dmu = b,     d2logN/dmu2 = -P,
      dlogN/deta = (b' C_e b - tr(P C_e)) / 2,
      d2logN/dmu deta = -P C_e b,
      d2logN/deta deta' = -b' C_e P C_e' b + tr(P C_e P C_e')/2 + (b' C_ee' b - tr(P C_ee'))/2,
    and N' = N dlogN, N'' = N (dlogN dlogN^T + d2logN).
    Returns N (n,), grad (n,2+k), hess (n,2+k,2+k).
    """
    n = d.shape[0]
    k = 0 if dC is None else dC.shape[0]
    P = np.linalg.inv(C)
    det = np.linalg.det(C)
    b = d @ P.T                                         # (n,2)
    logN = -math.log(2.0 * math.pi) - 0.5 * math.log(det) - 0.5 * _quad(d, P)
    N = np.exp(logN)
    D = 2 + k
    g = np.empty((n, D))
    h = np.empty((n, D, D))
    g[:, 0:2] = b
    h[:, 0:2, 0:2] = -P[None, :, :]
    for e in range(k):
        Ce = dC[e]
        g[:, 2 + e] = 0.5 * (_quad(b, Ce) - np.trace(P @ Ce))
        h[:, 0:2, 2 + e] = -(b @ (P @ Ce).T)
        h[:, 2 + e, 0:2] = h[:, 0:2, 2 + e]
        for f in range(k):
            Cf = dC[f]
            Cef = d2C[e, f]
            h[:, 2 + e, 2 + f] = (-_quad(b, Ce @ P @ Cf)
                                  + 0.5 * np.trace(P @ Ce @ P @ Cf)
                                  + 0.5 * (_quad(b, Cef) - np.trace(P @ Cef)))
    grad = N[:, None] * g
    hess = N[:, None, None] * (g[:, :, None] * g[:, None, :] + h)
    return N, grad, hess


def _psf_cov(row):
    return np.array([[row[3], row[4]], [row[4], row[5]]])


def star_mixture(dpix, psf):
    """Star profile G_s = sum_k w_k N(p; p_s + xi_k, Sigma_k) at dpix = p - p_s (O3).

    Returns value (n,), gradient wrt p_s (n,2), Hessian (n,2,2).
    """
    n = dpix.shape[0]
    G = np.zeros(n)
    dG = np.zeros((n, 2))
    d2G = np.zeros((n, 2, 2))
    for row in psf:
        N, g, h = gaussian_with_derivs(dpix - row[1:3][None, :], _psf_cov(row))
        G += row[0] * N
        dG += row[0] * g
        d2G += row[0] * h
    return G, dG, d2G


def star_value(dpix, psf):
    """Value-only star profile G_s (O3)."""
    G = np.zeros(dpix.shape[0])
    for row in psf:
        G += row[0] * gaussian_value(dpix - row[1:3][None, :], _psf_cov(row))
    return G


def galaxy_value(dpix, psf, e_dev, e_axis, e_angle, e_scale, profiles, A=np.eye(2)):
    """Value-only galaxy profile G_g (O4)."""
    W = A @ shape_matrix(e_axis, e_angle, e_scale)[0] @ A.T
    G = np.zeros(dpix.shape[0])
    for row in psf:
        Sig = _psf_cov(row)
        for name, mix in (("dev", e_dev), ("exp", 1.0 - e_dev)):
            amp, var = profiles[name]
            for aj, nu in zip(amp, var):
                G += row[0] * aj * mix * gaussian_value(dpix - row[1:3][None, :], nu * W + Sig)
    return G


def galaxy_mixture(dpix, psf, e_dev, e_axis, e_angle, e_scale, profiles, A=np.eye(2)):
    """Galaxy profile G_g (O4) with derivatives wrt y = (p_x, p_y, e_dev, e_axis, e_angle, e_scale).

    G_g = sum_k w_k [e_dev sum_j a^dev_j N(p; p_s+xi_k, nu^dev_j W + Sigma_k)
                    + (1-e_dev) sum_j a^exp_j N(p; p_s+xi_k, nu^exp_j W + Sigma_k)]
    with W the shape matrix mapped into the image frame by the WCS matrix A.
    """
    n = dpix.shape[0]
    W, dW, d2W = shape_matrix(e_axis, e_angle, e_scale)
    W = A @ W @ A.T
    dW = np.stack([A @ m @ A.T for m in dW])
    d2W = np.stack([np.stack([A @ d2W[i, j] @ A.T for j in range(3)]) for i in range(3)])
    G = np.zeros(n)
    dG = np.zeros((n, 6))
    d2G = np.zeros((n, 6, 6))
    five = [0, 1, 3, 4, 5]               # y-indices of (p_x, p_y, e_axis, e_angle, e_scale)
    fi, fj = np.ix_(five, five)
    for row in psf:
        Sig = _psf_cov(row)
        for name, mix in (("dev", e_dev), ("exp", 1.0 - e_dev)):
            sign = 1.0 if name == "dev" else -1.0
            amp, var = profiles[name]
            for aj, nu in zip(amp, var):
                N, g, h = gaussian_with_derivs(dpix - row[1:3][None, :], nu * W + Sig, nu * dW, nu * d2W)
                wt = row[0] * aj
                G += wt * mix * N
                dG[:, 2] += wt * sign * N                       # d/de_dev
                dG[:, five] += wt * mix * g
                d2G[:, five, 2] += wt * sign * g                # d2/de_dev d(.)
                d2G[:, 2, five] += wt * sign * g
                d2G[:, fi, fj] += wt * mix * h
    return G, dG, d2G


# ----------------------------------------------------------------------------
# pixel rate moments and the delta-method pixel term (O5, O6)
# ----------------------------------------------------------------------------

def _embed_star(G, dG, d2G):
    n = G.shape[0]
    g = np.zeros((n, NZ))
    h = np.zeros((n, NZ, NZ))
    g[:, Z_PX:Z_PY + 1] = dG
    h[:, Z_PX:Z_PY + 1, Z_PX:Z_PY + 1] = d2G
    return Jet(G, g, h)


def _embed_gal(G, dG, d2G):
    n = G.shape[0]
    idx = [Z_PX, Z_PY, Z_DEV, Z_AXIS, Z_ANGLE, Z_SCALE]
    g = np.zeros((n, NZ))
    h = np.zeros((n, NZ, NZ))
    g[:, idx] = dG
    h[:, np.ix_(idx, idx)[0], np.ix_(idx, idx)[1]] = d2G
    return Jet(G, g, h)


def rate_moments(z, Gs, Gg, sky, calib, nbr_mean, nbr_var):
    """E[F] and Var[F] per pixel as jets in z (O5).

    F = sky + neighbours + calib * (A l_s G_s + (1-A) l_g G_g), A ~ Bernoulli(a),
    log l_i ~ N(m_i, v_i).  Since A^2 = A,
      E[F]   = sky + nE + calib (a E[l_s] G_s + (1-a) E[l_g] G_g)
      Var[F] = nV + calib^2 (a E[l_s^2] G_s^2 + (1-a) E[l_g^2] G_g^2 - (a E[l_s] G_s + (1-a) E[l_g] G_g)^2).
    """
    n = Gs.v.shape[0]
    a = Jet.var(z[Z_A], Z_A, n)
    ms, vs = Jet.var(z[Z_MS], Z_MS, n), Jet.var(z[Z_VS], Z_VS, n)
    mg, vg = Jet.var(z[Z_MG], Z_MG, n), Jet.var(z[Z_VG], Z_VG, n)
    mu_s = (ms + 0.5 * vs).exp()
    mu_g = (mg + 0.5 * vg).exp()
    nu_s = (2.0 * ms + 2.0 * vs).exp()
    nu_g = (2.0 * mg + 2.0 * vg).exp()
    one_m_a = 1.0 - a
    mean_src = a * mu_s * Gs + one_m_a * mu_g * Gg
    second = a * nu_s * Gs.square() + one_m_a * nu_g * Gg.square()
    E = calib * mean_src + (sky + nbr_mean)
    V = (calib * calib) * (second - mean_src.square()) + nbr_var
    return E, V


def rate_values(z, Gs, Gg, sky, calib, nbr_mean, nbr_var):
    """Value-only form of rate_moments on plain arrays."""
    a = z[Z_A]
    mu_s, nu_s = lognormal_moments(z[Z_MS], z[Z_VS])
    mu_g, nu_g = lognormal_moments(z[Z_MG], z[Z_VG])
    mean_src = a * mu_s * Gs + (1.0 - a) * mu_g * Gg
    second = a * nu_s * Gs ** 2 + (1.0 - a) * nu_g * Gg ** 2
    return sky + nbr_mean + calib * mean_src, nbr_var + calib * calib * (second - mean_src ** 2)


def pixel_term(x, E, V):
    """Delta-method expected Poisson log-likelihood per pixel (O6), as a jet.

    E_q[x log F - F - log x!] ~= x (log E - V / (2 E^2)) - E - lgamma(x + 1).
    """
    e, v = E.v, V.v
    val = x * (np.log(e) - v / (2.0 * e * e)) - e - gammaln(x + 1.0)
    lE = x / e + x * v / e ** 3 - 1.0
    lV = -x / (2.0 * e * e)
    lEE = -x / e ** 2 - 3.0 * x * v / e ** 4
    lEV = x / e ** 3
    g = E.g * lE[:, None] + V.g * lV[:, None]
    h = (E.h * lE[:, None, None] + V.h * lV[:, None, None]
         + E.g[:, :, None] * E.g[:, None, :] * lEE[:, None, None]
         + (E.g[:, :, None] * V.g[:, None, :] + V.g[:, :, None] * E.g[:, None, :]) * lEV[:, None, None])
    return Jet(val, g, h)


def pixel_value(x, e, v):
    """Value-only form of pixel_term on plain arrays."""
    return x * (np.log(e) - v / (2.0 * e * e)) - e - gammaln(x + 1.0)


# ----------------------------------------------------------------------------
# per-image z-space sums and the theta projection
# ----------------------------------------------------------------------------

def image_z(theta, band, wcs):
    """z for one image: (a, m_s, v_s, m_g, v_g, p_x, p_y, e_dev, e_axis, e_angle, e_scale)."""
    A = np.array([[wcs[0], wcs[1]], [wcs[2], wcs[3]]])
    p = A @ theta[0:2] + wcs[4:6]
    m_s, v_s, m_g, v_g = band_moments(theta, band)
    return np.array([theta[I_A], m_s, v_s, m_g, v_g, p[0], p[1],
                     theta[I_DEV], theta[I_AXIS], theta[I_ANGLE], theta[I_SCALE]])


def image_jacobian(band, wcs):
    """J (11,27) with dz = J dtheta for one image (theta -> z is linear)."""
    J = np.zeros((NZ, NP))
    S = COLOUR_SIGNS[band]
    J[Z_A, I_A] = 1.0
    J[Z_MS, I_R1[0]] = 1.0
    J[Z_MS, I_C1[0]] = S
    J[Z_VS, I_R2[0]] = 1.0
    J[Z_VS, I_C2[0]] = S * S
    J[Z_MG, I_R1[1]] = 1.0
    J[Z_MG, I_C1[1]] = S
    J[Z_VG, I_R2[1]] = 1.0
    J[Z_VG, I_C2[1]] = S * S
    J[Z_PX, 0:2] = wcs[0:2]
    J[Z_PY, 0:2] = wcs[2:4]
    J[Z_DEV, I_DEV] = 1.0
    J[Z_AXIS, I_AXIS] = 1.0
    J[Z_ANGLE, I_ANGLE] = 1.0
    J[Z_SCALE, I_SCALE] = 1.0
    return J


def image_pixel_grid(h, w, origin):
    """Image-frame centres of the h x w patch elements, row-major: (n,2) as (x, y)."""
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    return np.stack([origin[0] + c.ravel(), origin[1] + r.ravel()], axis=1).astype(np.float64)


def image_sums(theta, img, profiles, want_derivs=True, chunk=8192):
    """Sum over one image's patch of the pixel term: value and (optionally) z-gradient/Hessian.

    img: dict with band, h, w, origin, wcs, sky, calib, psf (K,6), pixels (h,w) and optional
    nbr_mean / nbr_var (h,w) arrays.

    Optional img["weights"] (h,w): the pixel-subsampled sum (the paper's closing section names
    subsampling pixels, "doubly" stochastic VI, as a further speed-up).  Each pixel's term is
    split into the part that does not depend on theta, c = x log E_bg - E_bg - lgamma(x+1)
    with E_bg = sky + nbr_mean (the term with no light from the source), and the rest; the
    estimate is sum c + w (term - c).  Weights 1/p on pixels kept with probability p and 0 on
    the others make it unbiased.
    """
    z = image_z(theta, img["band"], img["wcs"])
    A = np.array([[img["wcs"][0], img["wcs"][1]], [img["wcs"][2], img["wcs"][3]]])
    grid = image_pixel_grid(img["h"], img["w"], img["origin"])
    x = np.asarray(img["pixels"], dtype=np.float64).ravel()
    nE = img.get("nbr_mean")
    nV = img.get("nbr_var")
    nE = np.zeros_like(x) if nE is None else np.asarray(nE, np.float64).ravel()
    nV = np.zeros_like(x) if nV is None else np.asarray(nV, np.float64).ravel()
    wts = img.get("weights")
    wts = None if wts is None else np.asarray(wts, np.float64).ravel()
    val = 0.0
    g = np.zeros(NZ)
    H = np.zeros((NZ, NZ))
    for a in range(0, x.size, chunk):
        b = min(x.size, a + chunk)
        dpix = grid[a:b] - z[Z_PX:Z_PY + 1][None, :]
        if wts is not None:
            # the theta-free part of every pixel, counted in full
            c = pixel_value(x[a:b], img["sky"] + nE[a:b], np.zeros(b - a))
            val += ((1.0 - wts[a:b]) * c).sum()
        w = None if wts is None else wts[a:b]
        if not want_derivs:
            Gs = star_value(dpix, img["psf"])
            Gg = galaxy_value(dpix, img["psf"], z[Z_DEV], z[Z_AXIS], z[Z_ANGLE], z[Z_SCALE], profiles, A)
            e, v = rate_values(z, Gs, Gg, img["sky"], img["calib"], nE[a:b], nV[a:b])
            pv = pixel_value(x[a:b], e, v)
            val += pv.sum() if w is None else (w * pv).sum()
            continue
        Gs = _embed_star(*star_mixture(dpix, img["psf"]))
        Gg = _embed_gal(*galaxy_mixture(dpix, img["psf"], z[Z_DEV], z[Z_AXIS], z[Z_ANGLE], z[Z_SCALE],
                                        profiles, A))
        E, V = rate_moments(z, Gs, Gg, img["sky"], img["calib"], nE[a:b], nV[a:b])
        t = pixel_term(x[a:b], E, V)
        if w is None:
            v_, g_, h_ = t.sum()
        else:
            v_ = (w * t.v).sum()
            g_ = (w[:, None] * t.g).sum(axis=0)
            h_ = (w[:, None, None] * t.h).sum(axis=0)
        val += v_
        g += g_
        H += h_
    return val, g, H


# ----------------------------------------------------------------------------
# Kullback-Leibler terms (O7)
# ----------------------------------------------------------------------------

def kl_terms(theta, prior):
    """Prior part of the ELBO: -KL(q || p) for a, r|a, c|a, with gradient and Hessian in theta.

      KL_a     = a log(a/Phi) + (1-a) log((1-a)/(1-Phi))
      KL_r,i   = [ (r2 + (r1-mu)^2)/s2 - 1 - log(r2/s2) ] / 2          (normal on log r)
      KL_c,i   = [ tr(Xi^-1 diag c2) + (c1-mu)' Xi^-1 (c1-mu) - 4 + log det Xi - sum log c2 ] / 2
      L_prior  = -KL_a - a (KL_r,s + KL_c,s) - (1-a) (KL_r,g + KL_c,g)
    """
    a = theta[I_A]
    phi = prior["p_star"]
    kla = a * math.log(a / phi) + (1 - a) * math.log((1 - a) / (1 - phi))
    dkla = math.log(a / phi) - math.log((1 - a) / (1 - phi))
    d2kla = 1.0 / a + 1.0 / (1.0 - a)
    K = []
    for i in range(2):
        gi = np.zeros(NP)
        hi = np.zeros((NP, NP))
        r1, r2 = theta[I_R1[i]], theta[I_R2[i]]
        mu, s2 = prior["r_mean"][i], prior["r_var"][i]
        kr = 0.5 * ((r2 + (r1 - mu) ** 2) / s2 - 1.0 - math.log(r2 / s2))
        gi[I_R1[i]] = (r1 - mu) / s2
        gi[I_R2[i]] = 0.5 * (1.0 / s2 - 1.0 / r2)
        hi[I_R1[i], I_R1[i]] = 1.0 / s2
        hi[I_R2[i], I_R2[i]] = 0.5 / r2 ** 2
        c1, c2 = theta[I_C1[i]], theta[I_C2[i]]
        Xi = np.asarray(prior["c_cov"][i], dtype=np.float64)
        Xinv = np.linalg.inv(Xi)
        dc = c1 - prior["c_mean"][i]
        kc = 0.5 * (np.sum(np.diag(Xinv) * c2) + dc @ Xinv @ dc - 4.0
                    + math.log(np.linalg.det(Xi)) - np.sum(np.log(c2)))
        gi[I_C1[i]] = Xinv @ dc
        gi[I_C2[i]] = 0.5 * (np.diag(Xinv) - 1.0 / c2)
        hi[I_C1[i], I_C1[i]] = Xinv
        idx = np.arange(NP)[I_C2[i]]
        hi[idx, idx] = 0.5 / c2 ** 2
        K.append((kr + kc, gi, hi))
    (Ks, gs, hs), (Kg, gg, hg) = K
    val = -kla - a * Ks - (1 - a) * Kg
    grad = -a * gs - (1 - a) * gg
    grad[I_A] += -dkla - Ks + Kg
    hess = -a * hs - (1 - a) * hg
    hess[I_A, :] += -gs + gg
    hess[:, I_A] += -gs + gg
    hess[I_A, I_A] += -d2kla
    return val, grad, hess


# ----------------------------------------------------------------------------
# the per-source ELBO (O8, O9)
# ----------------------------------------------------------------------------

def source_images(batch, s, nbr=None):
    """Image dicts for source s of a synth.SynthBatch (host pixels)."""
    out = []
    for i in range(int(batch.src_img_off[s]), int(batch.src_img_off[s + 1])):
        d = dict(band=int(batch.img_band[i]), h=int(batch.img_h[i]), w=int(batch.img_w[i]),
                 origin=batch.img_origin[i], wcs=batch.img_wcs[i], sky=float(batch.img_sky[i]),
                 calib=float(batch.img_calib[i]), psf=batch.img_psf[i][: int(batch.img_npsf[i])],
                 pixels=batch.image_pixels(i))
        if nbr is not None:
            d["nbr_mean"], d["nbr_var"] = nbr[i]
        out.append(d)
    return out


def elbo(theta, images, prior, profiles, want="hess"):
    """ELBO of one source (O8) and, if want == 'hess', its gradient (27) and Hessian (27x27).

    L(theta) = sum_images sum_pixels pixel_term - KL terms.  The Hessian's two triangles
    are accumulated independently (no mirroring) so its symmetry is a real check.
    """
    theta = np.asarray(theta, dtype=np.float64)
    derivs = want == "hess"
    val, g, H = kl_terms(theta, prior)
    if not derivs:
        g, H = None, None
    for img in images:
        v_, gz, Hz = image_sums(theta, img, profiles, want_derivs=derivs)
        val += v_
        if derivs:
            J = image_jacobian(img["band"], img["wcs"])
            g = g + J.T @ gz
            H = H + J.T @ Hz @ J
    if derivs:
        return val, g, H
    return val


def elbo_value(theta, images, prior, profiles):
    return elbo(theta, images, prior, profiles, want="value")
