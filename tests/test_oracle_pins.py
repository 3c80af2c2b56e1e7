"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test ties one oracle function to something other than itself: a library
routine, a closed form, an invariant, numerical quadrature, Monte Carlo or
finite differences.  A plausible mistake (dropped term, wrong sign or index,
transposed operand) in the oracle breaks at least one of them.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss
from scipy import integrate, stats

import synth
from synth.generate import perturb_theta
from oracle import init as oinit
from oracle import model, newton, transforms


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_config(0)


def _img(h=25, w=25, origin=(0.0, 0.0), band=2, sky=100.0, calib=1.0, psf=None, pixels=None, wcs=None, seed=0):
    rng = np.random.default_rng(seed)
    if psf is None:
        psf = np.array([[0.5, 0.0, 0.0, 1.3, 0.1, 1.1], [0.3, 0.2, -0.1, 2.0, -0.2, 2.4],
                        [0.2, -0.1, 0.1, 3.5, 0.3, 3.0]])
    if pixels is None:
        pixels = rng.poisson(sky + 5.0, size=(h, w)).astype(np.float32)
    if wcs is None:
        wcs = np.array([1.0, 0.0, 0.0, 1.0, 0.0, 0.0])
    return dict(band=band, h=h, w=w, origin=np.asarray(origin, float), wcs=np.asarray(wcs, float),
                sky=sky, calib=calib, psf=psf, pixels=pixels)


# ---------------------------------------------------------------------------- P1 / P2 mixtures

def test_gaussian_matches_scipy():
    rng = np.random.default_rng(1)
    d = rng.normal(0, 2, (50, 2))
    C = np.array([[2.3, 0.4], [0.4, 1.1]])
    ours = model.gaussian_value(d, C)
    ref = stats.multivariate_normal(mean=[0, 0], cov=C).pdf(d)
    np.testing.assert_allclose(ours, ref, rtol=1e-13)
    N, g, h = model.gaussian_with_derivs(d, C)
    np.testing.assert_allclose(N, ref, rtol=1e-13)


@pytest.mark.parametrize("kind", ["star", "gal_round", "gal_flat"])
def test_mixture_integrates_to_one(kind):
    """Sum over a unit grid of a mixture with all widths >= 1 px equals its flux (Poisson summation)."""
    psf = np.array([[0.5, 0.0, 0.0, 1.1, 0.05, 1.3], [0.3, 0.3, -0.2, 2.0, -0.2, 2.4],
                    [0.2, -0.1, 0.1, 3.5, 0.3, 3.0]])
    r = np.arange(-60, 61, dtype=float)
    X, Y = np.meshgrid(r, r)
    d = np.stack([X.ravel() + 0.37, Y.ravel() - 0.21], axis=1)
    prof = synth.load_profiles()
    if kind == "star":
        G = model.star_value(d, psf)
    elif kind == "gal_round":
        G = model.galaxy_value(d, psf, 0.3, 1.0, 0.0, 1.2, prof)
    else:
        G = model.galaxy_value(d, psf, 0.7, 0.3, 0.8, 2.0, prof)
    assert abs(G.sum() - 1.0) < 1e-6


def test_rate_flux_sum():
    """sum_px (E - sky) = calib (a E[l_s] + (1-a) E[l_g]) on a patch much larger than the source."""
    th = np.zeros(27)
    th[0:2] = [40.3, 39.8]
    th[2], th[3], th[4], th[5], th[6] = 0.3, 0.4, 0.6, 0.4, 1.5
    th[7:11] = [2.0, 2.5, 0.2, 0.3]
    th[11:19] = 0.3
    th[19:27] = 0.05
    img = _img(h=81, w=81, band=0, calib=2.5)
    z = model.image_z(th, 0, img["wcs"])
    grid = model.image_pixel_grid(81, 81, img["origin"])
    dpix = grid - z[5:7]
    Gs = model.star_value(dpix, img["psf"])
    Gg = model.galaxy_value(dpix, img["psf"], th[3], th[4], th[5], th[6], synth.load_profiles())
    e, v = model.rate_values(z, Gs, Gg, img["sky"], img["calib"], 0.0, 0.0)
    m_s, v_s, m_g, v_g = model.band_moments(th, 0)
    expect = 2.5 * (0.3 * math.exp(m_s + v_s / 2) + 0.7 * math.exp(m_g + v_g / 2))
    assert abs((e - img["sky"]).sum() - expect) < 1e-6 * expect


def test_band_moments_colour_walk():
    """log l_b from r and adjacent-band log ratios, checked against a cumulative walk per band."""
    th = np.zeros(27)
    th[7], th[8] = 1.0, 2.0
    th[9], th[10] = 0.1, 0.2
    c_s = np.array([0.3, -0.2, 0.5, 0.7])
    c_g = np.array([-0.4, 0.1, 0.2, -0.3])
    th[11:15], th[15:19] = c_s, c_g
    th[19:23] = [0.01, 0.02, 0.03, 0.04]
    th[23:27] = [0.05, 0.06, 0.07, 0.08]
    # u = r - c_g_r(1) - c_ug(0); g = r - c1; i = r + c2; z = r + c2 + c3
    exp_ms = [1.0 - 0.3 + 0.2, 1.0 + 0.2, 1.0, 1.5, 2.2]
    exp_vs = [0.1 + 0.03, 0.1 + 0.02, 0.1, 0.13, 0.17]
    for b in range(5):
        m_s, v_s, m_g, v_g = model.band_moments(th, b)
        assert m_s == pytest.approx(exp_ms[b], abs=1e-14)
        assert v_s == pytest.approx(exp_vs[b], abs=1e-14)
    assert model.band_moments(th, 0)[2] == pytest.approx(2.0 + 0.4 - 0.1)
    assert model.band_moments(th, 4)[3] == pytest.approx(0.2 + 0.07 + 0.08)


# ---------------------------------------------------------------------------- P3 Poisson limit

@pytest.mark.parametrize("a", [1.0, 0.0])
def test_zero_variance_limit_is_poisson_logpmf(a):
    th = np.zeros(27)
    th[0:2] = [12.2, 11.7]
    th[2] = a
    th[3:7] = [0.4, 0.6, 0.3, 1.7]
    th[7:9] = [4.0, 4.2]
    th[11:19] = 0.2
    img = _img(band=3, sky=80.0, calib=1.3, seed=3)
    val, _, _ = model.image_sums(th, img, synth.load_profiles(), want_derivs=False)
    z = model.image_z(th, 3, img["wcs"])
    grid = model.image_pixel_grid(img["h"], img["w"], img["origin"])
    prof = synth.load_profiles()
    Gs = model.star_value(grid - z[5:7], img["psf"])
    Gg = model.galaxy_value(grid - z[5:7], img["psf"], *th[3:7], prof)
    m = z[1] if a == 1.0 else z[3]
    G = Gs if a == 1.0 else Gg
    rate = 80.0 + 1.3 * math.exp(m) * G
    ref = stats.poisson.logpmf(img["pixels"].ravel().astype(int), rate).sum()
    assert val == pytest.approx(ref, rel=1e-12)


# ---------------------------------------------------------------------------- P4 / P5 limits and symmetries

def test_galaxy_tends_to_star():
    psf = _img()["psf"]
    r = np.arange(-8, 9, dtype=float)
    X, Y = np.meshgrid(r, r)
    d = np.stack([X.ravel() + 0.25, Y.ravel()], axis=1)
    Gs = model.star_value(d, psf)
    Gg = model.galaxy_value(d, psf, 0.5, 0.5, 0.3, 1e-4, synth.load_profiles())
    np.testing.assert_allclose(Gg, Gs, rtol=1e-6, atol=1e-12)


def test_angle_period_and_round_galaxy(cfg0):
    imgs = model.source_images(cfg0, 0)
    th = perturb_theta(cfg0.theta_truth, 5)[0]
    v1 = model.elbo_value(th, imgs, cfg0.prior, cfg0.profiles)
    th2 = th.copy()
    th2[5] += math.pi
    v2 = model.elbo_value(th2, imgs, cfg0.prior, cfg0.profiles)
    assert v1 == pytest.approx(v2, rel=1e-12)
    th3 = th.copy()
    th3[4] = 1.0
    _, g, _ = model.elbo(th3, imgs, cfg0.prior, cfg0.profiles)
    assert abs(g[5]) <= 1e-9 * np.max(np.abs(g))


def test_integer_translation(cfg0):
    imgs = model.source_images(cfg0, 0)
    th = perturb_theta(cfg0.theta_truth, 6)[0]
    v1, g1, H1 = model.elbo(th, imgs, cfg0.prior, cfg0.profiles)
    th2 = th.copy()
    th2[0:2] += [3.0, -2.0]
    imgs2 = [dict(im, origin=im["origin"] + np.array([3.0, -2.0])) for im in imgs]
    v2, g2, H2 = model.elbo(th2, imgs2, cfg0.prior, cfg0.profiles)
    assert v1 == pytest.approx(v2, rel=1e-13)
    np.testing.assert_allclose(g1, g2, rtol=1e-9, atol=1e-9 * np.max(np.abs(g1)))


# ---------------------------------------------------------------------------- P6 / P7 derivatives

# coordinates whose scale is their value (variances, e_scale) or their distance to the
# bounds of (0, 1) (a, e_dev, e_axis); the others (u in px, e_angle in rad, the log-brightness
# and colour means) have unit scale
_POSITIVE = [6, 9, 10] + list(range(19, 27))
_UNIT = [2, 3, 4]


def _fd_steps(th, rel=1e-2):
    """Per-coordinate steps: rel times the coordinate's scale, so that every step stays inside
    the domain, the rounding of the differenced ELBO values (a few ulp of |L| ~ 2e4, divided
    by the step) stays far below the tolerance, and the O(h^4) error left by Richardson
    extrapolation is negligible."""
    s = np.ones_like(th)
    s[_POSITIVE] = th[_POSITIVE]
    s[_UNIT] = np.minimum(th[_UNIT], 1.0 - th[_UNIT])
    return rel * s


def _richardson(f, th, h):
    """Central differences of f along each coordinate, Richardson-extrapolated from steps
    h and h/2: (4 D(h/2) - D(h)) / 3 cancels the h^2 term, leaving an O(h^4) error."""
    out = []
    for j in range(th.size):
        def d(step):
            tp, tm = th.copy(), th.copy()
            tp[j] += step
            tm[j] -= step
            return (f(tp) - f(tm)) / (2.0 * step)
        out.append((4.0 * d(0.5 * h[j]) - d(h[j])) / 3.0)
    return np.array(out)


def _fd_check(th, imgs, prior, profiles, rtol_g=1e-6, rtol_h=1e-6):
    """Analytic gradient and Hessian against Richardson-extrapolated central differences of
    the value (gradient) and of the analytic gradient (Hessian), per entry relative to
    max(|e|, 1e-3 max|array|).  Returns the largest errors (they sit well below the
    tolerance, so harmless changes of the evaluation point do not trip the pin)."""
    v, g, H = model.elbo(th, imgs, prior, profiles)
    assert np.max(np.abs(H - H.T)) <= 1e-12 * np.max(np.abs(H))
    h = _fd_steps(th)
    fdg = _richardson(lambda t: model.elbo_value(t, imgs, prior, profiles), th, h)
    fdH = _richardson(lambda t: model.elbo(t, imgs, prior, profiles)[1], th, h).T
    eg = np.abs(fdg - g) / np.maximum(np.abs(g), 1e-3 * np.max(np.abs(g)))
    eh = np.abs(fdH - H) / np.maximum(np.abs(H), 1e-3 * np.max(np.abs(H)))
    assert eg.max() < rtol_g, (eg.max(), np.argmax(eg))
    assert eh.max() < rtol_h, (eh.max(), np.unravel_index(np.argmax(eh), eh.shape))
    return eg.max(), eh.max()


def test_gradient_hessian_finite_differences(cfg0):
    imgs = model.source_images(cfg0, 0)
    th = perturb_theta(cfg0.theta_truth, 1)[0]
    eg, eh = _fd_check(th, imgs, cfg0.prior, cfg0.profiles)
    assert eg < 1e-7 and eh < 1e-7          # ten times under the tolerance: room for harmless changes


def test_structural_zeros_are_exact(cfg0):
    """Colour entries that share no band and no prior term (A23's structural zeros) are exactly 0
    in the oracle's Hessian, at three points of config 0 and with a general WCS and neighbours."""
    from helpers import assert_structural_zeros, structural_zeros
    assert len(structural_zeros()) == 112
    imgs = model.source_images(cfg0, 0)
    for seed in (1, 2, 3):
        th = perturb_theta(cfg0.theta_truth, seed)[0]
        _, _, H = model.elbo(th, imgs, cfg0.prior, cfg0.profiles)
        assert_structural_zeros(H, what=f"seed {seed}")
        # the entries next to them are not zero: the mask is not trivially satisfied
        assert H[12, 13] != 0.0 and H[13, 14] != 0.0 and H[11, 12] != 0.0


def test_fd_general_wcs_and_neighbours():
    """Non-identity WCS (rotation + scale + offset), per-pixel neighbour mean/variance, two bands."""
    rng = np.random.default_rng(7)
    prof = synth.load_profiles()
    ang = 0.3
    A = 1.1 * np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    imgs = []
    for band in (1, 4):
        im = _img(h=19, w=21, origin=(-3.0, -4.0), band=band, sky=60.0, calib=3.0, seed=band,
                  wcs=np.array([A[0, 0], A[0, 1], A[1, 0], A[1, 1], 0.3, -0.2]))
        im["nbr_mean"] = rng.uniform(0, 20, (19, 21))
        im["nbr_var"] = rng.uniform(0, 5, (19, 21))
        imgs.append(im)
    th = perturb_theta(np.array([[5.2, 4.1] + [0.5] * 5 + [3.0, 3.2, 0.1, 0.1] + [0.3] * 8 + [0.05] * 8]), 3)[0]
    eg, eh = _fd_check(th, imgs, synth.PRIOR, prof)
    assert eg < 1e-7 and eh < 1e-7


# ---------------------------------------------------------------------------- P8 delta method

def _exact_elog(eps, calib, a, G_s, G_g, ms, vs, mg, vg, nodes=80):
    xs, ws = hermegauss(nodes)
    ws = ws / ws.sum()
    ls = np.exp(ms + math.sqrt(vs) * xs)
    lg = np.exp(mg + math.sqrt(vg) * xs)
    return (a * np.sum(ws * np.log(eps + calib * ls * G_s))
            + (1 - a) * np.sum(ws * np.log(eps + calib * lg * G_g)))


def test_delta_method_vs_quadrature_and_monte_carlo():
    """Conditional on a, log l_b is normal: E[log F] is a 1-D Gauss-Hermite integral (exact to ~1e-12)."""
    rng = np.random.default_rng(11)
    th = np.zeros(27)
    th[0:2] = [4.1, 3.8]
    th[2:7] = [0.4, 0.5, 0.7, 0.2, 1.2]
    th[7:9] = [math.log(20.0), math.log(25.0)]
    th[9:11] = [0.1, 0.15]
    th[11:19] = rng.normal(0.3, 0.1, 8)
    th[19:27] = 0.01
    prof = synth.load_profiles()
    img = _img(h=9, w=9, band=2, sky=100.0, seed=4)
    z = model.image_z(th, 2, img["wcs"])
    grid = model.image_pixel_grid(9, 9, img["origin"])
    Gs = model.star_value(grid - z[5:7], img["psf"])
    Gg = model.galaxy_value(grid - z[5:7], img["psf"], *th[3:7], prof)
    e, v = model.rate_values(z, Gs, Gg, 100.0, 1.0, 0.0, 0.0)
    delta = np.log(e) - v / (2 * e * e)
    exact = np.array([_exact_elog(100.0, 1.0, th[2], Gs[i], Gg[i], *z[1:5]) for i in range(81)])
    # faint regime: the delta-method error is below 1e-7 per pixel and well below its own correction
    assert np.max(np.abs(delta - exact)) < 1e-7
    assert np.max(np.abs(delta - exact)) < 0.05 * np.max(v / (2 * e * e))
    # brute-force Monte Carlo over (a, r, c) at the brightest pixel agrees with the quadrature
    i = int(np.argmax(Gs + Gg))
    n = 2_000_000
    A_ = rng.random(n) < th[2]
    lr_s = rng.normal(th[7], math.sqrt(th[9]), n)
    lr_g = rng.normal(th[8], math.sqrt(th[10]), n)
    # band r: no colour dependence
    F = 100.0 + np.where(A_, np.exp(lr_s) * Gs[i], np.exp(lr_g) * Gg[i])
    lf = np.log(F)
    se = lf.std() / math.sqrt(n)
    assert abs(lf.mean() - exact[i]) < 4 * se
    # bright, high-variance regime: the approximation error grows as expected (documented, not hidden)
    big = _exact_elog(100.0, 1.0, 1.0, 0.05, 0.05, math.log(1e4), 1.0, 0, 1) - (
        lambda E, V: math.log(E) - V / (2 * E * E))(100 + 0.05 * math.exp(math.log(1e4) + 0.5),
                                                      (math.exp(2 * math.log(1e4) + 2) - math.exp(2 * math.log(1e4) + 1)) * 0.0025)
    assert 0.1 < big < 1.0


def test_pixel_term_band_colour_mc():
    """Monte Carlo over colours: in band u the log-flux variance includes two colour variances."""
    rng = np.random.default_rng(12)
    th = np.zeros(27)
    th[7:11] = [3.0, 3.0, 0.05, 0.05]
    th[11:15] = [0.4, 0.3, 0.2, 0.1]
    th[19:23] = [0.2, 0.3, 0.01, 0.01]
    m_s, v_s, _, _ = model.band_moments(th, 0)
    n = 1_000_000
    lr = rng.normal(3.0, math.sqrt(0.05), n)
    c0 = rng.normal(0.4, math.sqrt(0.2), n)
    c1 = rng.normal(0.3, math.sqrt(0.3), n)
    lu = lr - c1 - c0
    assert abs(lu.mean() - m_s) < 4 * lu.std() / math.sqrt(n)
    assert abs(lu.var() - v_s) < 0.01 * v_s


# ---------------------------------------------------------------------------- P9 KL

def test_kl_terms_against_integration():
    prior = synth.PRIOR
    rng = np.random.default_rng(2)
    th = np.zeros(27)
    th[2] = 0.37
    th[7:11] = [2.5, 3.4, 0.3, 0.6]
    th[11:19] = rng.normal(0.5, 0.3, 8)
    th[19:27] = rng.uniform(0.01, 0.1, 8)
    val, g, H = model.kl_terms(th, prior)
    kls = []
    for i in range(2):
        q = stats.norm(th[7 + i], math.sqrt(th[9 + i]))
        p = stats.norm(prior["r_mean"][i], math.sqrt(prior["r_var"][i]))
        klr = integrate.quad(lambda x: q.pdf(x) * (q.logpdf(x) - p.logpdf(x)), -30, 30, limit=200)[0]
        qc = stats.multivariate_normal(th[11 + 4 * i:15 + 4 * i], np.diag(th[19 + 4 * i:23 + 4 * i]))
        pc = stats.multivariate_normal(prior["c_mean"][i], prior["c_cov"][i])
        xs = qc.rvs(size=400_000, random_state=rng)
        d = qc.logpdf(xs) - pc.logpdf(xs)
        kls.append((klr, d.mean(), d.std() / math.sqrt(xs.shape[0])))
    a, phi = th[2], prior["p_star"]
    kla = a * math.log(a / phi) + (1 - a) * math.log((1 - a) / (1 - phi))
    mc = -kla - a * (kls[0][0] + kls[0][1]) - (1 - a) * (kls[1][0] + kls[1][1])
    se = math.hypot(a * kls[0][2], (1 - a) * kls[1][2])
    assert abs(val - mc) < 4 * se + 1e-9
    # derivatives of the KL part by finite differences
    for j in range(27):
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        fd = (model.kl_terms(tp, prior)[0] - model.kl_terms(tm, prior)[0]) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-7)
        fdh = (model.kl_terms(tp, prior)[1] - model.kl_terms(tm, prior)[1]) / (2 * h)
        np.testing.assert_allclose(fdh, H[:, j], rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------------------- transforms

def test_transforms_roundtrip_and_derivatives():
    th = perturb_theta(np.array([[5.0, 5.0, 0.5, 0.5, 0.5, 1.0, 1.5, 3, 3, .1, .1] + [0.2] * 8 + [0.05] * 8]), 9)[0]
    u0 = np.array([5.2, 4.9])
    psi = transforms.to_psi(th, u0)
    back, d1, d2 = transforms.to_theta(psi, u0)
    np.testing.assert_allclose(back, th, rtol=1e-12, atol=1e-12)
    h = 1e-5
    for j in range(27):
        pp, pm = psi.copy(), psi.copy()
        pp[j] += h
        pm[j] -= h
        tp, tm = transforms.to_theta(pp, u0)[0][j], transforms.to_theta(pm, u0)[0][j]
        assert (tp - tm) / (2 * h) == pytest.approx(d1[j], rel=1e-7, abs=1e-12)
        assert (tp - 2 * back[j] + tm) / h ** 2 == pytest.approx(d2[j], rel=1e-3, abs=1e-5)


# ---------------------------------------------------------------------------- P10 TR subproblem

@pytest.mark.parametrize("case", ["pd_interior", "pd_boundary", "indefinite", "hard"])
def test_tr_subproblem_kkt(case):
    rng = np.random.default_rng({"pd_interior": 1, "pd_boundary": 2, "indefinite": 3, "hard": 4}[case])
    n = 27
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = rng.uniform(0.5, 5.0, n)
    if case in ("indefinite", "hard"):
        lam[:3] = [-2.0, -0.5, 0.1]
    B = Q @ np.diag(lam) @ Q.T
    H = -B
    g = rng.normal(size=n)
    if case == "hard":
        g -= Q[:, 0] * (Q[:, 0] @ g)        # g orthogonal to the bottom eigenvector
        g *= 1e-2
    delta = {"pd_interior": 100.0, "pd_boundary": 0.1, "indefinite": 0.7, "hard": 3.0}[case]
    p, pred, s, lam_sorted = newton.tr_subproblem(g, H, delta)
    # KKT: (B + sI) p = g, s >= 0, s (delta - |p|) = 0, B + sI psd, |p| <= delta
    np.testing.assert_allclose((B + s * np.eye(n)) @ p, g, atol=1e-10 * max(1, np.linalg.norm(g)))
    assert s >= 0
    assert np.linalg.norm(p) <= delta * (1 + 1e-10)
    assert abs(s * (delta - np.linalg.norm(p))) < 1e-9
    assert np.linalg.eigvalsh(B + s * np.eye(n))[0] >= -1e-10
    assert pred == pytest.approx(g @ p - 0.5 * p @ B @ p, rel=1e-12)
    if case == "pd_interior":
        np.testing.assert_allclose(p, np.linalg.solve(B, g), rtol=1e-10)
    # the step beats random feasible points
    for _ in range(50):
        r = rng.normal(size=n)
        r *= delta * rng.random() / np.linalg.norm(r)
        assert g @ r - 0.5 * r @ B @ r <= pred + 1e-12


# ---------------------------------------------------------------------------- P11 fit invariants

def test_fit_config0_invariants(cfg0):
    imgs = model.source_images(cfg0, 0)
    th0 = oinit.plain_init(cfg0.u_cat[0], imgs, cfg0.prior)
    res = newton.fit(th0, imgs, cfg0.prior, cfg0.profiles, record=True)
    assert res.status == newton.CONVERGED
    assert res.iters <= 50
    el = [h["elbo"] for h in res.history]
    assert all(b >= a - 1e-9 for a, b in zip(el, el[1:]))
    # the converged ELBO beats the start and the point near the truth
    v0 = model.elbo_value(th0, imgs, cfg0.prior, cfg0.profiles)
    vt = model.elbo_value(cfg0.theta_truth[0], imgs, cfg0.prior, cfg0.profiles)
    assert res.elbo >= v0 and res.elbo >= vt - 1e-6 * abs(vt)
    # gradient in psi is (near) zero at the optimum
    psi = transforms.to_psi(res.theta, th0[0:2])
    th, d1, d2 = transforms.to_theta(psi, th0[0:2])
    f, g, H = model.elbo(th, imgs, cfg0.prior, cfg0.profiles)
    gp, Hp = transforms.grad_hess_psi(g, H, d1, d2)
    newton_gain = 0.5 * gp @ np.linalg.solve(-Hp, gp) if np.all(np.linalg.eigvalsh(-Hp) > 0) else np.inf
    assert newton_gain < 1e-6 * abs(f)


# ---------------------------------------------------------------------------- plain init

def test_plain_init_aperture_brute_force():
    img = _img(h=15, w=15, origin=(0.0, 0.0), band=2, sky=50.0, calib=2.0)
    x = np.full((15, 15), 50.0, np.float32)
    x[7, 7] += 60.0          # inside (distance 0)
    x[7, 10] += 20.0         # inside (distance 3)
    x[7, 11] += 1000.0       # outside (distance 4)
    x[10, 9] += 40.0         # distance sqrt(13) > 3: outside
    img["pixels"] = x
    th = oinit.plain_init(np.array([7.0, 7.0]), [img], synth.PRIOR)
    assert th[7] == pytest.approx(math.log((60.0 + 20.0) / 2.0))
    assert th[2] == 0.5 and th[6] == 1.5


# ---------------------------------------------------------------------------- model constants

def test_profile_tables():
    prof = synth.load_profiles()
    for name in ("exp", "dev"):
        amp, var = prof[name]
        assert abs(amp.sum() - 1.0) < 1e-12
        assert np.all(var > 0)
        # half the light of the prototype lies (nearly) within r_e = 1
        frac = np.sum(amp * (1 - np.exp(-0.5 / var)))
        assert abs(frac - 0.5) < 0.01
