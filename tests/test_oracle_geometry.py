"""Pins of the oracle's geometric conventions (CPU only).

The model of section III-A places each source's light on the image through its position
and galaxy shape; the readings shared by the oracle and the kernels are:

  * the source frame maps to an image by p = A u + b (A row-major from wcs[0:4], b = wcs[4:6]);
  * element (r, c) of a patch has its centre at origin + (c, r): x runs along columns,
    y along rows;
  * the galaxy's major axis lies at e_angle counter-clockwise from +x (towards +y), with
    minor/major ratio e_axis and half-light radius e_scale, and the shape is stretched by A.

Three independent pins fix them:

  1. photons shot by the generator's own sampler (synth.generate, which draws PSF, profile
     and shape offsets by code of its own and bins photons into pixels by column = x,
     row = y) give a histogram whose first and second moments equal those of the oracle's
     density on the same patch;
  2. the conventions restated on the array axes of the oracle's density (major axis along
     columns at angle 0, along rows at pi/2, at the stated angle in between; a quarter-turn
     WCS turns the major axis onto the rows);
  3. the whole model: on the bright variant, oracle fits from the plain start recover the
     generator's truth within 3 linear-response standard deviations for at least 90% of the
     identifiable parameters (and for most of each group).

A rotation in the wrong sense, swapped pixel axes or a transposed WCS matrix fails each.
"""
import math
import multiprocessing as mp
import os

import numpy as np
import pytest

import synth
from synth.generate import _bin_photons, _shoot_photons
from oracle import init as oinit
from oracle import lr, model, newton

PSF = np.array([[0.5, 0.0, 0.0, 1.2, 0.15, 1.0],
                [0.3, 0.25, -0.15, 2.1, -0.2, 2.6],
                [0.2, -0.1, 0.2, 3.3, 0.4, 2.9]])
POINT = np.array([[[1.0, 0.0, 0.0, 1e-24, 0.0, 1e-24]]])    # a PSF of one point-like component


def _shoot(rng, n, psf, shape, A, p_s, profiles):
    """Image positions of n photons of one galaxy: shape offsets drawn in the source frame by
    the generator, mapped by A, plus PSF offsets drawn by the generator, at image position p_s."""
    zero = np.zeros(n, dtype=np.int64)
    gal = _shoot_photons(rng, zero, np.zeros((1, 2)), POINT, np.array([False]), np.asarray([shape]), profiles)
    blur = _shoot_photons(rng, zero, np.zeros((1, 2)), psf[None], np.array([True]), np.zeros((1, 4)), profiles)
    return p_s[None, :] + gal @ A.T + blur


def _moments(wt, h, w, origin):
    """Normalised mean (x, y) and covariance of weights wt (h x w, row-major) placed at the
    element centres origin + (c, r), computed from the array axes alone."""
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    x = origin[0] + c
    y = origin[1] + r
    tot = wt.sum()
    mx, my = (wt * x).sum() / tot, (wt * y).sum() / tot
    cxx = (wt * (x - mx) ** 2).sum() / tot
    cyy = (wt * (y - my) ** 2).sum() / tot
    cxy = (wt * (x - mx) * (y - my)).sum() / tot
    return np.array([mx, my]), np.array([[cxx, cxy], [cxy, cyy]])


CASES = [
    # e_dev, e_axis, e_angle, e_scale, wcs (A row-major, b), h, w, origin, u
    (0.2, 0.3, 0.5, 2.2, (1.0, 0.0, 0.0, 1.0, 0.3, -0.2), 61, 79, (-30.0, -20.0), (4.3, 7.6)),
    (0.8, 0.25, 2.3, 1.4, (0.9, -0.35, 0.3, 1.1, 1.7, 0.4), 71, 53, (-20.0, -30.0), (-2.2, 3.1)),
    (0.5, 0.45, 1.2, 1.8, (0.0, -1.0, 1.0, 0.0, -3.5, 2.0), 57, 66, (-36.0, -25.0), (1.5, -2.5)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_photon_histogram_moments_match_oracle_density(case):
    e_dev, e_axis, e_angle, e_scale, wcs, h, w, origin, u = CASES[case]
    profiles = synth.load_profiles()
    wcs = np.asarray(wcs, float)
    A = wcs[:4].reshape(2, 2)
    p_s = A @ np.asarray(u, float) + wcs[4:6]
    origin = np.asarray(origin, float)
    n = 1_000_000
    rng = np.random.default_rng(20170 + case)
    xy = _shoot(rng, n, PSF, (e_dev, e_axis, e_angle, e_scale), A, p_s, profiles)
    idx, cnt = _bin_photons(xy, np.zeros(n, np.int64), origin[None], np.array([h]), np.array([w]),
                            np.array([0], np.int64))
    hist = np.zeros(h * w)
    hist[idx] = cnt
    hist = hist.reshape(h, w)
    assert hist.sum() >= 0.995 * n          # the patch holds (nearly) all of the light

    # the oracle's density at the patch's element centres, in its own grid order
    dpix = model.image_pixel_grid(h, w, origin) - p_s[None, :]
    G = model.galaxy_value(dpix, PSF, e_dev, e_axis, e_angle, e_scale, profiles, A=A).reshape(h, w)
    assert G.sum() == pytest.approx(hist.sum() / n, abs=2e-3)

    m_h, C_h = _moments(hist, h, w, origin)
    m_o, C_o = _moments(G, h, w, origin)
    C_h = C_h - np.eye(2) / 12.0           # binning into unit pixels adds 1/12 px^2 per axis
    # standard errors of the photon moments, plus an allowance for point sampling vs binning
    se_m = np.sqrt(np.diag(C_h) / hist.sum())
    se_c = np.sqrt((np.outer(np.diag(C_h), np.diag(C_h)) + C_h ** 2) / hist.sum())
    assert np.all(np.abs(m_h - m_o) <= 5 * se_m + 2e-3), (m_h, m_o, se_m)
    assert np.all(np.abs(C_h - C_o) <= 5 * se_c + 1e-2 * np.abs(C_o).max()), (C_h, C_o, se_c)
    # the elongation is strong enough that the off-diagonal sign is far outside the noise
    assert abs(C_o[0, 1]) > 20 * se_c[0, 1]


def _gal_image(h, w, origin, u, e_angle, A=np.eye(2), b=(0.0, 0.0)):
    psf = np.array([[1.0, 0.0, 0.0, 1.0, 0.0, 1.0]])
    p_s = A @ np.asarray(u, float) + np.asarray(b, float)
    dpix = model.image_pixel_grid(h, w, np.asarray(origin, float)) - p_s[None, :]
    return model.galaxy_value(dpix, psf, 0.0, 0.2, e_angle, 3.0, synth.load_profiles(), A=A).reshape(h, w)


def test_axis_conventions_on_array_axes():
    h, w, origin, u = 41, 57, (-20.0, -30.0), (3.0, -5.0)
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")

    def spread(G):
        tot = G.sum()
        mc, mr = (G * c).sum() / tot, (G * r).sum() / tot
        vc = (G * (c - mc) ** 2).sum() / tot
        vr = (G * (r - mr) ** 2).sum() / tot
        cv = (G * (c - mc) * (r - mr)).sum() / tot
        return mc, mr, vc, vr, cv

    # position: the density peaks at column x - origin_x, row y - origin_y
    G = _gal_image(h, w, origin, u, 0.0)
    rr, cc = np.unravel_index(np.argmax(G), G.shape)
    assert (cc, rr) == (u[0] - origin[0], u[1] - origin[1])
    mc, mr, vc, vr, cv = spread(G)
    assert (mc, mr) == pytest.approx((u[0] - origin[0], u[1] - origin[1]), abs=1e-3)   # tails cut by the patch
    # angle 0: major axis along +x, i.e. along the columns
    assert vc > 3 * vr and abs(cv) < 1e-9 * vc
    # angle pi/2: along +y, the rows
    _, _, vc, vr, cv = spread(_gal_image(h, w, origin, u, math.pi / 2))
    assert vr > 3 * vc and abs(cv) < 1e-9 * vr
    # angle t: the principal axis points at t counter-clockwise from +x (towards +y = rows)
    for t in (math.pi / 6, 2.0, 2.9):
        _, _, vc, vr, cv = spread(_gal_image(h, w, origin, u, t))
        lam, vec = np.linalg.eigh(np.array([[vc, cv], [cv, vr]]))
        ang = math.atan2(vec[1, 1], vec[0, 1]) % math.pi
        assert abs((ang - t + math.pi / 2) % math.pi - math.pi / 2) < 1e-3, (t, ang)
    # WCS: a quarter turn A (source +x -> image +y) turns the angle-0 galaxy onto the rows,
    # and the source position lands at A u + b
    A = np.array([[0.0, -1.0], [1.0, 0.0]])
    b = (2.0, -1.0)
    p = A @ np.asarray(u) + np.asarray(b)
    h2, w2 = 61, 41
    origin2 = (p[0] - 18.0, p[1] - 31.0)
    G = _gal_image(h2, w2, origin2, u, 0.0, A=A, b=b)
    r, c = np.meshgrid(np.arange(h2), np.arange(w2), indexing="ij")
    mc, mr, vc, vr, cv = spread(G)
    assert (mc, mr) == pytest.approx((18.0, 31.0), abs=1e-3)
    assert vr > 3 * vc
    # a shear A = [[1, 0.5], [0, 1]] moves source +y towards image +x: a galaxy along +y
    # then leans to positive x-y covariance
    A = np.array([[1.0, 0.5], [0.0, 1.0]])
    _, _, vc, vr, cv = spread(_gal_image(h2, w2, (-18.0, -31.0), (0.0, 0.0), math.pi / 2, A=A))
    assert cv > 0.2 * math.sqrt(vc * vr)


# ---------------------------------------------------------------------------- P12 whole model

BRIGHT_DRAW = 40      # sources drawn; the test fits the small-patch ones below
N_FIT = 10


def _fit_one(args):
    sb, s = args
    imgs = model.source_images(sb, s)
    th0 = oinit.plain_init(sb.u_cat[s], imgs, sb.prior)
    r = newton.fit(th0, imgs, sb.prior, sb.profiles)
    _, g, H = model.elbo(r.theta, imgs, sb.prior, sb.profiles)
    return r.theta, r.status, lr.lr_covariance(r.theta, g, H, th0[0:2])


def test_bright_truth_recovery_within_linear_response():
    """P12: bright sources (calibration 100 counts/nMgy) are fitted by the oracle from the
    plain start.  Position, log-brightness and colour means have a truth whichever type the
    fit favours (those of the type with q > 1/2 are compared); the galaxy shape is compared
    for galaxies the fit types as galaxies.  Each such parameter with a small linear-response
    standard deviation (identifiable: below 10% of its box width for u and the shape, below
    half its prior standard deviation for the brightness and colour means) lies within 3
    standard deviations of the truth (e_angle modulo pi) for >= 90% of those entries, and for
    at least two thirds of each parameter group.  (Bright stars are often fitted as tiny thin
    galaxies: the generator bins photons over whole pixels while the model samples pixel
    centres, so a star's image is slightly broader than its PSF; position, flux and colours
    are unaffected.)"""
    sb_all = synth.make_config(1, n_sources=BRIGHT_DRAW, bright=True)
    t = sb_all.truth
    order = np.argsort(t["side"], kind="stable")
    stars = [int(s) for s in order if t["is_star"][s]][: N_FIT // 2 - 1]
    gals = [int(s) for s in order if not t["is_star"][s]][: N_FIT - len(stars)]
    pick = sorted(stars + gals)
    sb = sb_all.subset(pick)
    with mp.get_context("fork").Pool(min(len(pick), os.cpu_count() or 1)) as pool:
        fits = pool.map(_fit_one, [(sb, k) for k in range(len(pick))])
    prior = sb.prior
    box = {0: 6.0, 1: 6.0, 3: 1.0 - 2e-4, 4: 0.98, 5: math.pi, 6: 14.8}
    groups = {}
    with_cov = 0
    for k, (th, status, S) in enumerate(fits):
        assert status == newton.CONVERGED
        if S is None:
            continue                           # a flat direction: no linear-response covariance
        with_cov += 1
        ty = 0 if th[2] > 0.5 else 1
        sd = np.sqrt(np.diag(S))
        entries = [("u", j, sb.truth["u"][k][j], box[j]) for j in (0, 1)]
        entries.append(("r1", 7 + ty, sb.truth["log_flux_r"][k], 5 * math.sqrt(prior["r_var"][ty])))
        c_sd = np.sqrt(np.diag(prior["c_cov"][ty]))
        entries += [("c1", 11 + 4 * ty + j, sb.truth["colours"][k][j], 5 * c_sd[j]) for j in range(4)]
        if ty == 1 and not sb.truth["is_star"][k]:
            entries += [("e_dev", 3, sb.truth["e_dev"][k], box[3]), ("e_axis", 4, sb.truth["e_axis"][k], box[4]),
                        ("e_angle", 5, sb.truth["e_angle"][k], box[5]), ("e_scale", 6, sb.truth["e_scale"][k], box[6])]
        for name, j, truth, width in entries:
            if sd[j] >= 0.1 * width:
                continue                       # not identifiable from these pixels
            d = th[j] - truth
            if name == "e_angle":
                d = (d + math.pi / 2) % math.pi - math.pi / 2
            groups.setdefault(name, []).append(abs(d) / sd[j])
    assert with_cov >= 0.7 * len(pick)
    z = np.concatenate([np.asarray(v) for v in groups.values()])
    assert z.size >= 40
    summary = {k: np.round(v, 2).tolist() for k, v in groups.items()}
    assert np.mean(z <= 3.0) >= 0.9, summary
    for name in ("u", "r1", "c1", "e_angle"):
        v = np.asarray(groups.get(name, []))
        assert v.size >= 3, (name, summary)
        assert np.mean(v <= 3.0) >= 2 / 3, (name, summary)
