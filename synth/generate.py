"""Seeded generator of Celeste-shaped synthetic workloads.

Every array here is an *input*: catalog truth, per-image metadata (band,
patch geometry, WCS offset, sky, calibration, PSF mixture) and Poisson pixel
counts.  The parameter vector layout (27 natural coordinates) is the public
interface order:

    0,1   u (source-frame position, px)        2   a = q(star)
    3     e_dev   4 e_axis   5 e_angle   6 e_scale (half-light radius, px)
    7,8   r1 [star, gal]  mean of log reference-band (r) brightness
    9,10  r2 [star, gal]  variance of the same
    11-14 c1 star colour means   15-18 c1 galaxy colour means
    19-22 c2 star colour vars    23-26 c2 galaxy colour vars

Seeds: config k uses SeedSequence(161103404 + k).spawn(4) for
[truth, psf/sky, noise, init].
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

N_PARAMS = 27
N_BANDS = 5
REF_BAND = 2          # r band; colours are log ratios of adjacent bands
CONFIG_SEED_BASE = 161103404

# Prior parameters (Phi, Upsilon, Xi).  The paper learns them from existing
# catalogs; none are published in it, so these are stated values: P(star)=0.5,
# log r-band brightness ~ N(ln 20, 1) for both types, colours MVN with the
# means below and covariance sigma_j sigma_k 0.3^|j-k|.
_SIG = np.array([0.3, 0.2, 0.15, 0.15])
_CCOV = _SIG[:, None] * _SIG[None, :] * 0.3 ** np.abs(np.subtract.outer(np.arange(4), np.arange(4)))
PRIOR = {
    "p_star": 0.5,
    "r_mean": np.array([math.log(20.0), math.log(20.0)]),
    "r_var": np.array([1.0, 1.0]),
    "c_mean": np.array([[1.2, 0.45, 0.2, 0.1], [1.4, 0.7, 0.35, 0.25]]),
    "c_cov": np.stack([_CCOV, _CCOV]),
}

_PROFILE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "galaxy_profiles.json")


def load_profiles():
    """Galaxy prototype mixtures: dict(exp=(amp, var), dev=(amp, var)), var in r_e^2."""
    with open(_PROFILE_PATH) as f:
        d = json.load(f)
    return {k: (np.array(d[k]["amp"]), np.array(d[k]["var"])) for k in ("exp", "dev")}


@dataclass
class SynthBatch:
    """Structure-of-arrays workload: S sources, each with a CSR range of images."""
    n_sources: int
    src_img_off: np.ndarray          # int64 (S+1)
    img_band: np.ndarray             # int32 (I)
    img_h: np.ndarray                # int32 (I)
    img_w: np.ndarray                # int32 (I)
    img_pitch: np.ndarray            # int32 (I)
    img_origin: np.ndarray           # f64 (I,2) image-frame (x,y) of element (0,0) centre
    img_wcs: np.ndarray              # f64 (I,6) A (row-major 2x2), b : p = A u + b
    img_sky: np.ndarray              # f64 (I)
    img_calib: np.ndarray            # f64 (I) counts per nMgy
    img_psf: np.ndarray              # f64 (I,K,6) weight, mean_x, mean_y, cov_xx, cov_xy, cov_yy
    img_npsf: np.ndarray             # int32 (I)
    img_pix_off: np.ndarray          # int64 (I) offset of element (0,0) in the flat pixel buffer
    pixels: object                   # flat float32 numpy array, or a torch tensor on a device
    u_cat: np.ndarray                # f64 (S,2) catalog position (patch centre), source frame
    truth: dict = field(default_factory=dict)
    theta_truth: np.ndarray = None   # f64 (S,27) a natural-parameter point near the truth
    prior: dict = field(default_factory=lambda: PRIOR)
    profiles: dict = field(default_factory=load_profiles)
    name: str = ""

    @property
    def n_images(self):
        return int(self.img_band.shape[0])

    @property
    def n_pixels(self):
        return int(np.sum(self.img_h.astype(np.int64) * self.img_w))

    def image_pixels(self, i):
        """Host (h, w) float32 view/copy of image i."""
        h, w, p, o = int(self.img_h[i]), int(self.img_w[i]), int(self.img_pitch[i]), int(self.img_pix_off[i])
        px = self.pixels
        if not isinstance(px, np.ndarray):
            px = px[o:o + (h - 1) * p + w].cpu().numpy()
            o = 0
        rows = [px[o + r * p:o + r * p + w] for r in range(h)]
        return np.array(rows, dtype=np.float32)

    def subset(self, idx):
        """A new host batch holding only the sources in idx (pixels copied)."""
        idx = np.asarray(idx, dtype=np.int64)
        imgs = np.concatenate([np.arange(self.src_img_off[s], self.src_img_off[s + 1]) for s in idx])
        counts = np.array([self.src_img_off[s + 1] - self.src_img_off[s] for s in idx])
        pix = [self.image_pixels(i).ravel() for i in imgs]
        sizes = np.array([p.size for p in pix], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        truth = {k: v[idx] for k, v in self.truth.items()}
        return SynthBatch(
            n_sources=len(idx), src_img_off=np.concatenate([[0], np.cumsum(counts)]).astype(np.int64),
            img_band=self.img_band[imgs].copy(), img_h=self.img_h[imgs].copy(), img_w=self.img_w[imgs].copy(),
            img_pitch=self.img_w[imgs].copy(), img_origin=self.img_origin[imgs].copy(),
            img_wcs=self.img_wcs[imgs].copy(), img_sky=self.img_sky[imgs].copy(),
            img_calib=self.img_calib[imgs].copy(), img_psf=self.img_psf[imgs].copy(),
            img_npsf=self.img_npsf[imgs].copy(), img_pix_off=off,
            pixels=np.concatenate(pix).astype(np.float32) if pix else np.zeros(0, np.float32),
            u_cat=self.u_cat[idx].copy(), truth=truth,
            theta_truth=None if self.theta_truth is None else self.theta_truth[idx].copy(),
            prior=self.prior, profiles=self.profiles, name=self.name + "[subset]")


# ----------------------------------------------------------------------------
# sampling helpers
# ----------------------------------------------------------------------------

def _draw_psf(rng, n, sig_lo, sig_hi, k=3):
    """n PSFs of k components: weights ~ Dirichlet(2,..), sigma_x,y ~ U, rho ~ U(-0.2,0.2)."""
    w = rng.dirichlet(np.full(k, 2.0), size=n)
    sx = rng.uniform(sig_lo, sig_hi, size=(n, k))
    sy = rng.uniform(sig_lo, sig_hi, size=(n, k))
    rho = rng.uniform(-0.2, 0.2, size=(n, k))
    psf = np.zeros((n, k, 6))
    psf[:, :, 0] = w
    psf[:, :, 3] = sx * sx
    psf[:, :, 4] = rho * sx * sy
    psf[:, :, 5] = sy * sy
    return psf


def _band_log_flux(log_fr, colours):
    """log brightness in u,g,r,i,z from the r-band value and 4 adjacent-band log ratios."""
    out = np.empty(log_fr.shape + (N_BANDS,))
    out[..., REF_BAND] = log_fr
    for b in range(REF_BAND + 1, N_BANDS):          # walk redwards: l_{b} = l_{b-1} * e^{c_{b-1}}
        out[..., b] = out[..., b - 1] + colours[..., b - 1]
    for b in range(REF_BAND - 1, -1, -1):           # walk bluewards: l_{b} = l_{b+1} / e^{c_b}
        out[..., b] = out[..., b + 1] - colours[..., b]
    return out


def _shoot_photons(rng, img_of, pos, psf, is_star, shape, profiles):
    """Photon positions (image frame), vectorised over all photons of all images.

    img_of : (P,) image index of each photon; pos : (I,2) true source position per image;
    psf : (I,K,6); is_star : (I,) bool; shape : (I,4) e_dev, e_axis, e_angle, e_scale.
    Each photon takes a PSF component (prob. = weight) and a Gaussian offset from it; a
    galaxy photon adds an offset from the dev (prob. e_dev) or exp prototype mixture,
    stretched by the axis ratio, rotated by the angle and scaled by the half-light radius.
    """
    P = img_of.shape[0]
    if P == 0:
        return np.zeros((0, 2))
    w = psf[img_of, :, 0]
    cw = np.cumsum(w / w.sum(axis=1, keepdims=True), axis=1)
    comp = np.minimum((rng.random(P)[:, None] > cw).sum(axis=1), psf.shape[1] - 1)
    pc = psf[img_of, comp]                                    # (P,6)
    l11 = np.sqrt(pc[:, 3])
    l21 = pc[:, 4] / l11
    l22 = np.sqrt(np.maximum(pc[:, 5] - l21 * l21, 0.0))
    z = rng.standard_normal((P, 2))
    off = np.stack([pc[:, 1] + l11 * z[:, 0], pc[:, 2] + l21 * z[:, 0] + l22 * z[:, 1]], axis=1)
    gal = ~is_star[img_of]
    if gal.any():
        gi = np.nonzero(gal)[0]
        sh = shape[img_of[gi]]
        use_dev = rng.random(gi.size) < sh[:, 0]
        sd = np.empty(gi.size)
        for name, sel in (("dev", use_dev), ("exp", ~use_dev)):
            amp, var = profiles[name]
            ca = np.cumsum(amp / amp.sum())
            j = np.minimum(np.searchsorted(ca, rng.random(int(sel.sum()))), len(amp) - 1)
            sd[sel] = np.sqrt(var[j])
        zz = rng.standard_normal((gi.size, 2)) * sd[:, None]
        zz[:, 1] *= sh[:, 1]
        ca, sa = np.cos(sh[:, 2]), np.sin(sh[:, 2])
        off[gi, 0] += sh[:, 3] * (ca * zz[:, 0] - sa * zz[:, 1])
        off[gi, 1] += sh[:, 3] * (sa * zz[:, 0] + ca * zz[:, 1])
    return pos[img_of] + off


def _bin_photons(xy, img_of, origin, h, w, pix_off):
    """Flat pixel index of every photon that lands inside its image (unit pixels)."""
    c = np.floor(xy[:, 0] - origin[img_of, 0] + 0.5).astype(np.int64)
    r = np.floor(xy[:, 1] - origin[img_of, 1] + 0.5).astype(np.int64)
    ok = (c >= 0) & (c < w[img_of]) & (r >= 0) & (r < h[img_of])
    flat = pix_off[img_of[ok]] + r[ok] * w[img_of[ok]] + c[ok]
    idx, cnt = np.unique(flat, return_counts=True)
    return idx, cnt


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

CONFIGS = {
    # name: n_sources, side sampler, epochs sampler, psf sigma range, sky sampler, calib
    0: dict(n=1, side=("fixed", 31), epochs=("fixed", 1), psf=(1.0, 2.5), sky=("fixed", 100.0), calib=1.0,
            types="bern", axis=(0.2, 1.0)),
    1: dict(n=1000, side=("int", 21, 61), epochs=("fixed", 1), psf=(1.0, 2.5), sky=("fixed", 100.0), calib=1.0,
            types="half", axis=(0.2, 1.0)),
    2: dict(n=20000, side=("loguni", 15, 121), epochs=("int", 1, 10), psf=(1.0, 3.0), sky=("uni", 50.0, 300.0),
            calib=1.0, types="bern", axis=(0.2, 1.0)),
    3: dict(n=200000, side=("int", 21, 61), epochs=("fixed", 1), psf=(1.0, 2.5), sky=("fixed", 100.0), calib=1.0,
            types="half", axis=(0.2, 1.0)),
}


def _sample(rng, spec, n):
    kind = spec[0]
    if kind == "fixed":
        return np.full(n, spec[1])
    if kind == "int":
        return rng.integers(spec[1], spec[2] + 1, size=n)
    if kind == "uni":
        return rng.uniform(spec[1], spec[2], size=n)
    if kind == "loguni":
        return np.rint(np.exp(rng.uniform(math.log(spec[1]), math.log(spec[2]), size=n))).astype(np.int64)
    raise ValueError(kind)


def make_config(k, n_sources=None, seed=None, bright=False, device=None, pixel_chunk=1 << 27,
                source_offset=0):
    """Build config k (0..3) with its canonical seed.

    n_sources      : take the first n sources of the config's draw (None = all);
    bright         : calibration 100 counts/nMgy (the "bright" variant of config 1);
    device         : None -> numpy pixels; a torch device -> pixels generated and kept there
                     (sky by torch.poisson with a seeded generator, photons binned on the host);
    source_offset  : shift the seed for held-out draws (config 3 test set uses 1000).
    """
    spec = dict(CONFIGS[k])
    n_all = spec["n"] if n_sources is None else int(n_sources)
    seed = CONFIG_SEED_BASE + k + source_offset if seed is None else seed
    ss = np.random.SeedSequence(seed)
    r_truth, r_psf, r_noise, r_init = [np.random.default_rng(s) for s in ss.spawn(4)]
    profiles = load_profiles()
    calib = 100.0 if bright else spec["calib"]

    S = n_all
    # --- catalog truth -------------------------------------------------------------
    if spec["types"] == "half":
        is_star = np.zeros(S, bool)
        is_star[: S // 2] = True
        r_truth.shuffle(is_star)
    else:
        is_star = r_truth.random(S) < PRIOR["p_star"]
    log_fr = r_truth.normal(PRIOR["r_mean"][0], math.sqrt(PRIOR["r_var"][0]), size=S)
    colours = np.empty((S, 4))
    for t, sel in ((0, is_star), (1, ~is_star)):
        colours[sel] = r_truth.multivariate_normal(PRIOR["c_mean"][t], PRIOR["c_cov"][t], size=int(sel.sum()))
    e_dev = r_truth.uniform(0, 1, S)
    e_axis = r_truth.uniform(spec["axis"][0], spec["axis"][1], S)
    e_angle = r_truth.uniform(0, math.pi, S)
    e_scale = np.exp(r_truth.uniform(math.log(0.5), math.log(3.0), S))
    side = _sample(r_truth, spec["side"], S).astype(np.int64)
    epochs = _sample(r_truth, spec["epochs"], S).astype(np.int64)
    jitter = r_truth.uniform(-0.5, 0.5, size=(S, 2))

    # source frame: each source sits in its own frame; catalog position = integer centre
    half = side // 2
    u_cat = np.stack([half, half], axis=1).astype(np.float64)
    u_true = u_cat + jitter

    n_img_src = N_BANDS * epochs
    src_img_off = np.concatenate([[0], np.cumsum(n_img_src)]).astype(np.int64)
    I = int(src_img_off[-1])
    img_src = np.repeat(np.arange(S), n_img_src)
    local = np.arange(I) - src_img_off[img_src]
    img_band = (local % N_BANDS).astype(np.int32)       # epoch-major: [ugriz]_epoch0, [ugriz]_epoch1 ...
    img_side = side[img_src]
    img_h = img_side.astype(np.int32)
    img_w = img_side.astype(np.int32)
    # WCS: A = I, sub-pixel offset per epoch (single-epoch configs: zero offset)
    img_wcs = np.zeros((I, 6))
    img_wcs[:, 0] = 1.0
    img_wcs[:, 3] = 1.0
    multi = epochs[img_src] > 1
    offs = r_psf.uniform(-0.5, 0.5, size=(I, 2))
    epoch_of = local // N_BANDS
    # one offset per (source, epoch), shared by its 5 bands
    first = src_img_off[img_src] + epoch_of * N_BANDS
    img_wcs[:, 4:6] = np.where(multi[:, None], offs[first], 0.0)
    p_cat = u_cat[img_src] + img_wcs[:, 4:6]
    img_origin = np.rint(p_cat) - half[img_src][:, None]
    img_sky = _sample(r_psf, spec["sky"], I).astype(np.float64)
    # sky and PSF per (source, epoch, band) image
    img_psf = _draw_psf(r_psf, I, *spec["psf"])
    img_npsf = np.full(I, 3, np.int32)
    img_calib = np.full(I, calib)
    npx = img_h.astype(np.int64) * img_w
    img_pix_off = np.concatenate([[0], np.cumsum(npx)[:-1]]).astype(np.int64)
    n_pix = int(npx.sum())

    # --- photons -------------------------------------------------------------------
    log_fb = _band_log_flux(log_fr, colours)            # (S,5)
    lam = calib * np.exp(log_fb[img_src, img_band])
    n_phot = r_noise.poisson(lam)
    img_of = np.repeat(np.arange(I), n_phot)
    pos = u_true[img_src] + img_wcs[:, 4:6]
    shape = np.stack([e_dev, e_axis, e_angle, e_scale], axis=1)[img_src]
    xy = _shoot_photons(r_noise, img_of, pos, img_psf, is_star[img_src], shape, profiles)
    ph_idx, ph_cnt = _bin_photons(xy, img_of, img_origin, img_h.astype(np.int64),
                                  img_w.astype(np.int64), img_pix_off)
    del xy, img_of

    # --- sky + assemble ---------------------------------------------------------------
    if device is None:
        # in chunks of whole images (the draws are taken in pixel order either way)
        pixels = np.empty(n_pix, dtype=np.float32)
        ends = np.cumsum(npx)
        i0 = 0
        while i0 < I:
            a = int(img_pix_off[i0])
            i1 = max(int(np.searchsorted(ends, a + pixel_chunk, side="right")), i0 + 1)
            pixels[a:int(ends[i1 - 1])] = r_noise.poisson(np.repeat(img_sky[i0:i1], npx[i0:i1]))
            i0 = i1
        np.add.at(pixels, ph_idx, ph_cnt.astype(np.float32))
    else:
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        pixels = torch.empty(n_pix, dtype=torch.float32, device=device)
        # chunks of whole images so the per-pixel rate is built a slice at a time
        ends = np.cumsum(npx)
        i0 = 0
        while i0 < I:
            a = int(img_pix_off[i0])
            i1 = int(np.searchsorted(ends, a + pixel_chunk, side="right"))
            i1 = max(i1, i0 + 1)
            b = int(ends[i1 - 1])
            rate = torch.from_numpy(np.repeat(img_sky[i0:i1].astype(np.float32), npx[i0:i1])).to(device)
            pixels[a:b] = torch.poisson(rate, generator=gen)
            del rate
            i0 = i1
        pixels.index_add_(0, torch.from_numpy(ph_idx).to(device),
                          torch.from_numpy(ph_cnt.astype(np.float32)).to(device))

    # --- a natural-parameter point near the truth -----------------------------------
    th = np.zeros((S, N_PARAMS))
    th[:, 0:2] = u_true
    th[:, 2] = np.where(is_star, 0.99, 0.01)
    th[:, 3] = np.clip(e_dev, 0.02, 0.98)
    th[:, 4] = np.clip(e_axis, 0.02, 0.98)
    th[:, 5] = e_angle
    th[:, 6] = e_scale
    th[:, 7] = log_fr
    th[:, 8] = log_fr
    th[:, 9] = 0.05
    th[:, 10] = 0.05
    th[:, 11:15] = colours
    th[:, 15:19] = colours
    th[:, 19:27] = 0.01

    truth = dict(u=u_true, is_star=is_star, log_flux_r=log_fr, colours=colours, e_dev=e_dev,
                 e_axis=e_axis, e_angle=e_angle, e_scale=e_scale, side=side, epochs=epochs)
    return SynthBatch(
        n_sources=S, src_img_off=src_img_off, img_band=img_band, img_h=img_h, img_w=img_w,
        img_pitch=img_w.copy(), img_origin=img_origin, img_wcs=img_wcs, img_sky=img_sky,
        img_calib=img_calib, img_psf=img_psf, img_npsf=img_npsf, img_pix_off=img_pix_off,
        pixels=pixels, u_cat=u_cat, truth=truth, theta_truth=th, profiles=profiles,
        name=f"config{k}" + ("-bright" if bright else ""))


def perturb_theta(theta, seed, scale=1.0):
    """A random natural-parameter point around theta (for derivative tests); stays in-domain."""
    rng = np.random.default_rng(seed)
    t = np.array(theta, dtype=np.float64, copy=True)
    S = t.shape[0]
    t[:, 0:2] += rng.normal(0, 0.3 * scale, (S, 2))
    t[:, 2] = rng.uniform(0.2, 0.8, S)
    t[:, 3] = rng.uniform(0.2, 0.8, S)
    t[:, 4] = rng.uniform(0.3, 0.9, S)
    t[:, 5] = rng.uniform(0, math.pi, S)
    t[:, 6] = np.exp(rng.uniform(math.log(0.6), math.log(2.5), S))
    t[:, 7:9] += rng.normal(0, 0.3 * scale, (S, 2))
    t[:, 9:11] = rng.uniform(0.02, 0.5, (S, 2))
    t[:, 11:19] += rng.normal(0, 0.2 * scale, (S, 8))
    t[:, 19:27] = rng.uniform(0.01, 0.2, (S, 8))
    return t


# ----------------------------------------------------------------------------
# crowded field
# ----------------------------------------------------------------------------

@dataclass
class SynthField:
    """A multi-source field: n_fields images of size H x W and a SynthBatch whose patches are
    views into them (pitch = W); img_field[i] gives the field of patch image i."""
    batch: SynthBatch
    fields: object                 # (n_fields * H * W) float32, numpy or torch on a device
    n_fields: int
    H: int
    W: int
    img_field: np.ndarray          # int32 (I)
    field_band: np.ndarray         # int32 (n_fields)
    field_wcs: np.ndarray          # f64 (n_fields, 6)
    field_sky: np.ndarray
    field_psf: np.ndarray


def make_field(n_sources=100000, size=2048, epochs=4, seed=None, device=None, k=4):
    """Crowded-field workload: sources at Poisson positions with intensity proportional to
    1 + x/size across the field, patch sides log-uniform in 15..121 clipped to the field,
    5 bands x `epochs` field images each with its own PSF (widths 1..3 px), sky (50..300)
    and sub-pixel offset; catalog position = nearest pixel centre of the truth."""
    seed = CONFIG_SEED_BASE + k if seed is None else seed
    ss = np.random.SeedSequence(seed)
    r_truth, r_psf, r_noise, r_init = [np.random.default_rng(s) for s in ss.spawn(4)]
    profiles = load_profiles()
    S, H, W = int(n_sources), int(size), int(size)
    # x from the density 1 + x/W on [0, W): inverse CDF of (x + x^2/(2W)) / (1.5 W)
    uu = r_truth.random(S)
    x = -W + np.sqrt(W * W + 2.0 * W * 1.5 * W * uu)
    y = r_truth.uniform(0, H, S)
    u_true = np.stack([x - 0.5, y - 0.5], axis=1)          # pixel centres at integers 0..W-1
    is_star = r_truth.random(S) < PRIOR["p_star"]
    log_fr = r_truth.normal(PRIOR["r_mean"][0], math.sqrt(PRIOR["r_var"][0]), size=S)
    colours = np.empty((S, 4))
    for t, sel in ((0, is_star), (1, ~is_star)):
        colours[sel] = r_truth.multivariate_normal(PRIOR["c_mean"][t], PRIOR["c_cov"][t], size=int(sel.sum()))
    e_dev = r_truth.uniform(0, 1, S)
    e_axis = r_truth.uniform(0.2, 1.0, S)
    e_angle = r_truth.uniform(0, math.pi, S)
    e_scale = np.exp(r_truth.uniform(math.log(0.5), math.log(3.0), S))
    side = np.rint(np.exp(r_truth.uniform(math.log(15), math.log(121), S))).astype(np.int64)
    u_cat = np.clip(np.rint(u_true), 0, [W - 1, H - 1]).astype(np.float64)
    # field images: band-major within epoch
    NF = N_BANDS * epochs
    field_band = np.tile(np.arange(N_BANDS), epochs).astype(np.int32)
    field_psf = _draw_psf(r_psf, NF, 1.0, 3.0)
    field_sky = r_psf.uniform(50.0, 300.0, NF)
    field_wcs = np.zeros((NF, 6))
    field_wcs[:, 0] = field_wcs[:, 3] = 1.0
    eoff = r_psf.uniform(-0.5, 0.5, size=(epochs, 2))
    field_wcs[:, 4:6] = np.repeat(eoff, N_BANDS, axis=0)
    # patches: one per (source, field), centred on the catalog position in that field, clipped
    I = S * NF
    img_src = np.repeat(np.arange(S), NF)
    img_field = np.tile(np.arange(NF), S).astype(np.int32)
    half = side // 2
    pc = u_cat[img_src] + field_wcs[img_field, 4:6]
    cx, cy = np.rint(pc[:, 0]).astype(np.int64), np.rint(pc[:, 1]).astype(np.int64)
    x0 = np.clip(cx - half[img_src], 0, W - 1)
    y0 = np.clip(cy - half[img_src], 0, H - 1)
    x1 = np.clip(cx - half[img_src] + side[img_src], 1, W)
    y1 = np.clip(cy - half[img_src] + side[img_src], 1, H)
    img_w = (x1 - x0).astype(np.int32)
    img_h = (y1 - y0).astype(np.int32)
    img_origin = np.stack([x0, y0], axis=1).astype(np.float64)
    img_pix_off = (img_field.astype(np.int64) * H * W + y0 * W + x0).astype(np.int64)
    # pixels: Poisson sky + photons of every source in every field image
    lam = np.exp(_band_log_flux(log_fr, colours))[:, field_band]          # (S, NF) nMgy
    n_phot = r_noise.poisson(lam.ravel())
    img_of = np.repeat(np.arange(I), n_phot)
    pos = u_true[img_src] + field_wcs[img_field, 4:6]
    shape = np.stack([e_dev, e_axis, e_angle, e_scale], axis=1)[img_src]
    xy = _shoot_photons(r_noise, img_of, pos, field_psf[img_field], is_star[img_src], shape, profiles)
    fx = np.floor(xy[:, 0] + 0.5).astype(np.int64)
    fy = np.floor(xy[:, 1] + 0.5).astype(np.int64)
    ok = (fx >= 0) & (fx < W) & (fy >= 0) & (fy < H)
    flat = img_field[img_of[ok]].astype(np.int64) * H * W + fy[ok] * W + fx[ok]
    ph_idx, ph_cnt = np.unique(flat, return_counts=True)
    del xy, img_of, flat
    if device is None:
        fields = r_noise.poisson(np.repeat(field_sky, H * W)).astype(np.float32)
        np.add.at(fields, ph_idx, ph_cnt.astype(np.float32))
    else:
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        fields = torch.empty(NF * H * W, dtype=torch.float32, device=device)
        for f in range(NF):
            rate = torch.full((H * W,), float(field_sky[f]), dtype=torch.float32, device=device)
            fields[f * H * W:(f + 1) * H * W] = torch.poisson(rate, generator=gen)
        fields.index_add_(0, torch.from_numpy(ph_idx).to(device), torch.from_numpy(ph_cnt.astype(np.float32)).to(device))
    th = np.zeros((S, N_PARAMS))
    th[:, 0:2] = u_true
    th[:, 2] = np.where(is_star, 0.99, 0.01)
    th[:, 3] = np.clip(e_dev, 0.02, 0.98)
    th[:, 4] = np.clip(e_axis, 0.02, 0.98)
    th[:, 5] = e_angle
    th[:, 6] = e_scale
    th[:, 7] = th[:, 8] = log_fr
    th[:, 9] = th[:, 10] = 0.05
    th[:, 11:15] = th[:, 15:19] = colours
    th[:, 19:27] = 0.01
    sb = SynthBatch(
        n_sources=S, src_img_off=np.arange(0, I + 1, NF, dtype=np.int64), img_band=field_band[img_field].copy(),
        img_h=img_h, img_w=img_w, img_pitch=np.full(I, W, np.int32), img_origin=img_origin,
        img_wcs=field_wcs[img_field].copy(), img_sky=field_sky[img_field].copy(), img_calib=np.ones(I),
        img_psf=field_psf[img_field].copy(), img_npsf=np.full(I, 3, np.int32), img_pix_off=img_pix_off,
        pixels=fields, u_cat=u_cat,
        truth=dict(u=u_true, is_star=is_star, log_flux_r=log_fr, colours=colours, e_dev=e_dev, e_axis=e_axis,
                   e_angle=e_angle, e_scale=e_scale, side=side, epochs=np.full(S, epochs)),
        theta_truth=th, profiles=profiles, name=f"field{size}x{size}x{NF}")
    return SynthField(batch=sb, fields=fields, n_fields=NF, H=H, W=W, img_field=img_field, field_band=field_band,
                      field_wcs=field_wcs, field_sky=field_sky, field_psf=field_psf)
