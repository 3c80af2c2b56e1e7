"""Pins of the oracle's pixel-subsampled ELBO estimator (the closing section's doubly
stochastic direction): all-ones weights give the ELBO, all-zero weights the theta-free part,
and the exact expectation over every mask of a small image equals the ELBO, gradient and
Hessian (unbiasedness)."""
import itertools

import numpy as np
import pytest

import synth
from synth.generate import perturb_theta
from oracle import model
from synth.subsample import block_masks


def _weights(img, keep_blocks, p):
    w = np.repeat(np.asarray(keep_blocks, np.float64) / p, 8)[: img["h"]]
    return np.repeat(w[:, None], img["w"], axis=1)


def _one_image_case():
    sb = synth.make_config(0)
    th = perturb_theta(sb.theta_truth, 5)[0]
    img = dict(model.source_images(sb, 0)[0])
    img["nbr_mean"] = np.full((img["h"], img["w"]), 7.0)
    img["nbr_var"] = np.full((img["h"], img["w"]), 3.0)
    return sb, th, img


def test_all_ones_and_all_zeros():
    sb, th, img = _one_image_case()
    full = model.elbo(th, [img], sb.prior, sb.profiles)
    nb = (img["h"] + 7) // 8
    ones = dict(img, weights=_weights(img, np.ones(nb), 1.0))
    got = model.elbo(th, [ones], sb.prior, sb.profiles)
    for a, b in zip(got, full):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.max(np.abs(b)))
    zeros = dict(img, weights=np.zeros((img["h"], img["w"])))
    v, g, H = model.elbo(th, [zeros], sb.prior, sb.profiles)
    kv, kg, kH = model.kl_terms(th, sb.prior)
    x = np.asarray(img["pixels"], np.float64)
    c = model.pixel_value(x, img["sky"] + img["nbr_mean"], np.zeros_like(x)).sum()
    assert np.isclose(v, c + kv, rtol=1e-13)
    assert np.allclose(g, kg) and np.allclose(H, kH)


def test_exact_expectation_over_all_masks():
    sb, th, img = _one_image_case()
    nb = (img["h"] + 7) // 8          # 31 rows: 4 blocks
    full = model.elbo(th, [img], sb.prior, sb.profiles)
    for p in (0.5, 0.3):
        ev, eg, eH = 0.0, 0.0, 0.0
        for keep in itertools.product((0, 1), repeat=nb):
            prob = np.prod([p if k else 1.0 - p for k in keep])
            v, g, H = model.elbo(th, [dict(img, weights=_weights(img, keep, p))], sb.prior, sb.profiles)
            ev, eg, eH = ev + prob * v, eg + prob * g, eH + prob * H
        assert np.isclose(ev, full[0], rtol=1e-12)
        assert np.allclose(eg, full[1], rtol=1e-9, atol=1e-9 * np.max(np.abs(full[1])))
        assert np.allclose(eH, full[2], rtol=1e-9, atol=1e-9 * np.max(np.abs(full[2])))


def test_block_masks_shape_and_rate():
    keep, off = synth.subsample.block_masks([31, 8, 9, 121], 0.25, seed=3)
    assert list(off) == [0, 4, 5, 7, 23]
    assert keep.dtype == np.uint8 and keep.size == 23
    k2, _ = synth.subsample.block_masks(np.full(4000, 64), 0.25, seed=4)
    assert abs(k2.mean() - 0.25) < 0.01


def test_fit_with_subsampled_early_phase():
    """Trust-region fit whose early phase fits the subsampled estimate: with every block kept the
    estimate is the ELBO, and the two-phase fit ends at the plain fit's optimum; with p = 0.25 it
    spends its first iterations on the estimate, switches, and still reaches the plain fit's
    optimum (A22: within 1e-5 |L*| or above) from the same start."""
    from oracle import init as oinit
    from oracle import newton
    sb = synth.make_config(0)
    imgs = model.source_images(sb, 0)
    th0 = oinit.plain_init(sb.u_cat[0], imgs, sb.prior)
    ref = newton.fit(th0, imgs, sb.prior, sb.profiles)
    for p, seed in ((1.0, 0), (0.25, 3)):
        keep, off = block_masks(sb.img_h, p, seed)
        simgs = []
        for j, img in enumerate(imgs):
            w = np.repeat(keep[off[j]:off[j + 1]].astype(np.float64) / p, 8)[: img["h"]]
            simgs.append(dict(img, weights=np.repeat(w[:, None], img["w"], axis=1)))
        r = newton.fit_sampled(th0, imgs, simgs, sb.prior, sb.profiles, switch_rtol=1e-5, record=True)
        assert r.status == newton.CONVERGED
        assert abs(r.elbo - ref.elbo) <= 1e-5 * abs(ref.elbo) or r.elbo >= ref.elbo
        assert r.sampled_iters >= 1 and r.iters > r.sampled_iters
        phases = [h["sampled"] for h in r.history]
        assert phases == sorted(phases, reverse=True)           # the estimate first, then the ELBO
        if p == 1.0:
            # the estimate equals the ELBO: the first phase is the plain fit's first iterations
            for a, b in zip(r.history, ref.history):
                if not a["sampled"]:
                    break
                assert a["elbo"] == pytest.approx(b["elbo"], rel=1e-12)
