"""Pins of the oracle's pixel-subsampled ELBO estimator (the closing section's doubly
stochastic direction): all-ones weights give the ELBO, all-zero weights the theta-free part,
and the exact expectation over every mask of a small image equals the ELBO, gradient and
Hessian (unbiasedness)."""
import itertools

import numpy as np

import synth
from synth.generate import perturb_theta
from oracle import model


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
