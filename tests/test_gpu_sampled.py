"""GPU parity of the pixel-subsampled ELBO estimator (celeste_elbo_eval_sampled) against the
FP64 oracle with the same block masks as pixel weights, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from synth.generate import perturb_theta
from synth.subsample import block_masks
from oracle import model
from helpers import assert_derivs_close, assert_elbo_close, deriv_err

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1611_03404_amd import celeste as cb_
    cb_.load()
    return cb_


@pytest.fixture(scope="module")
def ctx(cb):
    c = cb.Context(0)
    yield c
    c.close()


def _oracle_sampled(sb, s, theta, keep, off, p, want="hess"):
    """The oracle's estimate for source s: each of its images weighted block by block."""
    imgs = []
    for j, img in enumerate(model.source_images(sb, s)):
        i = sb.src_img_off[s] + j
        kb = keep[off[i]:off[i + 1]].astype(np.float64) / p
        w = np.repeat(kb, 8)[: img["h"]]
        imgs.append(dict(img, weights=np.repeat(w[:, None], img["w"], axis=1)))
    if want == "hess":
        return model.elbo(theta, imgs, sb.prior, sb.profiles)
    return model.elbo_value(theta, imgs, sb.prior, sb.profiles), None, None


def _check(cb, ctx, sb, th, p, seed, what, want="hess"):
    keep, off = block_masks(sb.img_h, p, seed)
    b = cb.Batch.from_synth(sb)
    el, g, H = ctx.elbo_eval_sampled(b, th, keep, off, p, want=want)
    for s in range(sb.n_sources):
        v0, g0, H0 = _oracle_sampled(sb, s, th[s], keep, off, p, want=want)
        tag = f"{what} p={p} seed={seed} source {s}"
        if want == "hess":
            _say(tag, "elbo", el[s], v0, "gerr", deriv_err(g[s], g0), "herr", deriv_err(H[s], H0))
            assert_derivs_close(g[s], H[s], g0, H0, what=tag)
        else:
            _say(tag, "elbo", el[s], v0)
        assert_elbo_close(el[s], v0, what=tag)


def test_all_blocks_kept_equals_full_eval(cb, ctx):
    """An all-ones mask with keep_prob 1 runs the same sums as celeste_elbo_eval: bitwise equal."""
    sb = synth.make_config(1, n_sources=5)
    th = perturb_theta(sb.theta_truth, 21)
    b = cb.Batch.from_synth(sb)
    keep, off = block_masks(sb.img_h, 1.0, 0)
    assert keep.all()
    e0, g0, H0 = ctx.elbo_eval(b, th)
    e1, g1, H1 = ctx.elbo_eval_sampled(b, th, keep, off, 1.0)
    assert np.array_equal(e0, e1) and np.array_equal(g0, g1) and np.array_equal(H0, H1)
    v0, _, _ = ctx.elbo_eval(b, th, want="value")
    v1, _, _ = ctx.elbo_eval_sampled(b, th, keep, off, 1.0, want="value")
    assert np.array_equal(v0, v1)


@pytest.mark.parametrize("p,seed", [(0.5, 1), (0.3, 2), (0.1, 3)])
def test_config0_oracle_parity(cb, ctx, p, seed):
    sb = synth.make_config(0)
    _say("case: config0 sampled", p, seed)
    _check(cb, ctx, sb, perturb_theta(sb.theta_truth, 22), p, seed, "cfg0")


def test_no_block_kept(cb, ctx):
    """Nothing kept: no pixel work at all, the estimate is the theta-free part plus the prior
    terms (zero pixel gradient and Hessian)."""
    sb = synth.make_config(0)
    th = perturb_theta(sb.theta_truth, 25)
    keep, off = block_masks(sb.img_h, 0.5, 4)
    keep[:] = 0
    b = cb.Batch.from_synth(sb)
    for want in ("hess", "value"):
        el, g, H = ctx.elbo_eval_sampled(b, th, keep, off, 0.5, want=want)
        for s in range(sb.n_sources):
            v0, g0, H0 = _oracle_sampled(sb, s, th[s], keep, off, 0.5, want=want)
            assert_elbo_close(el[s], v0, what=f"none kept {want} source {s}")
            if want == "hess":
                assert_derivs_close(g[s], H[s], g0, H0, what=f"none kept source {s}")


def test_ragged_sides_tiles_and_value_kernel(cb, ctx):
    """Patches of the smallest and largest sides (ragged last blocks), every tile width of the
    derivative kernel and of the value kernel, and small work items (many bands per image)."""
    full = synth.make_config(1)
    side = full.truth["side"]
    idx = list(np.argsort(side)[:2]) + list(np.argsort(side)[-2:])
    sb = full.subset(idx)
    th = perturb_theta(sb.theta_truth, 23)
    _say("case: ragged sides", side[idx])
    try:
        ctx.set_option(cb.OPT_CHUNK_PX, 512)
        for tw in (8, 16, 32, 64):
            ctx.set_option(cb.OPT_TILE_W, tw)
            ctx.set_option(cb.OPT_VALUE_TILE_W, tw)
            _check(cb, ctx, sb, th, 0.4, 30 + tw, f"tile {tw}")
            _check(cb, ctx, sb, th, 0.4, 30 + tw, f"value tile {tw}", want="value")
    finally:
        for opt, v in ((cb.OPT_CHUNK_PX, 4096), (cb.OPT_TILE_W, 8), (cb.OPT_VALUE_TILE_W, 8)):
            ctx.set_option(opt, v)


def test_antithetic_pair_averages_to_full(cb, ctx):
    """At keep_prob 1/2 a mask and its complement weigh every block 2 and 0 in turn, so the
    mean of the two estimates is the full ELBO, gradient and Hessian (unbiasedness, exactly)."""
    sb = synth.make_config(1, n_sources=6)
    th = perturb_theta(sb.theta_truth, 24)
    b = cb.Batch.from_synth(sb)
    keep, off = block_masks(sb.img_h, 0.5, 7)
    ea, ga, Ha = ctx.elbo_eval_sampled(b, th, keep, off, 0.5)
    eb, gb, Hb = ctx.elbo_eval_sampled(b, th, (1 - keep).astype(np.uint8), off, 0.5)
    e0, g0, H0 = ctx.elbo_eval(b, th)
    for s in range(sb.n_sources):
        tag = f"antithetic source {s}"
        assert_elbo_close(0.5 * (ea[s] + eb[s]), e0[s], what=tag)
        assert_derivs_close(0.5 * (ga[s] + gb[s]), 0.5 * (Ha[s] + Hb[s]), g0[s], H0[s], what=tag)


def test_full_size_config2_sampled_sources(cb, ctx):
    """Config 2 at its full size on device memory, a quarter of the blocks kept; the oracle
    checks a sample of sources one by one with the same masks."""
    import torch
    sb = synth.make_config(2, device="cuda")
    p = 0.25
    keep, off = block_masks(sb.img_h, p, 41)
    _say("case: config2 full size sampled", sb.n_sources, "sources", int(keep.sum()), "of", keep.size, "blocks")
    th = perturb_theta(sb.theta_truth, 12, scale=0.5)
    b = cb.Batch.from_synth(sb)
    el, g, H = ctx.elbo_eval_sampled(b, torch.from_numpy(th).cuda(), keep, off, p)
    el, g, H = el.cpu().numpy(), g.cpu().numpy(), H.cpu().numpy()
    assert np.all(np.isfinite(el)) and np.all(np.isfinite(H))
    npx = np.array([np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64) ** 2)
                    for s in range(sb.n_sources)])
    rng = np.random.default_rng(43)
    pick = [int(np.argmin(npx)), int(rng.integers(sb.n_sources)), int(np.argsort(npx)[len(npx) // 2])]
    sub = sb.subset(pick)
    sub_off = np.concatenate([[0], np.cumsum((sub.img_h + 7) // 8)]).astype(np.int64)
    sub_keep = np.concatenate([keep[off[i]:off[i + 1]] for s in pick
                               for i in range(sb.src_img_off[s], sb.src_img_off[s + 1])])
    for k, s in enumerate(pick):
        v0, g0, H0 = _oracle_sampled(sub, k, th[s], sub_keep, sub_off, p)
        tag = f"cfg2 full sampled source {s} ({npx[s]} px)"
        _say(tag, el[s], v0, deriv_err(g[s], g0), deriv_err(H[s], H0))
        assert_elbo_close(el[s], v0, what=tag)
        assert_derivs_close(g[s], H[s], g0, H0, what=tag)


@pytest.mark.parametrize("bad", ["prob_zero", "prob_above_one", "first_offset", "block_count", "null_keep"])
def test_invalid_masks_rejected(cb, ctx, bad):
    sb = synth.make_config(0).subset([0])
    th = sb.theta_truth.copy()
    b = cb.Batch.from_synth(sb)
    keep, off = block_masks(sb.img_h, 0.5, 3)
    p = 0.5
    if bad == "prob_zero":
        p = 0.0
    elif bad == "prob_above_one":
        p = 1.5
    elif bad == "first_offset":
        off = off + 1
        keep = np.concatenate([[1], keep]).astype(np.uint8)
    elif bad == "block_count":
        off = off.copy()
        off[1] += 1           # image 0 one block too many, image 1 one too few
    if bad == "null_keep":
        el = np.zeros(1)
        rc = cb.load().celeste_elbo_eval_sampled(ctx._h, cb.ctypes.byref(b.c), th.ctypes.data, None,
                                                 off.ctypes.data, 0.5, el.ctypes.data, None, None, None)
        assert rc == cb.E_INVALID
        return
    with pytest.raises(cb.CelesteError) as ei:
        ctx.elbo_eval_sampled(b, th, keep, off, p)
    assert ei.value.code == cb.E_INVALID


def test_fit_with_subsampled_early_phase(cb, ctx):
    """celeste_batch_fit_sampled: trust-region fits that start on the subsampled estimate
    (p = 0.25) and switch to the full ELBO.  Config 0 reaches the optimum of the oracle's
    two-phase fit with the same mask (A22: within 1e-5 |L*| or above) and reports the oracle's
    ELBO at its parameters; on a ragged config-1 subset every source converges, the two smallest
    reach the oracle's two-phase optimum and most the plain batched fit's;
    graph replay gives the eager results bit for bit; bad arguments are refused.""" 
    from oracle import init as oinit
    from oracle import newton
    c0 = synth.make_config(0)
    keep, off = block_masks(c0.img_h, 0.25, 3)
    b = cb.Batch.from_synth(c0)
    th0 = np.zeros((1, 27))
    th0[:, 0:2] = c0.u_cat
    th, res = ctx.batch_fit_sampled(b, th0, keep, off, 0.25, switch_rtol=1e-5,
                                    opts=cb.default_opts(init_mode=cb.INIT_PLAIN))
    imgs = model.source_images(c0, 0)
    simgs = []
    for j, img in enumerate(imgs):
        w = np.repeat(keep[off[j]:off[j + 1]].astype(np.float64) / 0.25, 8)[: img["h"]]
        simgs.append(dict(img, weights=np.repeat(w[:, None], img["w"], axis=1)))
    ref = newton.fit_sampled(oinit.plain_init(c0.u_cat[0], imgs, c0.prior), imgs, simgs, c0.prior, c0.profiles,
                             switch_rtol=1e-5)
    _say("cfg0 two-phase: gpu", res[0]["elbo"], res[0]["iters"], res[0]["status"], "oracle", ref.elbo, ref.iters,
         ref.sampled_iters)
    assert res[0]["status"] == cb.CONVERGED and ref.status == newton.CONVERGED
    assert abs(res[0]["elbo"] - ref.elbo) <= 1e-5 * abs(ref.elbo) or res[0]["elbo"] >= ref.elbo
    assert_elbo_close(res[0]["elbo"], model.elbo_value(th[0], imgs, c0.prior, c0.profiles), what="cfg0 two-phase")

    full = synth.make_config(1, n_sources=40)
    side = full.truth["side"]
    small = list(np.argsort(side, kind="stable")[:2])
    sb = full.subset(small + list(np.argsort(side)[-4:]) + [3, 17, 29])
    keep, off = block_masks(sb.img_h, 0.25, 5)
    b = cb.Batch.from_synth(sb)
    th0 = np.zeros((sb.n_sources, 27))
    th0[:, 0:2] = sb.u_cat
    opts = cb.default_opts(init_mode=cb.INIT_PLAIN)
    _, plain = ctx.batch_fit(b, th0, opts)
    th_s, samp = ctx.batch_fit_sampled(b, th0, keep, off, 0.25, switch_rtol=1e-5, opts=opts)
    at_plain = 0
    for s in range(sb.n_sources):
        _say("source", s, "plain", plain[s]["elbo"], plain[s]["iters"], "two-phase", samp[s]["elbo"], samp[s]["iters"])
        assert samp[s]["status"] == cb.CONVERGED
        L = plain[s]["elbo"]
        at_plain += abs(samp[s]["elbo"] - L) <= 1e-5 * abs(L) or samp[s]["elbo"] >= L
    # the early phase can lead a source to another of its local optima (star/galaxy modes, flat
    # shape directions): most sources end at the plain fit's optimum, and the oracle's two-phase
    # fit with the same mask pins the small ones
    assert at_plain >= 0.7 * sb.n_sources, at_plain
    for s in range(2):
        imgs = model.source_images(sb, s)
        simgs = []
        for j, img in enumerate(imgs):
            i = int(sb.src_img_off[s]) + j
            w = np.repeat(keep[off[i]:off[i + 1]].astype(np.float64) / 0.25, 8)[: img["h"]]
            simgs.append(dict(img, weights=np.repeat(w[:, None], img["w"], axis=1)))
        ref = newton.fit_sampled(oinit.plain_init(sb.u_cat[s], imgs, sb.prior), imgs, simgs, sb.prior, sb.profiles,
                                 switch_rtol=1e-5)
        _say("source", s, "oracle two-phase", ref.elbo, ref.iters, ref.sampled_iters)
        assert abs(samp[s]["elbo"] - ref.elbo) <= 1e-5 * abs(ref.elbo) or samp[s]["elbo"] >= ref.elbo, s
        assert_elbo_close(samp[s]["elbo"], model.elbo_value(th_s[s], imgs, sb.prior, sb.profiles), what=f"src {s}")
    try:
        ctx.set_option(cb.OPT_USE_GRAPH, 0)
        th_e, eager = ctx.batch_fit_sampled(b, th0, keep, off, 0.25, switch_rtol=1e-5, opts=opts)
    finally:
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
    assert np.array_equal(th_e, th_s) and np.array_equal(eager["elbo"], samp["elbo"])
    assert np.array_equal(eager["iters"], samp["iters"])
    for kw in (dict(keep_prob=0.0), dict(switch_rtol=0.0)):
        args = dict(keep_prob=0.25, switch_rtol=1e-5)
        args.update(kw)
        with pytest.raises(cb.CelesteError) as ei:
            ctx.batch_fit_sampled(b, th0, keep, off, args["keep_prob"], switch_rtol=args["switch_rtol"], opts=opts)
        assert ei.value.code == cb.E_INVALID
    bad = off.copy()
    bad[1:] += 1
    with pytest.raises(cb.CelesteError):
        ctx.batch_fit_sampled(b, th0, np.concatenate([keep, np.zeros(sb.n_images, np.uint8)])[: bad[-1]], bad, 0.25,
                              opts=opts)
