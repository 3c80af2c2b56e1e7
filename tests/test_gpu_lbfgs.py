"""The value+gradient pixel kernel and the L-BFGS fit (the earlier Celeste optimiser, section
III-B) on the GPU against the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from synth.generate import perturb_theta
from oracle import init as oinit
from oracle import lbfgs as olbfgs
from oracle import model
from helpers import assert_elbo_close, deriv_err, oracle_eval

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


def _nbr_of(sb, nb, s):
    if nb is None:
        return None
    return {i: (nb[0][sb.img_pix_off[i]:sb.img_pix_off[i] + sb.img_h[i] * sb.img_w[i]].reshape(sb.img_h[i], sb.img_w[i]),
                nb[1][sb.img_pix_off[i]:sb.img_pix_off[i] + sb.img_h[i] * sb.img_w[i]].reshape(sb.img_h[i], sb.img_w[i]))
            for i in range(sb.src_img_off[s], sb.src_img_off[s + 1])}


def test_gradient_kernel_matches_oracle(cb, ctx):
    """celeste_elbo_eval with a gradient and no Hessian runs the value+gradient kernel: ELBO and
    gradient match the oracle (1e-5, 1e-4 with the A23 floor) on config 0 at three points, on a
    ragged config-1 subset with neighbour arrays and small work items, and on config-2 sources;
    and they agree with the value+gradient+Hessian kernel's to the same tolerance."""
    c0 = synth.make_config(0)
    c1 = synth.make_config(1, n_sources=40)
    side = c1.truth["side"]
    c1 = c1.subset(list(np.argsort(side)[:2]) + list(np.argsort(side)[-2:]))
    rng = np.random.default_rng(19)
    nb = (rng.uniform(0, 30, c1.n_pixels).astype(np.float32), rng.uniform(0, 8, c1.n_pixels).astype(np.float32))
    c2 = synth.make_config(2, n_sources=60).subset([5, 31, 59])
    cases = [(c0, c0.theta_truth, None, 4096), (c0, perturb_theta(c0.theta_truth, 1), None, 4096),
             (c1, perturb_theta(c1.theta_truth, 2), nb, 512), (c2, perturb_theta(c2.theta_truth, 3), None, 4096)]
    try:
        for k, (sb, th, n_, chunk) in enumerate(cases):
            ctx.set_option(cb.OPT_CHUNK_PX, chunk)
            b = cb.Batch.from_synth(sb, nbr=n_)
            e, g, _ = ctx.elbo_eval(b, th, want="grad")
            ef, gf, _ = ctx.elbo_eval(b, th)
            for s in range(sb.n_sources):
                v0, g0, _ = oracle_eval(sb, s, th[s], nbr=_nbr_of(sb, n_, s))
                tag = f"case {k} source {s}"
                _say(tag, "elbo rel", abs(e[s] - v0) / abs(v0), "grad err", deriv_err(g[s], g0),
                     "vs full kernel", deriv_err(g[s], gf[s]))
                assert_elbo_close(e[s], v0, what=tag)
                assert deriv_err(g[s], g0) <= 1e-4, tag
                assert deriv_err(g[s], gf[s]) <= 1e-4, tag
                assert abs(e[s] - ef[s]) <= 1e-9 * abs(ef[s]), tag
    finally:
        ctx.set_option(cb.OPT_CHUNK_PX, 4096)
    st = ctx.stats()
    assert st["grad_launches"] >= len(cases) and st["grad_px"] > 0


def test_lbfgs_fit_reaches_the_oracle_optimum(cb, ctx):
    """Config 0 and the two smallest config-1 sources: the GPU L-BFGS fit from the plain start
    converges; its ELBO is the oracle's at its parameters (1e-5) and reaches the oracle L-BFGS
    optimum (A22: within 1e-5 |L*| or above); both take more iterations than the trust-region
    fit."""
    c0 = synth.make_config(0)
    c1 = synth.make_config(1, n_sources=30)
    small = list(np.argsort(c1.truth["side"], kind="stable")[:2])
    for name, sb in (("cfg0", c0), ("cfg1 small", c1.subset(small))):
        b = cb.Batch.from_synth(sb)
        th0 = np.zeros((sb.n_sources, 27))
        th0[:, 0:2] = sb.u_cat
        th, res = ctx.lbfgs_fit(b, th0, cb.default_lbfgs_opts(init_mode=cb.INIT_PLAIN))
        _, rtr = ctx.batch_fit(b, th0, cb.default_opts(init_mode=cb.INIT_PLAIN))
        for s in range(sb.n_sources):
            imgs = model.source_images(sb, s)
            start = oinit.plain_init(sb.u_cat[s], imgs, sb.prior)
            ref = olbfgs.fit(start, imgs, sb.prior, sb.profiles)
            at = model.elbo_value(th[s], imgs, sb.prior, sb.profiles)
            tag = f"{name} source {s}"
            _say(tag, "gpu", res[s]["elbo"], res[s]["iters"], res[s]["status"], "oracle", ref.elbo, ref.iters,
                 ref.status, "tr iters", rtr[s]["iters"])
            assert res[s]["status"] == cb.CONVERGED and ref.status == olbfgs.CONVERGED, tag
            assert_elbo_close(res[s]["elbo"], at, what=tag)
            assert abs(res[s]["elbo"] - ref.elbo) <= 1e-5 * abs(ref.elbo) or res[s]["elbo"] >= ref.elbo, tag
            assert res[s]["iters"] > rtr[s]["iters"], tag
            assert res[s]["n_full_evals"] == res[s]["iters"] + 1, tag


def test_lbfgs_batch_equals_single_and_graph_equals_eager(cb, ctx):
    """Per-source state and fixed-order reductions: a batch of ragged sources gives bitwise the
    results of fitting each alone, and graph replay the results of eager launches."""
    sb = synth.make_config(1, n_sources=6)
    b = cb.Batch.from_synth(sb)
    th0 = np.zeros((6, 27))
    th0[:, 0:2] = sb.u_cat
    opts = cb.default_lbfgs_opts(init_mode=cb.INIT_PLAIN, max_iter=60)
    th, res = ctx.lbfgs_fit(b, th0, opts)
    for s in (0, 3, 5):
        sub = sb.subset([s])
        th1, r1 = ctx.lbfgs_fit(cb.Batch.from_synth(sub), th0[[s]], opts)
        assert np.array_equal(th1[0], th[s]) and r1[0]["elbo"] == res[s]["elbo"] and r1[0]["iters"] == res[s]["iters"]
    try:
        ctx.set_option(cb.OPT_USE_GRAPH, 0)
        th2, r2 = ctx.lbfgs_fit(b, th0, opts)
    finally:
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
    assert np.array_equal(th2, th) and np.array_equal(r2["elbo"], res["elbo"]) and np.array_equal(r2["iters"], res["iters"])


def test_lbfgs_status_paths_and_options(cb, ctx):
    sb = synth.make_config(1, n_sources=3)
    b = cb.Batch.from_synth(sb)
    th0 = np.zeros((3, 27))
    th0[:, 0:2] = sb.u_cat
    _, r = ctx.lbfgs_fit(b, th0, cb.default_lbfgs_opts(max_iter=2))
    assert np.all(r["status"] == cb.MAX_ITER) and np.all(r["iters"] == 2)
    # a tolerance below the FP32 pixel sums' rounding: the line search eventually finds no decrease
    _, r = ctx.lbfgs_fit(b, th0, cb.default_lbfgs_opts(pred_rtol=1e-18, max_iter=3000, max_backtracks=20))
    assert np.all(r["status"] == cb.LINE_SEARCH_FAILED), r["status"]
    for bad in (dict(memory=0), dict(memory=33), dict(max_backtracks=0), dict(armijo_c1=0.6), dict(max_iter=0)):
        with pytest.raises(cb.CelesteError) as ei:
            ctx.lbfgs_fit(b, th0, cb.default_lbfgs_opts(**bad))
        assert ei.value.code == cb.E_INVALID
