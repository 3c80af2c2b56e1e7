"""The trained surrogate start: labels certified against oracle fits, and the gain over the
plain start on held-out sources at the same ELBO tolerance."""
import multiprocessing as mp
import sys

import numpy as np
import pytest

import synth
from synth.surrogate import epoch_orders, init_params
from oracle import init as oinit
from oracle import model, newton
from helpers import ELBO_RTOL

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_fit(args):
    sb, s = args
    imgs = model.source_images(sb, s)
    r = newton.fit(oinit.plain_init(sb.u_cat[s], imgs, sb.prior), imgs, sb.prior, sb.profiles)
    return r.elbo


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1611_03404_amd import celeste as cb
    from paper_1611_03404_amd import surrogate
    ctx = cb.Context(0)
    tr = synth.make_config(3, n_sources=20000, device="cuda")
    b = cb.Batch.from_synth(tr)
    th_lab, res_lab = surrogate.fit_labels(ctx, b, tr.u_cat)
    net, info = surrogate.train(ctx, b, tr.u_cat, init_params(7), lambda n, e: epoch_orders(n, e, 8), epochs=8,
                                minibatch=256, lr=1e-3, log=_say)
    yield cb, ctx, net, tr, th_lab, res_lab, info
    net.close()
    ctx.close()


def test_labels_certified_by_oracle_fits(trained):
    cb, ctx, net, tr, th_lab, res_lab, info = trained
    rng = np.random.default_rng(3)
    pick = [int(s) for s in rng.choice(tr.n_sources, size=8, replace=False)]
    sub = tr.subset(pick)
    with mp.get_context("fork").Pool(8) as pool:
        ref = pool.map(_oracle_fit, [(sub, k) for k in range(len(pick))])
    for k, s in enumerate(pick):
        v = model.elbo_value(th_lab[s], model.source_images(sub, k), sub.prior, sub.profiles)
        _say("label", s, "status", res_lab["status"][s], "gpu label elbo", v, "oracle fit", ref[k])
        assert v >= ref[k] - ELBO_RTOL * abs(ref[k])


def test_surrogate_gain_on_held_out_sources(trained):
    cb, ctx, net, tr, th_lab, res_lab, info = trained
    assert info["epoch_loss"][-1] < 0.7 * info["epoch_loss"][0]
    te = synth.make_config(3, n_sources=1000, source_offset=1000)
    b = cb.Batch.from_synth(te)
    th0 = np.zeros((te.n_sources, 27))
    th0[:, 0:2] = te.u_cat
    ctx.set_surrogate(net)
    try:
        th_s, r_s = ctx.batch_fit(b, th0, cb.default_opts(init_mode=cb.INIT_SURROGATE))
    finally:
        ctx.set_surrogate(None)
    th_p, r_p = ctx.batch_fit(b, th0, cb.default_opts(init_mode=cb.INIT_PLAIN))
    best = np.maximum(r_s["elbo"], r_p["elbo"])
    ok_s = (r_s["status"] == cb.CONVERGED) & (r_s["elbo"] >= best - ELBO_RTOL * np.abs(best))
    ok_p = (r_p["status"] == cb.CONVERGED) & (r_p["elbo"] >= best - ELBO_RTOL * np.abs(best))
    fb = np.mean((r_s["flags"] & cb.FLAG_FALLBACK_USED) != 0)
    _say("iterations surrogate", np.mean(r_s["iters"]), "plain", np.mean(r_p["iters"]), "fallback", fb,
         "at tolerance surrogate", ok_s.mean(), "plain", ok_p.mean())
    assert np.mean(r_s["iters"]) < 0.9 * np.mean(r_p["iters"])
    assert np.mean(r_s["n_full_evals"]) < np.mean(r_p["n_full_evals"])
    assert ok_s.mean() >= 0.95
    assert fb < 0.5
    # the surrogate-started ELBO values agree with the oracle at the returned parameters (sample)
    for s in (0, 17, 400):
        v = model.elbo_value(th_s[s], model.source_images(te, s), te.prior, te.profiles)
        assert abs(v - r_s["elbo"][s]) <= ELBO_RTOL * abs(v)
