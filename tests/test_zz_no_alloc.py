"""celeste_elbo_eval_noalloc (the entry point that allocates nothing) against
celeste_elbo_eval, through the C ABI: bitwise-equal ELBO, gradient and Hessian on two calls
in a row, the second with a smaller batch, and the oracle's tolerance on a few sources."""
import sys

import numpy as np
import pytest

import synth
from synth.generate import perturb_theta
from helpers import assert_derivs_close, assert_elbo_close, oracle_eval

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


def _outputs(S, want):
    import torch
    e = torch.full((S,), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full((S, 27), float("nan"), dtype=torch.float64, device="cuda") if want != "value" else None
    h = torch.full((S, 27, 27), float("nan"), dtype=torch.float64, device="cuda") if want == "hess" else None
    return e, g, h


def _compare(cb, ctx, sb, th, want, oracle_sources=()):
    import torch
    b = cb.Batch.from_synth(sb)
    tht = torch.from_numpy(th).cuda()
    e0, g0, h0 = ctx.elbo_eval(b, tht, want=want)
    e1, g1, h1 = ctx.elbo_eval_noalloc(b, tht, *_outputs(sb.n_sources, want))
    torch.cuda.synchronize()
    assert torch.equal(e0, e1), "ELBO differs from celeste_elbo_eval"
    if want != "value":
        assert torch.equal(g0, g1), "gradient differs from celeste_elbo_eval"
    if want == "hess":
        assert torch.equal(h0, h1), "Hessian differs from celeste_elbo_eval"
    for s in oracle_sources:
        v, g, H = oracle_eval(sb, s, th[s], want="hess" if want == "hess" else "value")
        assert_elbo_close(float(e1[s]), v, what=f"noalloc source {s}")
        if want == "hess":
            assert_derivs_close(g1[s].cpu().numpy(), h1[s].cpu().numpy(), g, H, what=f"noalloc source {s}")


def test_noalloc_equals_elbo_eval_two_calls(cb, ctx):
    # first call: 60 ragged config-1 sources (300 images); second: a smaller batch of 9
    # sources of another draw, so the second call reuses the scratch array the first filled
    big = synth.make_config(1, n_sources=60, device="cuda")
    th_big = perturb_theta(big.theta_truth, 41)
    _say("case: noalloc first call", big.n_sources, "sources", big.n_images, "images")
    _compare(cb, ctx, big, th_big, "hess", oracle_sources=(0, 37))
    small = synth.make_config(2, n_sources=9, device="cuda")
    th_small = perturb_theta(small.theta_truth, 42)
    _say("case: noalloc second call", small.n_sources, "sources", small.n_images, "images")
    _compare(cb, ctx, small, th_small, "hess", oracle_sources=(4,))
    _say("case: noalloc value only and gradient only")
    _compare(cb, ctx, small, th_small, "value")
    _compare(cb, ctx, big, th_big, "grad")


def test_noalloc_rejects_oversize_and_host_batches(cb, ctx):
    import torch
    # 2,400 config-1 sources = 12,000 images: more than the fixed scratch array holds
    sb = synth.make_config(1, n_sources=2400, device="cuda")
    th = torch.from_numpy(sb.theta_truth).cuda()
    _say("case: noalloc oversize", sb.n_images, "images")
    b = cb.Batch.from_synth(sb)
    with pytest.raises(cb.CelesteError) as ei:
        ctx.elbo_eval_noalloc(b, th, *_outputs(sb.n_sources, "hess"))
    assert "scratch" in str(ei.value)
    # the context and the scratch still work after the refusal
    small = synth.make_config(1, n_sources=5, device="cuda")
    _compare(cb, ctx, small, perturb_theta(small.theta_truth, 43), "hess")
    # a host batch needs staging memory: refused
    host = synth.make_config(1, n_sources=3)
    with pytest.raises(cb.CelesteError) as ei:
        ctx.elbo_eval_noalloc(cb.Batch.from_synth(host), torch.from_numpy(host.theta_truth).cuda(),
                              *_outputs(3, "hess"))
    assert "device batches" in str(ei.value)
