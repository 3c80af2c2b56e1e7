"""GPU trust-region fits (celeste_newton_fit / celeste_batch_fit) against oracle fits."""
import multiprocessing as mp
import sys

import numpy as np
import pytest

import synth
from oracle import init as oinit
from oracle import model, newton
from helpers import ELBO_RTOL

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


def _oracle_fit(args):
    sb, s = args
    imgs = model.source_images(sb, s)
    th0 = oinit.plain_init(sb.u_cat[s], imgs, sb.prior)
    r = newton.fit(th0, imgs, sb.prior, sb.profiles)
    return th0, r.theta, r.elbo, r.iters, r.status


def _oracle_fits(sb):
    with mp.get_context("fork").Pool(min(8, sb.n_sources)) as pool:
        return pool.map(_oracle_fit, [(sb, s) for s in range(sb.n_sources)])


def _fit_ok(sb, s, theta_gpu, elbo_ref):
    """A22 rule: the oracle's ELBO at the GPU result is within 1e-5 relative of the oracle
    optimum, or above it."""
    v = model.elbo_value(theta_gpu, model.source_images(sb, s), sb.prior, sb.profiles)
    return v >= elbo_ref - ELBO_RTOL * abs(elbo_ref), v


def test_newton_fit_config0(cb, ctx):
    sb = synth.make_config(0)
    th0, th_ref, e_ref, it_ref, st_ref = _oracle_fit((sb, 0))
    th, res = ctx.newton_fit(cb.Batch.from_synth(sb), th0)
    ok, v = _fit_ok(sb, 0, th[0], e_ref)
    _say("newton config0: gpu", res["elbo"], v, res["iters"], res["status"], "oracle", e_ref, it_ref, st_ref)
    assert res["status"] == cb.CONVERGED and res["iters"] <= 50
    assert ok
    assert abs(res["elbo"] - v) <= ELBO_RTOL * abs(v)


def test_batch_fit_config1_subset(cb, ctx):
    full = synth.make_config(1)
    sb = full.subset(list(range(12)))
    ref = _oracle_fits(sb)
    th0 = np.stack([r[0] for r in ref])
    b = cb.Batch.from_synth(sb)
    th, res = ctx.batch_fit(b, th0)
    # the device plain start reproduces the oracle's plain start
    thp = sb.theta_truth.copy()
    thp[:, 0:2] = sb.u_cat
    th2, res2 = ctx.batch_fit(b, thp, cb.default_opts(init_mode=cb.INIT_PLAIN))
    n_ok = 0
    for s in range(sb.n_sources):
        ok, v = _fit_ok(sb, s, th[s], ref[s][2])
        ok2, v2 = _fit_ok(sb, s, th2[s], ref[s][2])
        _say(f"source {s}: gpu {v:.6f} it {res['iters'][s]} st {res['status'][s]} | plain-start {v2:.6f} "
             f"it {res2['iters'][s]} | oracle {ref[s][2]:.6f} it {ref[s][3]} st {ref[s][4]}")
        n_ok += ok and ok2
        assert res["iters"][s] <= 50
    assert n_ok == sb.n_sources


def test_batch_equals_single_and_graph_equals_eager(cb, ctx):
    full = synth.make_config(1, n_sources=3)
    b = cb.Batch.from_synth(full)
    th0 = full.theta_truth.copy()
    th0[:, 0:2] = full.u_cat
    o = cb.default_opts(init_mode=cb.INIT_PLAIN)
    th_b, res_b = ctx.batch_fit(b, th0, o)
    ctx.set_option(cb.OPT_USE_GRAPH, 0)
    try:
        th_e, res_e = ctx.batch_fit(b, th0, o)
    finally:
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
    assert np.array_equal(th_b, th_e) and np.array_equal(res_b["iters"], res_e["iters"])
    for s in range(3):
        one = full.subset([s])
        th_s, res_s = ctx.newton_fit(cb.Batch.from_synth(one), th0[s], o)
        assert np.array_equal(th_s[0], th_b[s]), s
        assert res_s["iters"] == res_b["iters"][s]


def test_persistent_work_queue_equals_one_block_per_item(cb, ctx):
    """Fits whose pixel kernels draw from the device list of the work items still being fitted
    (persistent grids of 1 and 4 blocks per compute unit) give every bit of the one-block-per-item
    fits: a ragged config-1 subset and config-2 sources, graph replay and eager, chunks small
    enough that many sources span several work items."""
    c1 = synth.make_config(1, n_sources=40)
    side = c1.truth["side"]
    sets = [c1.subset(list(np.argsort(side)[:5]) + list(np.argsort(side)[-5:])),
            synth.make_config(2, n_sources=30).subset(list(range(0, 30, 3)))]
    try:
        for sb in sets:
            b = cb.Batch.from_synth(sb)
            th0 = np.zeros((sb.n_sources, 27))
            th0[:, 0:2] = sb.u_cat
            o = cb.default_opts(init_mode=cb.INIT_PLAIN)
            for chunk in (4096, 1024):
                ctx.set_option(cb.OPT_CHUNK_PX, chunk)
                ctx.set_option(cb.OPT_PERSISTENT, 0)
                th_a, ra = ctx.batch_fit(b, th0, o)
                ctx.set_option(cb.OPT_PERSISTENT, 1)
                th_p, rp = ctx.batch_fit(b, th0, o)
                ctx.set_option(cb.OPT_PERSISTENT, 4)
                th_q, rq = ctx.batch_fit(b, th0, o)
                ctx.set_option(cb.OPT_USE_GRAPH, 0)
                th_e, re_ = ctx.batch_fit(b, th0, o)
                ctx.set_option(cb.OPT_USE_GRAPH, 1)
                for th_x, rx in ((th_p, rp), (th_q, rq), (th_e, re_)):
                    assert np.array_equal(th_x, th_a) and np.array_equal(rx["elbo"], ra["elbo"])
                    assert np.array_equal(rx["iters"], ra["iters"]) and np.array_equal(rx["status"], ra["status"])
            _say("persistent", sb.name, "iterations", ra["iters"].tolist())
    finally:
        ctx.set_option(cb.OPT_PERSISTENT, -1)   # the library's default
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
        ctx.set_option(cb.OPT_CHUNK_PX, 4096)
    for bad in (-2, 17):
        with pytest.raises(cb.CelesteError):
            ctx.set_option(cb.OPT_PERSISTENT, bad)


def test_default_persistent_grid_follows_kernel_occupancy(cb, ctx):
    """The default persistent grid holds as many blocks per compute unit as the launched kernel
    instance keeps resident: the three-wave register budget (variant bit 0) gives 3 blocks of 256
    threads (6 of 128) per compute unit, the other budget 2 (4); every grid gives the
    one-block-per-item results bit for bit."""
    sb = synth.make_config(1, n_sources=12)
    b = cb.Batch.from_synth(sb)
    th0 = np.zeros((sb.n_sources, 27))
    th0[:, 0:2] = sb.u_cat
    o = cb.default_opts(init_mode=cb.INIT_PLAIN, max_iter=6)

    def grid():
        ctx.stats(reset=True)
        th, r = ctx.batch_fit(b, th0, o)
        return ctx.stats()["fit_grid_blocks"], th, r

    try:
        ctx.set_option(cb.OPT_PERSISTENT, 0)
        n0, th_a, ra = grid()
        assert n0 == 0
        ctx.set_option(cb.OPT_PERSISTENT, 1)
        n_cu, _, _ = grid()
        assert n_cu > 0
        ctx.set_option(cb.OPT_PERSISTENT, -1)
        first = {256: (th_a, ra)}   # the grids of one block size sum in the same order
        for block, variant, per_cu in ((256, 3, 3), (256, 2, 2), (128, 3, 6), (128, 2, 4)):
            ctx.set_option(cb.OPT_BLOCK, block)
            ctx.set_option(cb.OPT_VARIANT, variant)
            n, th, r = grid()
            _say("grid", block, variant, n, n_cu)
            assert n == per_cu * n_cu, (block, variant, n, n_cu)
            th_f, r_f = first.setdefault(block, (th, r))
            assert np.array_equal(th, th_f) and np.array_equal(r["elbo"], r_f["elbo"])
            assert np.array_equal(r["iters"], r_f["iters"])
    finally:
        ctx.set_option(cb.OPT_PERSISTENT, -1)
        ctx.set_option(cb.OPT_BLOCK, 256)
        ctx.set_option(cb.OPT_VARIANT, 3)


def test_trial_derivatives_match_derivatives_at_accepted_points(cb, ctx):
    """Trust-region fits that evaluate the gradient and Hessian at every trial point (the default)
    against fits that evaluate them only at accepted points (section III-B runs the same algorithm
    either way): the same statuses, ELBO values that agree to rounding, the same accepted steps on
    almost every source, and the evaluation counts each mode implies (with trial derivatives
    iterations + 1 full evaluations; otherwise accepted steps + 1).  A ragged config-1 subset
    and config-2 sources, graph replay and eager."""
    c1 = synth.make_config(1, n_sources=40)
    side = c1.truth["side"]
    sets = [c1.subset(list(np.argsort(side)[:6]) + list(np.argsort(side)[-6:])),
            synth.make_config(2, n_sources=30).subset(list(range(0, 30, 3)))]
    try:
        for sb in sets:
            b = cb.Batch.from_synth(sb)
            th0 = np.zeros((sb.n_sources, 27))
            th0[:, 0:2] = sb.u_cat
            o = cb.default_opts(init_mode=cb.INIT_PLAIN)
            ctx.set_option(cb.OPT_TRIAL_DERIVATIVES, 0)
            th_a, ra = ctx.batch_fit(b, th0, o)
            ctx.set_option(cb.OPT_TRIAL_DERIVATIVES, 1)
            ctx.stats(reset=True)
            th_t, rt = ctx.batch_fit(b, th0, o)
            st = ctx.stats()
            # the pixel counters: the start pass, one trial pass per iteration, and the pixels of
            # every accepted step (what the CPU baseline rebuilds the oracle's evaluations from)
            npix = np.array([int(np.sum(sb.img_h[sb.src_img_off[k]:sb.src_img_off[k + 1]].astype(np.int64)
                                        * sb.img_w[sb.src_img_off[k]:sb.src_img_off[k + 1]]))
                             for k in range(sb.n_sources)])
            assert st["trial_full_px"] == int(np.sum(npix * rt["iters"]))
            assert st["taken_px"] == int(np.sum(npix * rt["n_accepted"]))
            assert st["full_px"] - st["trial_full_px"] == int(np.sum(npix))
            ctx.set_option(cb.OPT_USE_GRAPH, 0)
            th_e, re_ = ctx.batch_fit(b, th0, o)
            ctx.set_option(cb.OPT_USE_GRAPH, 1)
            assert np.array_equal(th_e, th_t) and np.array_equal(re_["elbo"], rt["elbo"])
            assert np.array_equal(rt["status"], ra["status"]), (rt["status"], ra["status"])
            assert np.all(rt["status"] == cb.CONVERGED)
            rel = np.abs(rt["elbo"] - ra["elbo"]) / np.abs(ra["elbo"])
            _say("trial derivatives", sb.name, "iters", rt["iters"].tolist(), ra["iters"].tolist(),
                 "max rel ELBO diff", float(rel.max()))
            assert rel.max() <= 1e-7
            same = np.mean(rt["n_accepted"] == ra["n_accepted"])
            assert same >= 0.9, same
            assert np.array_equal(rt["n_full_evals"], rt["iters"] + 1)
            assert np.array_equal(ra["n_full_evals"], ra["n_accepted"] + 1)
            assert np.all(rt["n_accepted"] <= rt["iters"]) and np.all(rt["reserved"] == 0)
    finally:
        ctx.set_option(cb.OPT_TRIAL_DERIVATIVES, 1)
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
    for bad in (-1, 2):
        with pytest.raises(cb.CelesteError):
            ctx.set_option(cb.OPT_TRIAL_DERIVATIVES, bad)


def test_interior_cholesky_step_matches_eigendecomposition(cb, ctx):
    """The Cholesky paths of the subproblem (where -H is positive definite: the interior Newton
    step, or the boundary step by Newton's method on the multiplier) against the
    eigendecomposition path on every iteration: the same fits up to rounding (ELBO within 1e-9
    relative, parameters within 1e-5 of their scale, every source converged both ways, iteration
    counts within one) on a ragged config-1 subset and config-2 sources, graph replay, and eager
    with the option cleared; both Cholesky paths are taken."""
    c1 = synth.make_config(1, n_sources=40)
    side = c1.truth["side"]
    sets = [c1.subset(list(np.argsort(side)[:6]) + list(np.argsort(side)[-6:])),
            synth.make_config(2, n_sources=40).subset(list(range(0, 40, 4)))]
    try:
        for sb in sets:
            b = cb.Batch.from_synth(sb)
            th0 = np.zeros((sb.n_sources, 27))
            th0[:, 0:2] = sb.u_cat
            o = cb.default_opts(init_mode=cb.INIT_PLAIN)
            ctx.set_option(cb.OPT_TR_CHOLESKY, 1)
            ctx.stats(reset=True)
            th_c, rc = ctx.batch_fit(b, th0, o)
            st = ctx.stats()
            _say(sb.name, "subproblems: interior", st["tr_interior"], "boundary", st["tr_boundary"],
                 "eigendecomposition", st["tr_eigen"])
            assert st["tr_interior"] > 0 and st["tr_boundary"] > 0
            assert st["tr_interior"] + st["tr_boundary"] + st["tr_eigen"] == int(np.sum(rc["iters"])) + sb.n_sources
            ctx.set_option(cb.OPT_TR_CHOLESKY, 0)
            th_e, re_ = ctx.batch_fit(b, th0, o)
            ctx.set_option(cb.OPT_USE_GRAPH, 0)
            th_e2, re2 = ctx.batch_fit(b, th0, o)
            ctx.set_option(cb.OPT_USE_GRAPH, 1)
            _say(sb.name, "iterations cholesky", rc["iters"].tolist(), "eigen", re_["iters"].tolist())
            assert np.array_equal(th_e2, th_e) and np.array_equal(re2["iters"], re_["iters"])
            assert np.all(rc["status"] == cb.CONVERGED) and np.all(re_["status"] == cb.CONVERGED)
            assert np.all(np.abs(rc["elbo"] - re_["elbo"]) <= 1e-9 * np.abs(re_["elbo"]))
            assert np.all(np.abs(rc["iters"] - re_["iters"]) <= 1)
            assert np.max(np.abs(th_c - th_e) / np.maximum(1.0, np.abs(th_e))) <= 1e-5
    finally:
        ctx.set_option(cb.OPT_TR_CHOLESKY, 1)
        ctx.set_option(cb.OPT_USE_GRAPH, 1)
    with pytest.raises(cb.CelesteError):
        ctx.set_option(cb.OPT_TR_CHOLESKY, 2)


def test_status_paths_forced_from_host(cb, ctx):
    sb = synth.make_config(0)
    b = cb.Batch.from_synth(sb)
    th0 = oinit.plain_init(sb.u_cat[0], model.source_images(sb, 0), sb.prior)[None, :]
    _, r = ctx.batch_fit(b, th0, cb.default_opts(max_iter=1))
    assert r["status"][0] == cb.MAX_ITER and r["iters"][0] == 1
    _, r = ctx.batch_fit(b, th0, cb.default_opts(delta0=1e-12, delta_min=1e-10))
    assert r["status"][0] == cb.TR_COLLAPSED
    bad = th0.copy()
    bad[0, 7:9] = 800.0          # brightness overflows: non-finite starting ELBO
    _, r = ctx.batch_fit(b, bad, cb.default_opts())
    assert r["status"][0] == cb.NONFINITE and r["iters"][0] == 0
    with pytest.raises(cb.CelesteError):
        ctx.batch_fit(b, th0, cb.default_opts(max_iter=0))
