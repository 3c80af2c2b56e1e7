"""GPU parity of celeste_elbo_eval against the FP64 oracle (through the C ABI)."""
import math
import sys

import numpy as np
import pytest

import synth
from synth.generate import perturb_theta
from oracle import init as oinit
from oracle import model
from helpers import assert_derivs_close, assert_elbo_close, assert_structural_zeros, deriv_err, oracle_eval

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


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_config(0)


def _points(sb, seed):
    pts = [sb.theta_truth.copy(), perturb_theta(sb.theta_truth, seed)]
    plain = np.stack([oinit.plain_init(sb.u_cat[s], model.source_images(sb, s), sb.prior)
                      for s in range(sb.n_sources)])
    pts.append(plain)
    return pts


def _check_batch(cb, ctx, sb, thetas, nbr=None, what=""):
    b = cb.Batch.from_synth(sb, nbr=nbr)
    for k, th in enumerate(thetas):
        el, g, H = ctx.elbo_eval(b, th)
        for s in range(sb.n_sources):
            onbr = None
            if nbr is not None:
                onbr = {i: (nbr[0][sb.img_pix_off[i]:sb.img_pix_off[i] + sb.img_h[i] * sb.img_w[i]].reshape(
                    sb.img_h[i], sb.img_w[i]),
                    nbr[1][sb.img_pix_off[i]:sb.img_pix_off[i] + sb.img_h[i] * sb.img_w[i]].reshape(
                        sb.img_h[i], sb.img_w[i])) for i in range(sb.src_img_off[s], sb.src_img_off[s + 1])}
            v0, g0, H0 = oracle_eval(sb, s, th[s], nbr=onbr)
            tag = f"{what} point {k} source {s}"
            _say(tag, "elbo", el[s], v0, "gerr", deriv_err(g[s], g0), "herr", deriv_err(H[s], H0))
            assert_elbo_close(el[s], v0, what=tag)
            assert_derivs_close(g[s], H[s], g0, H0, what=tag)
            assert_structural_zeros(H0, what="oracle " + tag)
            assert_structural_zeros(H[s], what="GPU " + tag)


def test_config0_three_points(cb, ctx, cfg0):
    _say("case: config0, 3 points")
    _check_batch(cb, ctx, cfg0, _points(cfg0, 1), what="cfg0")


def test_config1_ragged_subset_small_chunks(cb, ctx):
    """Sources of the smallest and largest patch sides, work items of 512 px (ragged tails)."""
    full = synth.make_config(1)
    side = full.truth["side"]
    idx = list(np.argsort(side)[:3]) + list(np.argsort(side)[-3:])
    sb = full.subset(idx)
    _say("case: config1 subset sides", side[idx])
    ctx.set_option(cb.OPT_CHUNK_PX, 512)
    try:
        _check_batch(cb, ctx, sb, [perturb_theta(sb.theta_truth, 3)], what="cfg1")
    finally:
        ctx.set_option(cb.OPT_CHUNK_PX, 4096)


def test_multi_epoch_wcs_offsets(cb, ctx):
    full = synth.make_config(2, n_sources=40)
    npx = np.array([np.sum(full.img_h[full.src_img_off[s]:full.src_img_off[s + 1]].astype(np.int64) ** 2)
                    for s in range(full.n_sources)])
    multi = [s for s in range(full.n_sources) if full.truth["epochs"][s] > 1 and npx[s] < 60000]
    sb = full.subset(multi[:3])
    _say("case: multi-epoch", sb.truth["epochs"], sb.truth["side"])
    _check_batch(cb, ctx, sb, [perturb_theta(sb.theta_truth, 4), sb.theta_truth], what="cfg2")


def test_neighbours_and_general_wcs(cb, ctx, cfg0):
    sb = cfg0.subset([0])
    rng = np.random.default_rng(5)
    ang = 0.4
    A = 0.9 * np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    sb.img_wcs[:, 0:4] = A.ravel()
    sb.img_wcs[:, 4:6] = [1.3, -0.7]
    n = sb.n_pixels
    nbr = (rng.uniform(0, 30, n).astype(np.float32), rng.uniform(0, 8, n).astype(np.float32))
    th = perturb_theta(sb.theta_truth, 6)
    th[:, 0:2] = np.linalg.solve(A, (np.array([15.0, 15.0]) - sb.img_wcs[0, 4:6]))[None, :]
    _say("case: neighbours + rotated WCS")
    _check_batch(cb, ctx, sb, [th], nbr=nbr, what="nbr")


@pytest.mark.parametrize("case", ["round", "pure_star", "pure_gal", "dev_edge", "bright", "tiny_patch"])
def test_degenerate_points(cb, ctx, cfg0, case):
    sb = cfg0.subset([0])
    th = perturb_theta(sb.theta_truth, 7)
    if case == "round":
        th[0, 4] = 1.0
    elif case == "pure_star":
        th[0, 2] = 1 - 1e-4
    elif case == "pure_gal":
        th[0, 2] = 1e-4
    elif case == "dev_edge":
        th[0, 3] = 0.0
    elif case == "bright":
        sb = synth.make_config(1, n_sources=2, bright=True).subset([0])
        th = perturb_theta(sb.theta_truth, 8)
    elif case == "tiny_patch":
        sb.img_h[:] = 1
        sb.img_w[:] = 1
        sb.img_pitch[:] = cfg0.img_w
        th[0, 0:2] = [0.2, -0.1]
    _say("case: degenerate", case)
    _check_batch(cb, ctx, sb, [th], what=case)


def test_deterministic_and_batch_equals_single(cb, ctx):
    full = synth.make_config(1, n_sources=6)
    th = perturb_theta(full.theta_truth, 9)
    b = cb.Batch.from_synth(full)
    e1, g1, H1 = ctx.elbo_eval(b, th)
    e2, g2, H2 = ctx.elbo_eval(b, th)
    assert np.array_equal(e1, e2) and np.array_equal(g1, g2) and np.array_equal(H1, H2)
    for s in (0, 3, 5):
        one = full.subset([s])
        e, g, H = ctx.elbo_eval(cb.Batch.from_synth(one), th[s:s + 1])
        assert e[0] == e1[s] and np.array_equal(g[0], g1[s]) and np.array_equal(H[0], H1[s])
    # block size regroups the per-lane FP32 sums of the derivative terms (the value is
    # summed in FP64 per lane): results move by FP32 rounding of those partial sums only
    ctx.set_option(cb.OPT_BLOCK, 128)
    try:
        e3, g3, H3 = ctx.elbo_eval(b, th)
    finally:
        ctx.set_option(cb.OPT_BLOCK, 256)
    assert np.allclose(e3, e1, rtol=1e-12) and deriv_err(g3, g1) < 2e-5 and deriv_err(H3, H1) < 2e-5


def test_exact_zero_threshold_changes_no_bit(cb, ctx):
    """Skipping components below 2^-127 instead of 2^-160 on a tile skips only work that is
    exactly zero on this device (its exp2 flushes results below 2^-126): every output bit is the
    same, with and without neighbour arrays."""
    full = synth.make_config(1, n_sources=6)
    th = perturb_theta(full.theta_truth, 14)
    rng = np.random.default_rng(15)
    n = full.n_pixels
    nbr = (rng.uniform(0, 30, n).astype(np.float32), rng.uniform(0, 8, n).astype(np.float32))
    try:
        for batch in (cb.Batch.from_synth(full), cb.Batch.from_synth(full, nbr=nbr)):
            ctx.set_option(cb.OPT_EXACT_ZERO, 160)
            e1, g1, H1 = ctx.elbo_eval(batch, th)
            try:
                ctx.set_option(cb.OPT_EXACT_ZERO, 127)
            except cb.CelesteError as err:
                assert err.code == cb.E_UNSUPPORTED
                pytest.skip("this device's exp2 keeps subnormal results")
            e2, g2, H2 = ctx.elbo_eval(batch, th)
            assert np.array_equal(e1, e2) and np.array_equal(g1, g2) and np.array_equal(H1, H2)
    finally:
        ctx.set_option(cb.OPT_EXACT_ZERO, 0)
    with pytest.raises(cb.CelesteError) as ei:
        ctx.set_option(cb.OPT_EXACT_ZERO, 100)
    assert ei.value.code == cb.E_INVALID


def test_skips_match_no_skip_reference(cb, ctx):
    """Every exact-zero skip of the value+gradient+Hessian kernel (single components, whole
    galaxy groups under their bound, tiles no component reaches) against the option that skips
    nothing: every output bit is the same, on a ragged config-1 subset (with and without
    neighbour arrays, vector and matrix-core J^T W J, tile widths 8 and 16) and on a sample of
    config-2 sources (multi-epoch, per-epoch PSF and sky)."""
    c1 = synth.make_config(1, n_sources=8)
    th1 = perturb_theta(c1.theta_truth, 16)
    rng = np.random.default_rng(17)
    nbr = (rng.uniform(0, 30, c1.n_pixels).astype(np.float32), rng.uniform(0, 8, c1.n_pixels).astype(np.float32))
    c2 = synth.make_config(2, n_sources=120).subset([3, 40, 77, 119])
    th2 = perturb_theta(c2.theta_truth, 18)
    cases = [(c1, th1, None, 3, 8), (c1, th1, nbr, 3, 8), (c1, th1, nbr, 7, 16), (c2, th2, None, 3, 8)]
    try:
        for k, (sb, th, nb, variant, tw) in enumerate(cases):
            _say("case: no-skip reference", k, sb.name, "variant", variant, "tile", tw, "nbr", nb is not None)
            ctx.set_option(cb.OPT_VARIANT, variant)
            ctx.set_option(cb.OPT_TILE_W, tw)
            b = cb.Batch.from_synth(sb, nbr=nb)
            ctx.set_option(cb.OPT_EXACT_ZERO, 1)
            e0, g0, H0 = ctx.elbo_eval(b, th)
            ctx.set_option(cb.OPT_EXACT_ZERO, 0)
            e1, g1, H1 = ctx.elbo_eval(b, th)
            assert np.array_equal(e0, e1), f"case {k}: ELBO"
            assert np.array_equal(g0, g1), f"case {k}: gradient"
            assert np.array_equal(H0, H1), f"case {k}: Hessian"
            # the reference itself meets the oracle on one source
            v, g, H = oracle_eval(sb, 0, th[0], nbr=_oracle_nbr(sb, nb))
            assert_elbo_close(e0[0], v, what=f"no-skip case {k}")
            assert_derivs_close(g0[0], H0[0], g, H, what=f"no-skip case {k}")
    finally:
        ctx.set_option(cb.OPT_EXACT_ZERO, 0)
        ctx.set_option(cb.OPT_VARIANT, 3)
        ctx.set_option(cb.OPT_TILE_W, 8)


def _oracle_nbr(sb, nb):
    if nb is None:
        return None
    out = {}
    for i in range(int(sb.src_img_off[0]), int(sb.src_img_off[1])):
        o, h, w = int(sb.img_pix_off[i]), int(sb.img_h[i]), int(sb.img_w[i])
        out[i] = (nb[0][o:o + h * w].reshape(h, w), nb[1][o:o + h * w].reshape(h, w))
    return out


def test_value_only_matches_full(cb, ctx):
    full = synth.make_config(1, n_sources=5)
    th = perturb_theta(full.theta_truth, 10)
    b = cb.Batch.from_synth(full)
    ev, _, _ = ctx.elbo_eval(b, th, want="value")
    ef, gf, _ = ctx.elbo_eval(b, th, want="grad")
    for s in range(5):
        v0, _, _ = oracle_eval(full, s, th[s], want="value")
        assert_elbo_close(ev[s], v0, what=f"value-only {s}")
        assert_elbo_close(ef[s], v0, what=f"grad-only {s}")


def test_device_memory_batch(cb, ctx):
    import torch
    full = synth.make_config(1, n_sources=4)
    dev = synth.make_config(1, n_sources=4)
    dev.pixels = torch.from_numpy(full.pixels).cuda()
    th = perturb_theta(full.theta_truth, 11)
    eh, gh, Hh = ctx.elbo_eval(cb.Batch.from_synth(full), th)
    ed, gd, Hd = ctx.elbo_eval(cb.Batch.from_synth(dev), torch.from_numpy(th).cuda())
    assert np.array_equal(eh, ed.cpu().numpy()) and np.array_equal(Hh, Hd.cpu().numpy())


@pytest.mark.parametrize("bad", ["nan_pixel", "neg_pixel", "band", "n_psf", "a_range", "pitch"])
def test_invalid_inputs_rejected(cb, ctx, cfg0, bad):
    sb = cfg0.subset([0])
    th = sb.theta_truth.copy()
    b = cb.Batch.from_synth(sb)
    if bad == "nan_pixel":
        b._keep[0][17] = np.nan
    elif bad == "neg_pixel":
        b._keep[0][3] = -1.0
    elif bad == "band":
        b.images["band"][2] = 7
    elif bad == "n_psf":
        b.images["n_psf"][0] = 5
    elif bad == "a_range":
        th[0, 2] = 1.5
    elif bad == "pitch":
        b.images["pitch"][1] = 3
    with pytest.raises(cb.CelesteError) as ei:
        ctx.elbo_eval(b, th)
    assert ei.value.code == cb.E_INVALID


def test_full_size_config2_sampled(cb, ctx):
    """Config 2 at its full size on device memory, launch as the benchmark runs it;
    the oracle checks a sample of sources one by one."""
    import torch
    sb = synth.make_config(2, device="cuda")
    _say("case: config2 full size", sb.n_sources, "sources", sb.n_pixels, "pixels")
    th = perturb_theta(sb.theta_truth, 12, scale=0.5)
    b = cb.Batch.from_synth(sb)
    el, g, H = ctx.elbo_eval(b, torch.from_numpy(th).cuda())
    el, g, H = el.cpu().numpy(), g.cpu().numpy(), H.cpu().numpy()
    assert np.all(np.isfinite(el)) and np.all(np.isfinite(H))
    npx = np.array([np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64) ** 2)
                    for s in range(sb.n_sources)])
    rng = np.random.default_rng(13)
    pick = [int(np.argmin(npx)), int(rng.integers(sb.n_sources)), int(np.argsort(npx)[len(npx) // 2])]
    sub = sb.subset(pick)
    for k, s in enumerate(pick):
        v0, g0, H0 = oracle_eval(sub, k, th[s])
        tag = f"cfg2 full source {s} ({npx[s]} px)"
        _say(tag, el[s], v0, deriv_err(g[s], g0), deriv_err(H[s], H0))
        assert_elbo_close(el[s], v0, what=tag)
        assert_derivs_close(g[s], H[s], g0, H0, what=tag)


def test_fp64_sums(cb, ctx, cfg0):
    """CELESTE_OPT_FP64_SUMS: every pixel's FP32 gradient and Hessian terms summed in FP64 from the
    first addition.  Against the oracle to the same tolerances on config 0 (three points), a ragged
    config-1 subset with neighbour arrays and small work items, and config-2 sources; and, since
    only the FP64 summation order then depends on the launch shape, two different launch shapes
    (block 256 / tile 8 / vector variant, block 128 / tile 32 / unrolled variant) agree to 1e-11 of
    each array's largest entry (the default FP32 lane sums differ by about 1e-6 there)."""
    c1 = synth.make_config(1, n_sources=40)
    side = c1.truth["side"]
    c1 = c1.subset(list(np.argsort(side)[:3]) + list(np.argsort(side)[-3:]))
    rng = np.random.default_rng(23)
    nb = (rng.uniform(0, 30, c1.n_pixels).astype(np.float32), rng.uniform(0, 8, c1.n_pixels).astype(np.float32))
    c2 = synth.make_config(2, n_sources=60).subset([3, 29, 58])
    shapes = ((256, 8, 3, 4096), (128, 32, 2, 1024))

    def spread(a, b):
        return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))

    try:
        ctx.set_option(cb.OPT_FP64_SUMS, 1)
        _check_batch(cb, ctx, cfg0, _points(cfg0, 4), what="fp64 sums cfg0")
        ctx.set_option(cb.OPT_CHUNK_PX, 512)
        _check_batch(cb, ctx, c1, [perturb_theta(c1.theta_truth, 5)], nbr=nb, what="fp64 sums cfg1")
        ctx.set_option(cb.OPT_CHUNK_PX, 4096)
        _check_batch(cb, ctx, c2, [perturb_theta(c2.theta_truth, 6)], what="fp64 sums cfg2")
        for sb, th, n_ in ((c1, perturb_theta(c1.theta_truth, 5), nb), (c2, perturb_theta(c2.theta_truth, 6), None)):
            b = cb.Batch.from_synth(sb, nbr=n_)
            out = {}
            for f64 in (1, 0):
                ctx.set_option(cb.OPT_FP64_SUMS, f64)
                res = []
                for blk, tw, var, chunk in shapes:
                    ctx.set_option(cb.OPT_BLOCK, blk)
                    ctx.set_option(cb.OPT_TILE_W, tw)
                    ctx.set_option(cb.OPT_VARIANT, var)
                    ctx.set_option(cb.OPT_CHUNK_PX, chunk)
                    res.append(ctx.elbo_eval(b, th))
                out[f64] = [(spread(res[0][0][s], res[1][0][s]), spread(res[0][1][s], res[1][1][s]),
                             spread(res[0][2][s], res[1][2][s])) for s in range(sb.n_sources)]
            _say(sb.name, "launch-shape spread (elbo, grad, hess) fp64 sums", np.max(out[1], axis=0),
                 "fp32 lane sums", np.max(out[0], axis=0))
            for s, (de, dg, dh) in enumerate(out[1]):
                assert de <= 1e-13 and dg <= 1e-11 and dh <= 1e-11, (sb.name, s, de, dg, dh)
    finally:
        ctx.set_option(cb.OPT_FP64_SUMS, 0)
        _restore_defaults(cb, ctx)
    with pytest.raises(cb.CelesteError):
        ctx.set_option(cb.OPT_FP64_SUMS, 2)


def _autotune_case(cb):
    full = synth.make_config(1, n_sources=12)
    th = perturb_theta(full.theta_truth, 31)
    ref = [oracle_eval(full, s, th[s]) for s in (0, 7)]
    return full, th, cb.Batch.from_synth(full), ref


def _restore_defaults(cb, ctx):
    for opt, v in ((cb.OPT_CHUNK_PX, 4096), (cb.OPT_BLOCK, 256), (cb.OPT_VARIANT, 3), (cb.OPT_TILE_W, 8),
                   (cb.OPT_VALUE_BLOCK, 256), (cb.OPT_VALUE_TILE_W, 8)):
        ctx.set_option(opt, v)


def test_tile_shapes(cb, ctx):
    """Every tile width and launch shape gives the oracle's results."""
    full, th, b, ref = _autotune_case(cb)
    try:
        for tw, variant in ((8, 7), (8, 3), (16, 6), (32, 2), (64, 7)):
            ctx.set_option(cb.OPT_VARIANT, variant)   # 6, 7: J^T W J on the matrix cores
            ctx.set_option(cb.OPT_TILE_W, tw)
            ctx.set_option(cb.OPT_VALUE_TILE_W, 64 // (tw // 8))
            e, g, H = ctx.elbo_eval(b, th)
            ev, _, _ = ctx.elbo_eval(b, th, want="value")
            for k, s in enumerate((0, 7)):
                what = f"tile {tw} variant {variant} source {s}"
                assert_elbo_close(e[s], ref[k][0], what=what)
                assert_elbo_close(ev[s], ref[k][0], what="value " + what)
                assert_derivs_close(g[s], H[s], ref[k][1], ref[k][2], what=what)
    finally:
        _restore_defaults(cb, ctx)


def test_autotune_and_cache(cb, ctx, tmp_path):
    """The autotuner picks a launch configuration, applies it (the oracle's results still hold),
    reads it back from its cache file and rejects a bad cache entry.  The default options are
    re-timed in the same pass as the finalists, so the pick is never slower than the default by
    that pass's own timings (an identity of the selection, not a timing claim)."""
    full, th, b, ref = _autotune_case(cb)
    try:
        cache = str(tmp_path / "tune.txt")
        r = ctx.autotune(b, th, sample_px=200000, cache_path=cache)
        _say("autotune", r)
        assert r["from_cache"] == 0 and r["n_candidates"] == 104 and r["sample_sources"] >= 1
        assert r["tile_w"] in (8, 16, 32, 64) and r["value_tile_w"] in (8, 16, 32, 64)
        assert r["block"] in (128, 256) and r["chunk_px"] in (4096, 8192, 16384) and r["variant"] in (2, 3, 6, 7)
        assert 0 < r["full_ms"] <= r["default_full_ms"] and 0 < r["value_ms"]
        e, g, H = ctx.elbo_eval(b, th)
        for k, s in enumerate((0, 7)):
            assert_elbo_close(e[s], ref[k][0], what=f"tuned source {s}")
            assert_derivs_close(g[s], H[s], ref[k][1], ref[k][2], what=f"tuned source {s}")
        r2 = ctx.autotune(b, th, cache_path=cache)
        assert r2["from_cache"] == 1
        assert all(r2[k] == r[k] for k in ("chunk_px", "block", "variant", "tile_w", "value_block", "value_tile_w"))
        with open(cache, "a") as f:
            key = open(cache).read().split()[0]
            f.write(f"{key} 4096 100 3 8 256 8 1.0 1.0\n")
        with pytest.raises(cb.CelesteError):
            ctx.autotune(b, th, cache_path=cache)
    finally:
        _restore_defaults(cb, ctx)
