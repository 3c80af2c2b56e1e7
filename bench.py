#!/usr/bin/env python3
"""Benchmark of the Celeste hot path on one MI355X.

One step = a whole batched trust-region Newton fit (celeste_batch_fit) of the
batched-uneven workload, started by the surrogate network with the plain start
as fallback (the network is trained first, outside the timed region, on plain
fits of 200,000 single-epoch sources): 20,000 sources,
patch side log-uniform in 15..121 px, 5 bands x 1..10 epochs per source, each
epoch with its own PSF (widths 1..3 px) and sky (50..300 counts/px); 1.90e9
pixels resident in HBM before the timed region.  Every step evaluates ELBO,
gradient and dense Hessian by the pixel sum for all still-active sources,
solves the 27x27 trust-region subproblems, evaluates trial points and applies
the ratio test, until every source has stopped.

Prints one JSON line: converged sources/s (whole job), pixel evaluations/s,
the roofline of the dominant kernel (value+gradient+Hessian pixel kernel,
timed with HIP events on the library's stream) and the FP64 CPU oracle timed
on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sources N] [--no-surrogate] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 FLOP x 2.4 GHz, one FMA per lane per clock
PEAK_HBM_GBS = 8000.0


PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_eval_full_batched_uneven_20k.json")


def pmc_traffic(px_per_launch):
    """HBM bytes per launch of the value+gradient+Hessian kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated, per pixel-eval), scaled to the launch's
    pixel count; None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        d = json.load(open(PMC_SUMMARY))
        src = open(os.path.join(ROOT, "paper_1611_03404_amd", "csrc", "pixel_kernels.hip"), "rb").read()
    except OSError:
        return None, None
    if hashlib.sha256(src).hexdigest() != d["pixel_kernels_sha256"]:
        return None, None
    k = d["kernels"]["k_eval_full"]
    per_px = (k["fetch_bytes"] + k["write_bytes"]) / d["n_pixels"]
    sq = k["sq"]
    util = sq["SQ_INSTS_VALU"] / (1024 * sq["GRBM_GUI_ACTIVE"] / 8 / 4)
    return per_px * px_per_launch, {"bytes_per_pixel_eval": per_px, "valu_issue_utilisation": util,
                                    "valu_insts_per_pixel_eval": sq["SQ_INSTS_VALU"] * 64 / d["n_pixels"],
                                    "source": "profiles/pmc_eval_full_batched_uneven_20k.md"}


def dtype_str(args, network=True):
    """The arithmetic types of the timed path (the pixel sums' precision follows --fp64-sums)."""
    sums = ("f64 pixel sums from the first addition" if args.fp64_sums == 1 else
            "f64 pixel sums after f32 lane sums of up to 16 pixels and an f32 wavefront butterfly")
    return "f32 pixel arithmetic, " + sums + ", f64 trust-region solve" + (", bf16 network" if network else "")


def flop_full_per_px(K, E, D):
    """FLOPs of the kernel's own arithmetic for one value+gradient+Hessian pixel evaluation
    without exact-zero skipping (add/mul 1, FMA 2, exp/log/rcp 1): star components 35 each,
    5 per PSF component for the offsets, 84 per galaxy component (Gaussian, Hermite moments
    to order 4, 18 accumulations), and 661 per pixel, the per-pixel block as compiled (profile
    mixing, shape contractions, rate moments, delta-method weights, the geometry entries in the
    basis of the two profile gradients, 12 brightness product sums and the FP32 lane
    accumulations)."""
    return 2 + 35 * K + 5 * K + 84 * K * (E + D) + 661


def flop_value_per_px(K, E, D):
    return K * (13 + 8 * (E + D)) + 30


def flop_full_per_px_algorithmic(K, E, D):
    """Algorithmic FP32 FLOPs of one value+gradient+Hessian pixel evaluation by the work units
    of the formulation: about 170 per galaxy component (the value, 5 gradient and 15 Hessian
    entries of a PSF-convolved Gaussian), 30 per star component and 400 per pixel for the rate
    moments and the delta-method term; the 78 FP64 accumulations (about 200 FLOP) are not
    counted.  The roofline's achieved rate uses this figure: it counts the work of every
    component, including those the kernel skips where they are exactly zero."""
    return 170 * K * (E + D) + 30 * K + 400


def host_cpu():
    """The host CPU the oracle ran on: model name and logical CPUs."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def stratified_sample(npx, n, seed):
    """One source drawn at random from each of n equal-count strata of the pixel-count order
    (a size-stratified sample of n sources)."""
    import numpy as np
    order = np.argsort(npx, kind="stable")
    edges = np.linspace(0, len(order), n + 1).astype(np.int64)
    rng = np.random.default_rng(seed)
    return [int(order[rng.integers(edges[i], edges[i + 1])]) for i in range(n) if edges[i + 1] > edges[i]]


def _one_thread():
    """Pool initialiser: one BLAS/OpenMP thread per worker process."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


class _indexed:
    """Wraps a worker so imap_unordered results carry their task index."""

    def __init__(self, fn):
        self.fn = fn

    def __call__(self, k):
        return k, self.fn(k)


def _oracle_eval_worker(args):
    sb, s, theta = args
    from oracle import model
    imgs = model.source_images(sb, s)
    t0 = time.perf_counter()
    v, g, H = model.elbo(theta, imgs, sb.prior, sb.profiles)
    t1 = time.perf_counter()
    model.elbo_value(theta, imgs, sb.prior, sb.profiles)
    t2 = time.perf_counter()
    npx = int(sum(int(im["h"]) * int(im["w"]) for im in imgs))
    return npx, t1 - t0, t2 - t1, v, g, H


def _rel_stats(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"max": float(np.max(x)), "median": float(np.median(x))}


def oracle_pattern_px(st):
    """Pixel evaluations (value+gradient+Hessian, value only) of the fits counted in the stats st,
    as the oracle's own trust-region iteration makes them: the ELBO alone at every trial point and
    the value, gradient and Hessian at the start and at each accepted point.  The GPU fits make
    exactly these without trial derivatives; with them, their trial-point passes (trial_full_px)
    stand for the oracle's value evaluations, and taken_px counts the oracle's evaluations at
    accepted points."""
    return (st["full_px"] - st["trial_full_px"] + st["taken_px"], st["value_px"] + st["trial_full_px"])


def cpu_baseline(sb, theta_fit, gpu_eval, gpu_full_px_per_step, gpu_value_px_per_step, converged_per_step,
                 budget_s=20.0):
    """Oracle timed on the host cores on a size-stratified sample of the workload: one
    value+gradient+Hessian and one value evaluation of each sampled source at the GPU fit's
    final parameters, scaled to whole fits with the GPU fits' pixel-evaluation counts per step.
    The same evaluations give the GPU's error against the oracle there: gpu_eval(pick) returns
    the GPU's ELBO, gradient and Hessian of the picked sources at theta_fit."""
    import multiprocessing as mp
    import numpy as np
    cores = max(1, min(16, os.cpu_count() or 1))
    npx = np.array([int(np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64)
                               * sb.img_w[sb.src_img_off[s]:sb.src_img_off[s + 1]])) for s in range(sb.n_sources)])
    # as many strata as the budget holds at ~8e-5 core-s per pixel (one full and one value evaluation)
    n = int(max(cores, min(4 * cores, budget_s * cores / (8e-5 * float(np.mean(npx))))))
    pick = stratified_sample(npx, n, 161103404)
    sub = sb.subset(pick)
    args = [(sub, k, np.asarray(theta_fit[s], dtype=np.float64)) for k, s in enumerate(pick)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_one_thread) as pool:
        out = pool.map(_oracle_eval_worker, args, chunksize=1)
    wall = time.perf_counter() - t0
    px = sum(o[0] for o in out)
    full_rate = px / sum(o[1] for o in out) * cores          # full pixel-evals/s on all cores
    val_rate = px / sum(o[2] for o in out) * cores
    step_s = gpu_full_px_per_step / full_rate + gpu_value_px_per_step / val_rate
    el, g, H = gpu_eval(pick)
    e_rel = [abs(el[k] - o[3]) / abs(o[3]) for k, o in enumerate(out)]

    def a23(got, ref):
        scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
        return float(np.max(np.abs(got - ref) / scale))

    return {
        "value": converged_per_step / step_s, "unit": "converged sources/s", "cores": cores, "kind": "oracle",
        "sample": (f"size-stratified sample of {len(pick)} sources of the same workload (one per equal-count "
                   f"stratum of the pixel-count order, {px} px): one value+gradient+Hessian and one value "
                   f"evaluation each at the GPU fit's final parameters on {cores} processes ({wall:.1f} s wall); "
                   f"scaled to whole fits with the pixel evaluations per step of the oracle's own iteration "
                   f"(the ELBO alone at trial points, value+gradient+Hessian at the start and at accepted points), "
                   f"counted in the GPU fits (extrapolated)"),
        "full_pixel_evals_per_s": full_rate, "value_pixel_evals_per_s": val_rate,
        "full_pixel_evals_per_s_per_core": full_rate / cores, "value_pixel_evals_per_s_per_core": val_rate / cores,
        "host_cpu": host_cpu(),
        "gpu_error_at_fitted_theta": {
            "sources": len(pick),
            "elbo_rel": _rel_stats(e_rel),
            "hessian_a23": _rel_stats([a23(H[k], o[5]) for k, o in enumerate(out)]),
            "gradient_a23": _rel_stats([a23(g[k], o[4]) for k, o in enumerate(out)]),
            "note": ("relative to max(|e*|, 1e-3 max|array*|) per source; the fitted point is stationary in the "
                     "fit's coordinates, so gradient entries there are differences of nearly cancelling terms"),
        },
    }


_FIT_JOB = None   # the sampled subset: inherited by forked workers


def _oracle_fit_worker(s):
    sb = _FIT_JOB
    from oracle import init as oinit
    from oracle import model, newton
    imgs = model.source_images(sb, s)
    t0 = time.perf_counter()
    th0 = oinit.plain_init(sb.u_cat[s], imgs, sb.prior)
    r = newton.fit(th0, imgs, sb.prior, sb.profiles)
    return time.perf_counter() - t0, float(r.elbo), int(r.iters), int(r.status)


def oracle_fit_baseline(sb, n, gpu_plain_elbo, gpu_head_elbo, log):
    """Complete oracle fits from the plain start of a size-stratified sample of n sources,
    timed on the host cores (measured fits, extrapolated to the workload by stratum), and the
    GPU fits' final ELBO against the oracle-converged one (pass: within 1e-5 |L*| or above)."""
    import multiprocessing as mp
    import numpy as np
    cores = max(1, min(16, os.cpu_count() or 1))
    npx = np.array([int(np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64)
                               * sb.img_w[sb.src_img_off[s]:sb.src_img_off[s + 1]])) for s in range(sb.n_sources)])
    pick = stratified_sample(npx, n, 161103408)
    sub = sb.subset(pick)
    order = np.argsort(-npx[pick], kind="stable")       # largest first, for the pool's balance
    out = [None] * len(pick)
    global _FIT_JOB
    _FIT_JOB = sub
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_one_thread) as pool:
        for done, (j, o) in enumerate(pool.imap_unordered(_indexed(_oracle_fit_worker), [int(j) for j in order])):
            out[j] = o
            log(f"oracle fit {done + 1}/{len(pick)}: source {pick[j]} ({npx[pick[j]]} px) {o[0]:.1f} s, "
                f"{o[2]} iterations, status {o[3]} ({time.perf_counter() - t0:.0f} s)")
    wall = time.perf_counter() - t0
    _FIT_JOB = None
    t_fit = np.array([o[0] for o in out])
    ref = np.array([o[1] for o in out])
    conv = np.array([o[3] == 0 for o in out])
    # each sampled source stands for its stratum (sb.n_sources / n sources)
    est_core_s = float(np.sum(t_fit)) * sb.n_sources / len(pick)
    est_conv = float(np.mean(conv)) * sb.n_sources

    def a22(gpu):
        got = np.asarray(gpu)[pick]
        return int(np.sum((np.abs(got - ref) <= 1e-5 * np.abs(ref)) | (got >= ref)))

    return {
        "value": est_conv / (est_core_s / cores), "unit": "converged sources/s", "cores": cores, "kind": "oracle",
        "sample": (f"complete oracle fits from the plain start of a size-stratified sample of {len(pick)} sources "
                   f"(one per equal-count stratum of the pixel-count order) on {cores} processes, {wall:.0f} s wall; "
                   f"the rate scales the sample's measured fit times to the {sb.n_sources}-source workload"),
        "measured_fits_per_s": len(pick) / wall, "host_cpu": host_cpu(),
        "oracle_iterations_mean": float(np.mean([o[2] for o in out])),
        "oracle_converged": int(np.sum(conv)),
        "a22_pass_plain_start": a22(gpu_plain_elbo), "a22_pass_headline_start": a22(gpu_head_elbo),
        "sources": len(pick),
    }


def oracle_fits_from(args, log):
    """The GPU fits saved by --save-fits (run with --host-generated) against complete oracle fits
    of a size-stratified sample, on this machine's cores: one JSON line."""
    import numpy as np
    import synth
    d = np.load(args.oracle_fits_from, allow_pickle=False)
    if not bool(d["host_generated"]):
        sys.exit("the saved fits are not of a host-generated workload (run the GPU side with --host-generated)")
    n = int(d["n_sources"])
    t = time.perf_counter()
    sb = synth.make_config(2, n_sources=n)
    log(f"workload rebuilt on the host: {sb.n_sources} sources, {sb.n_pixels} px ({time.perf_counter() - t:.0f} s)")
    res = oracle_fit_baseline(sb, args.cpu_baseline_fits or 200, d["plain_elbo"], d["head_elbo"], log)
    res["headline_start"] = str(d["head"])
    res["gpu_converged_status"] = {"plain": int(np.sum(d["plain_status"] == 0)), "headline": int(np.sum(d["head_status"] == 0))}
    print(json.dumps({"oracle_fits": res, "workload": f"batched uneven sources, {n} sources (host-generated pixels)"}),
          flush=True)


_SAMPLED_JOB = None   # (subset, keep, off, keep_prob, thetas): inherited by forked workers


def _sampled_oracle_worker(k):
    import numpy as np
    from oracle import model
    sub, keep, off, p, th = _SAMPLED_JOB
    imgs = []
    for j, img in enumerate(model.source_images(sub, k)):
        i = sub.src_img_off[k] + j
        w = np.repeat(keep[off[i]:off[i + 1]].astype(np.float64) / p, 8)[: img["h"]]
        imgs.append(dict(img, weights=np.repeat(w[:, None], img["w"], axis=1)))
    t0 = time.perf_counter()
    model.elbo(th[k], imgs, sub.prior, sub.profiles)
    return time.perf_counter() - t0


def sampled_cpu_baseline(sb, theta, keep_prob, seed, budget_s=20.0):
    """The oracle's subsampled estimate (value, gradient, Hessian) of random sources of the
    same workload with their own masks, timed on the host cores: source evaluations/s."""
    global _SAMPLED_JOB
    import multiprocessing as mp
    import numpy as np
    from synth.subsample import block_masks
    cores = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(161103407)
    order = rng.permutation(sb.n_sources)
    pick, est = [], 0.0
    for s in order:
        if est > budget_s * cores or len(pick) >= 4 * cores:
            break
        pick.append(int(s))
        est += 7e-5 * int(np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64) ** 2))
    sub = sb.subset(pick)
    keep, off = block_masks(sub.img_h, keep_prob, seed)
    _SAMPLED_JOB = (sub, keep, off, keep_prob, theta[pick])
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_one_thread) as pool:
        ts = pool.map(_sampled_oracle_worker, range(sub.n_sources), chunksize=1)
    wall = time.perf_counter() - t0
    _SAMPLED_JOB = None
    return {"value": len(pick) / sum(ts) * cores, "unit": "source evaluations/s", "cores": cores, "kind": "oracle",
            "sample": (f"{len(pick)} random sources of the same workload, one subsampled value+gradient+Hessian "
                       f"estimate each at the plain start, keep_prob {keep_prob}, on {cores} processes "
                       f"({wall:.1f} s wall)"),
            "host_cpu": host_cpu()}


_FIELD_JOB = None   # (subset, per-source neighbour dicts, thetas, n_full): inherited by forked workers


def _field_oracle_worker(k):
    sb, nbrs, thetas, n_full = _FIELD_JOB
    s, theta, nbr, full = k, thetas[k], nbrs[k], k < n_full
    from oracle import model
    imgs = model.source_images(sb, s, nbr=nbr)
    t0 = time.perf_counter()
    if full:
        model.elbo(theta, imgs, sb.prior, sb.profiles)
    t1 = time.perf_counter()
    v = model.elbo_value(theta, imgs, sb.prior, sb.profiles)
    t2 = time.perf_counter()
    npx = int(sum(int(im["h"]) * int(im["w"]) for im in imgs))
    return npx, t1 - t0, t2 - t1, v


def _field_host_subset(sb, pick, nbr):
    """Host copies of the picked sources' patches and of their neighbour arrays (image index
    of the subset -> (mean, var)), for the oracle."""
    import numpy as np
    import torch
    nm, nv, off = nbr
    sub = sb.subset(pick)
    out = []
    for k, s in enumerate(pick):
        i0, i1 = int(sb.src_img_off[s]), int(sb.src_img_off[s + 1])
        sizes = [int(sb.img_h[i]) * int(sb.img_w[i]) for i in range(i0, i1)]
        m = torch.cat([nm[int(off[i]):int(off[i]) + n] for i, n in zip(range(i0, i1), sizes)]).cpu().numpy()
        v = torch.cat([nv[int(off[i]):int(off[i]) + n] for i, n in zip(range(i0, i1), sizes)]).cpu().numpy()
        d, o = {}, 0
        for j, i in enumerate(range(i0, i1)):
            h, w = int(sb.img_h[i]), int(sb.img_w[i])
            d[int(sub.src_img_off[k]) + j] = (m[o:o + h * w].reshape(h, w), v[o:o + h * w].reshape(h, w))
            o += h * w
        out.append(d)
    return sub, out


def field_cpu_baseline(sb, theta, res, nbr, gpu_full_px_per_step, gpu_value_px_per_step, sources_per_step,
                       n_check, budget_s=15.0):
    """Oracle on the host cores for the crowded field, at the GPU's final estimates with the
    last sweep's neighbour arrays: value+gradient+Hessian and value evaluations of a few
    random sources, scaled to the step with the GPU's pixel-evaluation counts; and the
    ELBO of n_check random sources against the GPU's."""
    import multiprocessing as mp
    import numpy as np
    cores = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(161103406)
    check = [int(s) for s in rng.choice(sb.n_sources, size=min(n_check, sb.n_sources), replace=False)]
    npx = np.array([int(np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64)
                               * sb.img_w[sb.src_img_off[s]:sb.src_img_off[s + 1]])) for s in check])
    n_full, est = 0, 0.0
    while n_full < len(check) and est < budget_s * cores and n_full < 4 * cores:
        est += 7e-5 * npx[n_full]
        n_full += 1
    t = time.perf_counter()
    sub, nbrs = _field_host_subset(sb, check, nbr)
    t_copy = time.perf_counter() - t
    global _FIELD_JOB
    _FIELD_JOB = (sub, nbrs, theta[check], n_full)
    t0 = time.perf_counter()
    out = [None] * len(check)
    with mp.get_context("fork").Pool(cores, initializer=_one_thread) as pool:
        for done, (k, o) in enumerate(pool.imap_unordered(_indexed(_field_oracle_worker), range(len(check)))):
            out[k] = o
            if (done + 1) % 100 == 0 or done + 1 == len(check):
                print(f"[bench] oracle: {done + 1}/{len(check)} sources, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
    _FIELD_JOB = None
    wall = time.perf_counter() - t0
    px_full = sum(o[0] for o in out[:n_full])
    full_rate = px_full / sum(o[1] for o in out[:n_full]) * cores
    val_rate = sum(o[0] for o in out) / sum(o[2] for o in out) * cores
    step_s = gpu_full_px_per_step / full_rate + gpu_value_px_per_step / val_rate
    ref = np.array([o[3] for o in out])
    gpu = np.asarray(res["elbo"])[check]
    rel = np.abs(gpu - ref) / np.abs(ref)
    return {
        "value": sources_per_step / step_s, "unit": "sources/s", "cores": cores, "kind": "oracle",
        "sample": (f"{n_full} random sources ({px_full} px): one value+gradient+Hessian and one value evaluation "
                   f"each at the GPU's final estimates with the last sweep's neighbour arrays, on {cores} processes; "
                   f"scaled to the step with the pixel evaluations of the oracle's own iteration (the ELBO alone "
                   f"at trial points, value+gradient+Hessian at the start and at accepted points) counted in the "
                   f"GPU fits"),
        "full_pixel_evals_per_s": full_rate, "value_pixel_evals_per_s": val_rate,
        "full_pixel_evals_per_s_per_core": full_rate / cores, "value_pixel_evals_per_s_per_core": val_rate / cores,
        "host_cpu": host_cpu(),
        "elbo_check": {"sources": len(check), "max_rel_err": float(rel.max()), "median_rel_err": float(np.median(rel)),
                       "host_copy_s": t_copy, "oracle_wall_s": wall},
    }


def probe(args, ctx, log):
    """A short program for hardware-counter runs: the dominant kernels on the batched workload
    (launch shapes from the autotuner, as in the benchmark) and a plain copy of known size
    whose counters calibrate the byte counts."""
    import numpy as np
    import torch
    import synth
    from paper_1611_03404_amd import celeste as cb
    sb = synth.make_config(2, n_sources=args.sources, device="cuda")
    batch = cb.Batch.from_synth(sb)
    theta0 = np.zeros((sb.n_sources, 27))
    theta0[:, 0:2] = sb.u_cat
    th, _ = ctx.start(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
    tune = None if args.no_autotune else ctx.autotune(batch, th, cache_path=args.tune_cache)
    log(f"probe: {sb.n_sources} sources, {sb.n_pixels} px, autotune {tune}")
    for _ in range(2):
        ctx.elbo_eval(batch, th)
    for _ in range(2):
        ctx.elbo_eval(batch, th, want="value")
    n = 1 << 28   # 1 GiB of float32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"probe": True, "n_pixels": sb.n_pixels, "n_images": sb.n_images, "copy_bytes": 4 * n,
                      "autotune": tune}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sources", type=int, default=None, help="first N sources only (default: all 20,000)")
    ap.add_argument("--train-sources", type=int, default=200000, help="surrogate training sources")
    ap.add_argument("--epochs", type=int, default=20, help="surrogate training epochs")
    ap.add_argument("--no-surrogate", action="store_true", help="plain start only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--host-generated", action="store_true",
                    help="batched workload: draw the pixels with NumPy on the host (the same draws on any machine) "
                         "and move them to the device before the timed region, so that --oracle-fits-from can "
                         "rebuild the same workload without a GPU")
    ap.add_argument("--save-fits", default=None,
                    help="batched workload: write the final ELBO and status of every source, per start, to this "
                         ".npz file")
    ap.add_argument("--oracle-fits-from", default=None,
                    help="no GPU: rebuild the host-generated batched workload and fit a size-stratified sample of "
                         "--cpu-baseline-fits sources (default 200) with the oracle on the host cores, checking the "
                         "GPU fits saved by --save-fits against the oracle-converged ELBO")
    ap.add_argument("--cpu-baseline-fits", type=int, default=0,
                    help="batched workload: also fit a size-stratified sample of this many sources with the oracle "
                         "(complete fits on the host cores; 200 = 1%% of the workload takes about 15 minutes on 16 "
                         "cores) and check the GPU fits' final ELBO against the oracle-converged one")
    ap.add_argument("--workload", choices=("batched", "field", "sampled", "lbfgs", "twophase"), default="batched",
                    help="batched: 20,000 independent uneven sources (default); field: crowded 2048x2048 field, "
                         "100,000 sources, 5 bands x 4 epochs, 3 block-coordinate sweeps; sampled: pixel-subsampled "
                         "evaluations of the batched workload; lbfgs: L-BFGS against trust-region Newton from the "
                         "plain start on the 1,000 isolated sources, their bright variant and the batched workload")
    ap.add_argument("--lbfgs-max-iter", type=int, default=1000, help="lbfgs workload: L-BFGS iteration cap")
    ap.add_argument("--switch-rtol", type=float, default=1e-5,
                    help="twophase workload: predicted-gain tolerance of the subsampled early phase")
    ap.add_argument("--keep-prob", type=float, default=0.25,
                    help="sampled workload: probability of keeping each 8-row block of an image")
    ap.add_argument("--sweep-probs", default="1,0.5,0.25,0.1",
                    help="sampled workload: further keep probabilities timed besides --keep-prob")
    ap.add_argument("--sweeps", type=int, default=3, help="field workload: sweeps (the maximum with --until-rtol)")
    ap.add_argument("--until-rtol", type=float, default=None,
                    help="field workload: sweep until a sweep raises the joint ELBO by at most this fraction")
    ap.add_argument("--schedule", choices=("jacobi", "colour"), default="colour",
                    help="field workload: Jacobi sweeps (all sources see the previous sweep) or Gauss-Seidel "
                         "sweeps over conflict-free colours")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pixel-kernel launch shapes")
    ap.add_argument("--persistent", type=int, choices=range(-1, 17), default=None, metavar="-1..16",
                    help="trust-region fits: persistent pixel kernels with this many blocks per compute unit "
                         "drawing from the device work list, as many as the kernel keeps resident (-1), or one "
                         "block per work item (0); default: the library's (-1)")
    ap.add_argument("--trial-derivatives", type=int, choices=(0, 1), default=None,
                    help="trust-region fits: evaluate the gradient and Hessian at every trial point (1) or only at "
                         "accepted points (0); default: the library's (1)")
    ap.add_argument("--tr-cholesky", type=int, choices=(0, 1), default=None,
                    help="trust-region subproblem: interior Newton step by Cholesky first (1) or always the "
                         "eigendecomposition (0); default: the library's")
    ap.add_argument("--fp64-sums", type=int, choices=(0, 1), default=None,
                    help="value+gradient+Hessian kernel: every pixel term summed in FP64 (1) or FP32 lane sums "
                         "over up to 16 tile steps before FP64 (0); default: the library's")
    ap.add_argument("--field-chunk-px", type=int, default=4096,
                    help="crowded field, colour sweeps: pixels per work item after autotuning (0: the "
                         "autotuner's choice)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: read the launch shapes from it when it has an entry for this "
                         "device and workload, else time them and add one (runs that must share a launch "
                         "configuration, such as hardware-counter passes, pass the same file)")
    ap.add_argument("--probe", action="store_true",
                    help="counter-collection target: two value+gradient+Hessian and two value evaluations of the "
                         "batched workload at the plain start, then two 1 GiB device copies; no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (sources are "
              "independent: several GPUs would each fit a share of the source list)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from synth.surrogate import epoch_orders, init_params
    from paper_1611_03404_amd import celeste as cb
    from paper_1611_03404_amd import surrogate

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.oracle_fits_from:
        return oracle_fits_from(args, log)
    ctx = cb.Context(0)
    if args.persistent is not None:
        ctx.set_option(cb.OPT_PERSISTENT, args.persistent)
    if args.trial_derivatives is not None:
        ctx.set_option(cb.OPT_TRIAL_DERIVATIVES, args.trial_derivatives)
    if args.tr_cholesky is not None:
        ctx.set_option(cb.OPT_TR_CHOLESKY, args.tr_cholesky)
    if args.fp64_sums is not None:
        ctx.set_option(cb.OPT_FP64_SUMS, args.fp64_sums)
    if args.probe:
        return probe(args, ctx, log)
    if args.workload == "lbfgs":
        return lbfgs_bench(args, ctx, log)
    if args.workload == "twophase":
        return twophase_bench(args, ctx, log)
    if args.workload == "sampled":
        if not all(0.0 < float(x) <= 1.0 for x in args.sweep_probs.split(",") + [args.keep_prob] if x != ""):
            sys.exit("--keep-prob and --sweep-probs must be in (0, 1]")
        return sampled_bench(args, ctx, log)
    sur_info = None
    net = None
    if not args.no_surrogate:
        # offline: label the training sources by plain fits and train the network (not timed)
        t = time.perf_counter()
        tr = synth.make_config(3, n_sources=args.train_sources, device="cuda")
        trb = cb.Batch.from_synth(tr)
        net, sur_info = surrogate.train(ctx, trb, tr.u_cat, init_params(161103404),
                                        lambda n, e: epoch_orders(n, e, 161103405), epochs=args.epochs,
                                        minibatch=256, lr=1e-3, log=log)
        del trb, tr
        torch.cuda.empty_cache()
        sur_info["total_s"] = time.perf_counter() - t
        ctx.set_surrogate(net)

    if args.workload == "field":
        return field_bench(args, ctx, net, sur_info, log)
    t_gen = time.perf_counter()
    if args.host_generated:
        sb = synth.make_config(2, n_sources=args.sources)
        sb.pixels = torch.from_numpy(sb.pixels).to("cuda")
    else:
        sb = synth.make_config(2, n_sources=args.sources, device="cuda")
    torch.cuda.synchronize()
    log(f"workload: {sb.n_sources} sources, {sb.n_images} images, {sb.n_pixels} px "
        f"({time.perf_counter() - t_gen:.1f} s to generate{' on the host' if args.host_generated else ''})")
    batch = cb.Batch.from_synth(sb)
    theta0 = np.zeros((sb.n_sources, 27))
    theta0[:, 0:2] = sb.u_cat
    tune = None
    if not args.no_autotune:
        # launch and tile shapes of the pixel kernels, timed on a sample at the plain start (not timed)
        th_start, _ = ctx.start(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
        t = time.perf_counter()
        tune = ctx.autotune(batch, th_start, cache_path=args.tune_cache)
        tune["tune_s"] = time.perf_counter() - t
        log(f"autotune: {tune}")
    modes = [("plain", cb.INIT_PLAIN)] + ([] if net is None else [("surrogate", cb.INIT_SURROGATE)])
    runs = {}
    for name, mode in modes:
        opts = cb.default_opts(init_mode=mode)
        # timed steps: the production path (each iteration replays a captured HIP graph; the host
        # reads the active-source count every poll_every iterations)
        ctx.set_option(cb.OPT_PROFILE, 0)
        for w in range(args.warmup):
            t = time.perf_counter()
            ctx.batch_fit(batch, theta0, opts)
            log(f"{name} warmup {w}: {time.perf_counter() - t:.2f} s")
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        conv = 0
        for k in range(args.steps):
            ts = time.perf_counter()
            th, res = ctx.batch_fit(batch, theta0, opts)
            c = int(np.sum(res["status"] == cb.CONVERGED))
            conv += c
            log(f"{name} step {k}: {time.perf_counter() - ts:.2f} s, converged {c}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st_graph = ctx.stats()
        # one more step in profile mode (eager launches, HIP events around every kernel phase on
        # the library's stream, the stream drained at every host stage): the phase split and the
        # roofline's per-launch durations; its wall time is the eager path's
        ctx.set_option(cb.OPT_PROFILE, 1)
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        th_p, res_p = ctx.batch_fit(batch, theta0, opts)
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - tp
        st_prof = ctx.stats()
        ctx.set_option(cb.OPT_PROFILE, 0)
        same = bool(np.array_equal(res_p["elbo"], res["elbo"]) and np.array_equal(res_p["iters"], res["iters"]))
        log(f"{name} profiled step: {wall_p:.2f} s (graph path {wall / args.steps:.2f} s per step); "
            f"results identical to the graph path: {same}")
        runs[name] = dict(wall=wall, res=res, conv=conv, stats=st_graph, prof=st_prof, wall_prof=wall_p,
                          prof_same=same, theta=th)
    # ELBO tolerance rule against the best optimum either start reached
    best = np.max(np.stack([r["res"]["elbo"] for r in runs.values()]), axis=0)

    def at_tol(res):
        ok = (res["status"] == cb.CONVERGED) & (res["elbo"] >= best - 1e-5 * np.abs(best))
        return int(np.sum(ok))

    head = "surrogate" if net is not None else "plain"
    H = runs[head]
    st = H["stats"]
    wall = H["wall"]
    conv_tol = at_tol(H["res"]) * args.steps
    K = 3
    E, D = len(sb.profiles["exp"][0]), len(sb.profiles["dev"][0])
    f_full = flop_full_per_px_algorithmic(K, E, D)
    # roofline over the value+gradient+Hessian launches of the profiled steps of both starts
    # (HIP events on the library's stream around each launch)
    rl = {k: sum(r["prof"][k] for r in runs.values()) for k in ("ms_full", "full_px", "full_launches")}
    full_s = rl["ms_full"] / 1e3
    achieved = f_full * rl["full_px"] / full_s / 1e12 if full_s > 0 else 0.0
    hbm_bytes = 4.0 * rl["full_px"]
    traffic, counters = pmc_traffic(rl["full_px"] / max(1, rl["full_launches"]))
    res = H["res"]
    iters = res["iters"]
    status_counts = {name: int(np.sum(res["status"] == code)) for name, code in
                     (("converged", cb.CONVERGED), ("max_iter", cb.MAX_ITER), ("tr_collapsed", cb.TR_COLLAPSED),
                      ("nonfinite", cb.NONFINITE))}

    def summary(r):
        rr = r["res"]
        return {"converged_per_s": at_tol(rr) * args.steps / r["wall"], "ms_per_step": 1e3 * r["wall"] / args.steps,
                "ms_per_step_eager_profiled": 1e3 * r["wall_prof"], "profiled_results_identical": r["prof_same"],
                "converged_status": int(np.sum(rr["status"] == cb.CONVERGED)), "converged_at_tol": at_tol(rr),
                "iterations_mean": float(np.mean(rr["iters"])), "full_evals_mean": float(np.mean(rr["n_full_evals"])),
                "fallback_rate": float(np.mean((rr["flags"] & cb.FLAG_FALLBACK_USED) != 0)),
                "pixel_evals_per_s": r["stats"]["full_px"] / r["wall"]}

    out = {
        "metric": "converged sources/s at ELBO rel err<=1e-5 (surrogate start with plain fallback); pixel-evals/s",
        "value": conv_tol / wall,
        "unit": "converged sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "ms_per_step_eager_profiled": 1e3 * H["wall_prof"],
        "timed_path": "HIP-graph replay of each iteration, active count read every 4 iterations (profile mode off)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_str(args, network=True),
        "data": "synthetic",
        "config": {"workload": "batched uneven sources: 20,000 sources, side log-uniform 15-121 px, "
                               "5 bands x 1-10 epochs, per-epoch PSF and sky" if args.sources is None else
                   f"first {sb.n_sources} sources of the batched-uneven workload",
                   "n_sources": sb.n_sources, "n_images": sb.n_images, "n_pixels": sb.n_pixels,
                   "start": head, "max_iter": 50},
        "tolerance_rule": "status converged and ELBO >= best of the plain-start and surrogate-start optima - 1e-5 |L|",
        "pixel_evals_per_s": st["full_px"] / wall,
        "value_pixel_evals_per_s": st["value_px"] / wall,
        "kernel_pixel_evals_per_s": rl["full_px"] / full_s if full_s > 0 else None,
        "iterations_mean": float(np.mean(iters)), "iterations_max": int(np.max(iters)),
        "iterations_hist": np.bincount(iters, minlength=52).tolist(),
        "status": status_counts,
        "phase_ms_per_step": {k[3:]: v for k, v in H["prof"].items() if k.startswith("ms_")},
        "tr_subproblems": {"interior_cholesky": st["tr_interior"], "boundary_cholesky": st["tr_boundary"],
                           "eigendecomposition": st["tr_eigen"], "jacobi_sweeps": st["tr_sweeps"],
                           "jacobi_sweep_cap": st["tr_sweep_cap"], "newton_steps": st["tr_newton_steps"]},
        "fit_grid_blocks": st["fit_grid_blocks"],
        "phase_source": "the profiled step (eager launches with HIP events), one per start after the timed steps",
        "starts": {name: summary(r) for name, r in runs.items()},
        "autotune": tune,
        "surrogate_training": None if sur_info is None else
        {k: v for k, v in sur_info.items() if k not in ("psi_mean", "psi_std")},
        "roofline": {
            "kernel": "k_eval_full (value+gradient+Hessian pixel kernel)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_unpacked_peak": achieved / PEAK_FP32_UNPACKED_TFLOPS,
            "flop_per_pixel_eval": f_full,
            "flop_per_pixel_eval_counted": flop_full_per_px(K, E, D),
            "avg_launch_ms": rl["ms_full"] / max(1, rl["full_launches"]),
            "launches": rl["full_launches"],
            "over": "all value+gradient+Hessian launches of the profiled step of each start (same kernels, "
                    "launch shapes and work as the timed graph replays)",
            "hbm_algorithmic_GBs": hbm_bytes / full_s / 1e9 if full_s > 0 else None,
            "traffic": traffic,
            "counters": counters,
        },
    }
    out["lr_covariance"] = lr_measure(ctx, batch, runs["plain"]["theta"], sb, log)
    if "plain" in runs and net is not None:
        out["surrogate_gain"] = out["starts"]["surrogate"]["converged_per_s"] / out["starts"]["plain"]["converged_per_s"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        th_fit = H["theta"]
        th_np = th_fit.cpu().numpy() if hasattr(th_fit, "cpu") else np.asarray(th_fit)

        def gpu_eval(pick):
            # the GPU's ELBO, gradient and Hessian at the fitted parameters of the picked sources
            return ctx.elbo_eval(cb.Batch.from_synth(sb.subset(pick)), th_np[pick])

        full_o, value_o = oracle_pattern_px(st)
        out["cpu_baseline"] = cpu_baseline(sb, th_np, gpu_eval, full_o / args.steps, value_o / args.steps,
                                           conv_tol / args.steps)
    if args.save_fits:
        np.savez(args.save_fits, n_sources=sb.n_sources, host_generated=bool(args.host_generated),
                 plain_elbo=runs["plain"]["res"]["elbo"], plain_status=runs["plain"]["res"]["status"],
                 head_elbo=H["res"]["elbo"], head_status=H["res"]["status"], head=head)
    if args.cpu_baseline_fits:
        log(f"oracle fits of a size-stratified sample of {args.cpu_baseline_fits} sources ...")
        out["cpu_baseline_fits"] = oracle_fit_baseline(sb, args.cpu_baseline_fits, runs["plain"]["res"]["elbo"],
                                                       H["res"]["elbo"], log)
    print(json.dumps(out), flush=True)
    if net is not None:
        ctx.set_surrogate(None)
        net.close()
    ctx.close()


def sampled_bench(args, ctx, log):
    """Pixel-subsampled evaluation: one step = one subsampled ELBO + gradient + Hessian estimate
    of every source of the batched-uneven workload at the plain start, 8-row blocks kept with
    probability keep_prob (fresh seeded masks, uploaded by each call), timed for several
    keep_prob values; the headline is the one given by --keep-prob."""
    import numpy as np
    import torch

    import synth
    from synth.subsample import block_masks
    from paper_1611_03404_amd import celeste as cb
    sb = synth.make_config(2, n_sources=args.sources, device="cuda")
    batch = cb.Batch.from_synth(sb)
    theta0 = np.zeros((sb.n_sources, 27))
    theta0[:, 0:2] = sb.u_cat
    th, _ = ctx.start(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
    tune = None if args.no_autotune else ctx.autotune(batch, th, cache_path=args.tune_cache)
    log(f"sampled: {sb.n_sources} sources, {sb.n_pixels} px, autotune {tune}")
    ctx.set_option(cb.OPT_PROFILE, 1)
    w = sb.img_w.astype(np.int64)
    h = sb.img_h.astype(np.int64)
    K = 3
    E, D = len(sb.profiles["exp"][0]), len(sb.profiles["dev"][0])
    f_full = flop_full_per_px_algorithmic(K, E, D)   # the roofline's figure, as for the batched workload
    probs = sorted(set([float(x) for x in args.sweep_probs.split(",") if x] + [args.keep_prob]), reverse=True)
    sweep = {}
    for i, p in enumerate(probs):
        masks = [block_masks(sb.img_h, p, 161103410 + 97 * i + k) for k in range(args.warmup + args.steps)]
        img_of = np.repeat(np.arange(len(h)), (h + 7) // 8)
        blk_px = np.minimum(8, h[img_of] - 8 * (np.arange(img_of.size) - np.repeat(masks[0][1][:-1], (h + 7) // 8)))
        blk_px *= w[img_of]     # pixels of each 8-row block (the last block of an image may be shorter)
        kept_px = [int(np.sum(blk_px[keep != 0])) for keep, _ in masks]
        for k in range(args.warmup):
            ctx.elbo_eval_sampled(batch, th, masks[k][0], masks[k][1], p)
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            ctx.elbo_eval_sampled(batch, th, masks[k][0], masks[k][1], p)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stats()
        px = sum(kept_px[args.warmup:])
        kern_s = st["ms_full"] / 1e3
        sweep[p] = {"keep_prob": p, "ms_per_eval": 1e3 * wall / args.steps,
                    "source_evals_per_s": sb.n_sources * args.steps / wall,
                    "kept_pixel_fraction": px / (args.steps * sb.n_pixels),
                    "kernel_ms_per_eval": st["ms_full"] / args.steps,
                    "kernel_kept_pixel_evals_per_s": px / kern_s if kern_s > 0 else None,
                    "kernel_tflops": f_full * px / kern_s / 1e12 if kern_s > 0 else None, "_px": px,
                    "_kern_s": kern_s}
        log(f"keep_prob {p}: {sweep[p]['ms_per_eval']:.2f} ms/eval, kernel {sweep[p]['kernel_ms_per_eval']:.2f} ms")
    head = sweep[args.keep_prob]
    achieved = head["kernel_tflops"]
    out = {
        "metric": "pixel-subsampled ELBO+gradient+Hessian source evaluations/s",
        "value": head["source_evals_per_s"],
        "unit": "source evaluations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_eval"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_str(args, network=False),
        "data": "synthetic",
        "config": {"workload": f"batched uneven sources ({sb.n_sources} sources, {sb.n_pixels} px) at the plain "
                               f"start, 8-row blocks kept with probability {args.keep_prob}",
                   "keep_prob": args.keep_prob, "n_sources": sb.n_sources, "n_pixels": sb.n_pixels},
        "speedup_vs_full_eval": head["source_evals_per_s"] / sweep[1.0]["source_evals_per_s"] if 1.0 in sweep else None,
        "sweep": [{k: v for k, v in r.items() if not k.startswith("_")} for r in sweep.values()],
        "autotune": tune,
        "roofline": {
            "kernel": "k_eval_full (value+gradient+Hessian pixel kernel), kept pixels only",
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS if achieved else None,
            "flop_per_pixel_eval": f_full,
            "flop_per_pixel_eval_counted": flop_full_per_px(K, E, D),
            "avg_launch_ms": head["kernel_ms_per_eval"],
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = sampled_cpu_baseline(sb, th.cpu().numpy() if hasattr(th, "cpu") else th,
                                                   args.keep_prob, 161103408)
    print(json.dumps(out), flush=True)
    ctx.close()


def lr_measure(ctx, batch, theta, sb, log):
    """Linear-response covariance of every source at its plain-start fit (box centres = catalog
    positions, as in that fit), outside the timed steps: the call's wall time, the covariance
    kernel's HIP-event time, statuses, and how far linear response moves the variances."""
    import numpy as np
    import torch
    from paper_1611_03404_amd import celeste as cb
    S = sb.n_sources
    u0 = torch.from_numpy(np.asarray(sb.u_cat, dtype=np.float64)).cuda()
    ctx.set_option(cb.OPT_PROFILE, 1)     # HIP events around the evaluation and the covariance kernel
    ctx.stats(reset=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    cov, st = ctx.lr_covariance(batch, theta, u0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    s2 = ctx.stats()
    ctx.set_option(cb.OPT_PROFILE, 0)
    c = cov.cpu().numpy()
    th = theta.cpu().numpy() if hasattr(theta, "cpu") else np.asarray(theta)
    ok = st == 0
    idx = np.arange(S)
    star = th[:, 2] >= 0.5
    r1, r2 = np.where(star, 7, 8), np.where(star, 9, 10)
    ratio = c[idx, r1, r1] / th[idx, r2]
    # as executed: Cholesky n^3/3, inverse of L n^3/3, L^-T L^-1 over all entries 2n^3/3, scalings 3n^2
    flop = 4 * 27 ** 3 // 3 + 3 * 27 * 27
    kern_s = s2["ms_lr"] / 1e3
    info = {
        "ms_call": 1e3 * wall, "kernel_ms": s2["ms_lr"], "eval_kernel_ms": s2["ms_full"],
        "sources": S, "status_ok": int(ok.sum()), "not_positive_definite": int(np.sum(st == 1)),
        "nonfinite": int(np.sum(st == 2)),
        "median_lr_over_mean_field_var_log_r": float(np.median(ratio[ok])),
        "p90_lr_over_mean_field_var_log_r": float(np.quantile(ratio[ok], 0.9)),
        "median_lr_sd_position_px": float(np.median(np.sqrt(c[ok, 0, 0]))),
        "kernel_gflops": flop * S / kern_s / 1e9 if kern_s > 0 else None,
        "flop_per_source": flop,
        "u0": "catalog positions (the plain-start fits' box centres)",
    }
    log(f"lr covariance: {info}")
    return info


def twophase_bench(args, ctx, log):
    """Trust-region fits of the batched-uneven workload from the plain start, plain against a
    pixel-subsampled early phase (each source fits the subsampled ELBO estimate until its model's
    predicted gain falls to --switch-rtol max(1, |L|), then the full ELBO): wall time per fit
    (graph path, steps of each variant), iterations, pixel evaluations and sources converged at
    the tolerance rule against the better optimum of the variants, for keep probabilities
    --sweep-probs below 1 (a fresh seeded mask per step)."""
    import numpy as np
    import torch

    import synth
    from synth.subsample import block_masks
    from paper_1611_03404_amd import celeste as cb
    sb = synth.make_config(2, n_sources=args.sources, device="cuda")
    batch = cb.Batch.from_synth(sb)
    theta0 = np.zeros((sb.n_sources, 27))
    theta0[:, 0:2] = sb.u_cat
    th_start, _ = ctx.start(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
    tune = None if args.no_autotune else ctx.autotune(batch, th_start, cache_path=args.tune_cache)
    opts = cb.default_opts(init_mode=cb.INIT_PLAIN)
    probs = sorted({float(x) for x in args.sweep_probs.split(",") if x and float(x) < 1.0}, reverse=True)
    variants = [("plain", None)] + [(f"p={p}", p) for p in probs]
    runs = {}
    for name, p in variants:
        masks = [block_masks(sb.img_h, p, 161103420 + k) for k in range(args.warmup + args.steps)] if p else None
        for w in range(args.warmup):
            if p:
                ctx.batch_fit_sampled(batch, theta0, masks[w][0], masks[w][1], p, args.switch_rtol, opts)
            else:
                ctx.batch_fit(batch, theta0, opts)
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            if p:
                keep, off = masks[args.warmup + k]
                th, res = ctx.batch_fit_sampled(batch, theta0, keep, off, p, args.switch_rtol, opts)
            else:
                th, res = ctx.batch_fit(batch, theta0, opts)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        runs[name] = dict(res=res, wall=wall, stats=ctx.stats())
        log(f"twophase {name}: {wall:.3f} s per fit, iterations mean {np.mean(res['iters']):.2f}")
    best = np.max(np.stack([r["res"]["elbo"] for r in runs.values()]), axis=0)
    out = {"metric": "converged sources/s, trust-region fits with and without a pixel-subsampled early phase",
           "workload": f"batched uneven sources ({sb.n_sources}), plain start", "switch_rtol": args.switch_rtol,
           "steps": args.steps, "autotune": tune, "variants": {}}
    for name, r in runs.items():
        res, st = r["res"], r["stats"]
        ok = (res["status"] == cb.CONVERGED) & (res["elbo"] >= best - 1e-5 * np.abs(best))
        out["variants"][name] = {
            "ms_per_fit": 1e3 * r["wall"], "converged_at_tol": int(ok.sum()),
            "converged_per_s": int(ok.sum()) / r["wall"], "converged_status": int(np.sum(res["status"] == cb.CONVERGED)),
            "iterations_mean": float(np.mean(res["iters"])), "iterations_max": int(np.max(res["iters"])),
            "full_evals_mean": float(np.mean(res["n_full_evals"])),
            "full_pixel_evals_per_fit": st["full_px"] / args.steps, "value_pixel_evals_per_fit": st["value_px"] / args.steps,
            "elbo_shortfall_vs_best_max_rel": float(np.max((best - res["elbo"]) / np.abs(best))),
        }
    print(json.dumps(out), flush=True)
    ctx.close()


def lbfgs_bench(args, ctx, log):
    """The optimiser ablation of section III-B: L-BFGS (the earlier Celeste optimiser) against
    trust-region Newton, both from the plain start on the same sources and pixel sums, on the
    1,000 isolated sources of config 1, their bright variant (100 counts/nMgy) and the 20,000
    batched-uneven sources.  Per workload and method: wall time of one fit of all sources,
    iterations (mean, percentiles, max, histogram), gradient/Hessian and value evaluations,
    statuses, and sources converged at the tolerance rule (status converged and ELBO within
    1e-5 |L| of the better of the two methods' optima)."""
    import numpy as np
    import torch

    import synth
    from paper_1611_03404_amd import celeste as cb
    out = {"metric": "converged sources/s, L-BFGS vs trust-region Newton (plain start)", "workloads": {}}
    loads = [("config1", dict(k=1)), ("config1_bright", dict(k=1, bright=True)),
             ("batched_uneven", dict(k=2, n_sources=args.sources))]
    for name, kw in loads:
        sb = synth.make_config(kw.pop("k"), device="cuda", **kw)
        batch = cb.Batch.from_synth(sb)
        theta0 = np.zeros((sb.n_sources, 27))
        theta0[:, 0:2] = sb.u_cat
        th_start, _ = ctx.start(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
        tune = None if args.no_autotune else ctx.autotune(batch, th_start, cache_path=args.tune_cache)
        runs = {}
        for meth in ("trust_region", "lbfgs"):
            ctx.stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if meth == "trust_region":
                th, res = ctx.batch_fit(batch, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
            else:
                th, res = ctx.lbfgs_fit(batch, theta0, cb.default_lbfgs_opts(init_mode=cb.INIT_PLAIN,
                                                                             max_iter=args.lbfgs_max_iter))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            runs[meth] = dict(res=res, wall=wall, stats=ctx.stats())
            log(f"{name} {meth}: {wall:.2f} s, iterations mean {np.mean(res['iters']):.1f} max {np.max(res['iters'])}")
        best = np.maximum(runs["trust_region"]["res"]["elbo"], runs["lbfgs"]["res"]["elbo"])
        w = {"n_sources": sb.n_sources, "n_pixels": sb.n_pixels, "autotune": tune, "methods": {}}
        for meth, r in runs.items():
            res, st = r["res"], r["stats"]
            it = res["iters"]
            ok = (res["status"] == cb.CONVERGED) & (res["elbo"] >= best - 1e-5 * np.abs(best))
            edges = [0, 10, 20, 50, 100, 200, 500, 1000, 2000, 10 ** 9]
            w["methods"][meth] = {
                "wall_s": r["wall"], "converged_at_tol": int(ok.sum()), "converged_per_s": int(ok.sum()) / r["wall"],
                "status": {k: int(np.sum(res["status"] == c)) for k, c in
                           (("converged", cb.CONVERGED), ("max_iter", cb.MAX_ITER), ("tr_collapsed", cb.TR_COLLAPSED),
                            ("nonfinite", cb.NONFINITE), ("line_search_failed", cb.LINE_SEARCH_FAILED))},
                "iterations": {"mean": float(np.mean(it)), "p50": float(np.percentile(it, 50)),
                               "p90": float(np.percentile(it, 90)), "p99": float(np.percentile(it, 99)),
                               "max": int(np.max(it)), "over_50": int(np.sum(it > 50)),
                               "hist_edges": edges[:-1], "hist": np.histogram(it, bins=edges)[0].tolist()},
                "derivative_evals_mean": float(np.mean(res["n_full_evals"])),
                "pixel_evals": {"value_gradient_hessian": st["full_px"], "value_gradient": st["grad_px"],
                                "value": st["value_px"]},
                "loop_steps": st["iterations"],
                "elbo_shortfall_vs_best": {"median_rel": float(np.median((best - res["elbo"]) / np.abs(best))),
                                           "max_rel": float(np.max((best - res["elbo"]) / np.abs(best)))},
            }
        w["speedup_trust_region_over_lbfgs"] = (w["methods"]["trust_region"]["converged_per_s"]
                                                / max(1e-12, w["methods"]["lbfgs"]["converged_per_s"]))
        out["workloads"][name] = w
        del batch, sb
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    ctx.close()


def field_bench(args, ctx, net, sur_info, log):
    """Crowded field: one step = start + `sweeps` block-coordinate sweeps over all sources."""
    import numpy as np
    import torch

    import synth
    from paper_1611_03404_amd import celeste as cb
    from paper_1611_03404_amd import field

    t_gen = time.perf_counter()
    n = args.sources or 100000
    sf = synth.make_field(n_sources=n, size=2048, epochs=4, device="cuda")
    torch.cuda.synchronize()
    sb = sf.batch
    log(f"field: {sb.n_sources} sources, {sf.n_fields} fields of {sf.H}x{sf.W}, {sb.n_images} patches, "
        f"{sb.n_pixels} patch px ({time.perf_counter() - t_gen:.1f} s to generate)")
    meta = (sf.img_field, sf.n_fields, sf.H, sf.W)
    mode = cb.INIT_SURROGATE if net is not None else cb.INIT_PLAIN
    tune = None
    if not args.no_autotune:
        b0 = cb.Batch.from_synth(sb)
        th0 = np.zeros((sb.n_sources, 27))
        th0[:, 0:2] = sb.u_cat
        th_start, _ = ctx.start(b0, th0, cb.default_opts(init_mode=cb.INIT_PLAIN))
        tune = ctx.autotune(b0, th_start, cache_path=args.tune_cache)
        # the sweep's launches hold one colour's few hundred sources (fewer as they converge), where
        # the tuner's single launch over its whole sample does not reflect the tail of the
        # persistent grid: keep the library's 4,096-pixel work items (several per block) there
        if args.schedule == "colour" and args.field_chunk_px > 0:
            ctx.set_option(cb.OPT_CHUNK_PX, args.field_chunk_px)
            tune["chunk_px"] = args.field_chunk_px
        log(f"autotune: {tune}")
        del b0
    for w in range(args.warmup):
        t = time.perf_counter()
        field.bca(ctx, sb, meta, sweeps=1, start_mode=mode, schedule=args.schedule)
        log(f"warmup {w}: {time.perf_counter() - t:.2f} s")
    ctx.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv = 0
    info = res = None
    for k in range(args.steps):
        theta, res, info = field.bca(ctx, sb, meta, sweeps=args.sweeps, start_mode=mode, log=log,
                                     schedule=args.schedule, field_pixels=sf.fields, field_sky=sf.field_sky,
                                     until_rtol=args.until_rtol)
        conv += int(np.sum(res["status"] == cb.CONVERGED))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    # one more sweep in profile mode (eager launches, HIP events around every kernel phase): the
    # roofline's per-launch durations and the phase split of the fits
    ctx.set_option(cb.OPT_PROFILE, 1)
    ctx.stats(reset=True)
    tp = time.perf_counter()
    field.bca(ctx, sb, meta, sweeps=1, start_mode=mode, schedule=args.schedule)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - tp
    st_p = ctx.stats()
    ctx.set_option(cb.OPT_PROFILE, 0)
    log(f"profiled sweep: {wall_p:.2f} s")
    f_full = flop_full_per_px_algorithmic(3, len(sb.profiles["exp"][0]), len(sb.profiles["dev"][0]))
    full_s = st_p["ms_full"] / 1e3
    achieved = f_full * st_p["full_px"] / full_s / 1e12 if full_s > 0 else 0.0
    out = {
        "metric": "field-level sources/s (crowded field, block coordinate ascent); pixel-evals/s",
        "value": sb.n_sources * args.steps / wall,
        "unit": "sources/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_str(args, network=True), "data": "synthetic",
        "config": {"workload": f"crowded field {sf.W}x{sf.H} px, {sf.n_fields} images (5 bands x 4 epochs), "
                               f"{sb.n_sources} sources, "
                               + (f"{args.sweeps} " if args.until_rtol is None else
                                  f"up to {args.sweeps} (until a sweep gains <= {args.until_rtol:g} of the joint ELBO) ")
                               + f"{'Jacobi' if args.schedule == 'jacobi' else 'colour (Gauss-Seidel)'} sweeps",
                   "n_patch_pixels": sb.n_pixels, "start": "surrogate" if net is not None else "plain"},
        "converged_last_sweep": int(np.sum(res["status"] == cb.CONVERGED)),
        "schedule": args.schedule, "start_joint_elbo": info["start_joint_elbo"], "stopped": info["stopped"],
        "until_rtol": args.until_rtol,
        "autotune": tune,
        "sweeps": info["history"], "timings_s_last_step": dict(info["timings"]),
        "pixel_evals_per_s": st["full_px"] / wall,
        "tr_subproblems": {"interior_cholesky": st["tr_interior"], "boundary_cholesky": st["tr_boundary"],
                           "eigendecomposition": st["tr_eigen"], "jacobi_sweeps": st["tr_sweeps"],
                           "jacobi_sweep_cap": st["tr_sweep_cap"], "newton_steps": st["tr_newton_steps"]},
        "fit_grid_blocks": st["fit_grid_blocks"],
        "profiled_sweep": {"s": wall_p, "phase_ms": {k[3:]: v for k, v in st_p.items() if k.startswith("ms_")},
                           "kernel_pixel_evals_per_s": st_p["full_px"] / full_s if full_s > 0 else None},
        "roofline": {"kernel": "k_eval_full (value+gradient+Hessian pixel kernel)", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "frac_of_unpacked_peak": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                     "flop_per_pixel_eval_algorithmic": f_full,
                     "avg_launch_ms": st_p["ms_full"] / max(1, st_p["full_launches"]),
                     "launches": st_p["full_launches"],
                     "over": "the value+gradient+Hessian launches of one profiled colour sweep after the timed steps",
                     "traffic": None},   # counters were taken on the batched workload only
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) and ELBO check on a 1% sample ...")
        full_o, value_o = oracle_pattern_px(st)
        out["cpu_baseline"] = field_cpu_baseline(sb, theta.cpu().numpy(), res, info["nbr"],
                                                 full_o / args.steps, value_o / args.steps,
                                                 sb.n_sources, n_check=max(1, sb.n_sources // 100))
    print(json.dumps(out), flush=True)
    if net is not None:
        ctx.set_surrogate(None)
        net.close()
    ctx.close()


if __name__ == "__main__":
    main()
