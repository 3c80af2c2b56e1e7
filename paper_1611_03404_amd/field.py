"""Block coordinate ascent over a crowded field (argument marshalling around libceleste).

Section III-B optimises each source with the others held fixed.  In a crowded field the
fixed neighbours enter each source's pixel rates: the library renders all sources' expected
counts and variances into the field images, forms each source's neighbour arrays (field
totals minus its own contribution) and fits sources with those arrays held fixed.

Two schedules of a sweep:
- "jacobi": every source of the sweep sees the previous sweep's estimates; all sources are
  fitted in one batched call.
- "colour": Gauss-Seidel over conflict-free colours (celeste_colour_sources): the sources of
  one colour share no pixel, so fitting them together with everything else held fixed is an
  exact block step on the joint ELBO; the field images are moved to the new estimates
  (celeste_update_fields) before the next colour reads its neighbour arrays.
"""
from __future__ import annotations

import time

import numpy as np

from . import celeste as cb


def bca(ctx, batch_arrays, fields_meta, sweeps=3, start_mode=cb.INIT_SURROGATE, log=None, schedule="colour",
        field_pixels=None, field_sky=None, until_rtol=None):
    """batch_arrays: object with the SoA fields of Batch.from_synth (device pixels);
    fields_meta: (img_field, n_fields, height, width).  With field_pixels (device, the field
    images) and field_sky, the joint ELBO of the field is evaluated at the start and after every
    sweep (history[k]["joint_elbo"]).  With until_rtol, sweeps run (at most `sweeps` of them)
    until one raises the joint ELBO by no more than until_rtol * |joint ELBO|: a stationary point
    of block coordinate ascent.  Returns theta, last results, dict(timings, history, nbr, fields,
    start_joint_elbo, stopped)."""
    import torch
    if schedule not in ("jacobi", "colour"):
        raise ValueError("schedule must be 'jacobi' or 'colour'")
    if until_rtol is not None and field_pixels is None:
        raise ValueError("until_rtol needs field_pixels and field_sky (the joint ELBO)")
    img_field, n_fields, H, W = fields_meta
    img_field = np.asarray(img_field, dtype=np.int32)
    base = cb.Batch.from_synth(batch_arrays)
    S = base.n_sources
    th0 = np.zeros((S, cb.NP))
    th0[:, 0:2] = batch_arrays.u_cat
    timings = {"start": 0.0, "colour": 0.0, "render": 0.0, "neighbours": 0.0, "fit": 0.0, "update": 0.0,
               "joint_elbo": 0.0}
    torch.cuda.synchronize()
    t = time.perf_counter()
    theta, _ = ctx.start(base, th0, cb.default_opts(init_mode=start_mode))
    timings["start"] = time.perf_counter() - t
    npx = batch_arrays.img_h.astype(np.int64) * batch_arrays.img_w
    nbr_off = np.concatenate([[0], np.cumsum(npx)[:-1]]).astype(np.int64)
    dev = base.torch_device
    nbr_mean = torch.empty(int(npx.sum()), dtype=torch.float32, device=dev)
    nbr_var = torch.empty(int(npx.sum()), dtype=torch.float32, device=dev)
    fields = (torch.empty(n_fields * H * W, dtype=torch.float32, device=dev),
              torch.empty(n_fields * H * W, dtype=torch.float32, device=dev))
    meta = (img_field, n_fields, H, W)
    groups = None
    if schedule == "colour":
        t = time.perf_counter()
        col, nc = cb.colour_sources(base)
        order = np.argsort(col, kind="stable")
        bounds = np.searchsorted(col[order], np.arange(nc + 1))
        groups = []
        for c in range(nc):
            g = order[bounds[c]:bounds[c + 1]]
            sub, img_idx = base.subset(g)
            groups.append((torch.as_tensor(g, device=dev), sub, img_idx))
        timings["colour"] = time.perf_counter() - t
        if log:
            log(f"colouring: {nc} colours, {timings['colour']:.2f} s")

    def joint(k):
        if field_pixels is None:
            return None
        t = time.perf_counter()
        v = ctx.field_elbo(base, theta, img_field, n_fields, H, W, fields, field_pixels, field_sky)
        timings["joint_elbo"] += time.perf_counter() - t
        return v

    res = {"elbo": np.zeros(S), "status": np.zeros(S, np.int32), "iters": np.zeros(S, np.int32),
           "n_full_evals": np.zeros(S, np.int32), "flags": np.zeros(S, np.int32),
           "n_accepted": np.zeros(S, np.int32)}
    history = []
    t = time.perf_counter()
    ctx.render_fields(base, theta, img_field, n_fields, H, W, out=fields)
    timings["render"] += time.perf_counter() - t
    start_elbo = joint(-1)
    for k in range(sweeps):
        if k > 0:
            t = time.perf_counter()
            ctx.render_fields(base, theta, img_field, n_fields, H, W, out=fields)
            timings["render"] += time.perf_counter() - t
        fit_s = 0.0
        if schedule == "jacobi":
            t = time.perf_counter()
            ctx.neighbour_arrays(base, theta, img_field, n_fields, H, W, fields, nbr_off, nbr_mean, nbr_var)
            t2 = time.perf_counter()
            bk = base.with_nbr(nbr_mean, nbr_var, nbr_off)
            theta, r = ctx.batch_fit(bk, theta, cb.default_opts(init_mode=cb.INIT_AS_GIVEN))
            t3 = time.perf_counter()
            timings["neighbours"] += t2 - t
            fit_s = t3 - t2
            for name in res:
                res[name] = np.asarray(r[name])
        else:
            for g, sub, img_idx in groups:
                th_c = theta[g]
                t = time.perf_counter()
                ctx.neighbour_arrays(sub, th_c, img_field[img_idx], n_fields, H, W, fields, nbr_off[img_idx],
                                     nbr_mean, nbr_var)
                t2 = time.perf_counter()
                th_new, r = ctx.batch_fit(sub.with_nbr(nbr_mean, nbr_var, nbr_off[img_idx]), th_c,
                                          cb.default_opts(init_mode=cb.INIT_AS_GIVEN))
                t3 = time.perf_counter()
                ctx.update_fields(sub, th_c, th_new, img_field[img_idx], n_fields, H, W, fields)
                theta[g] = th_new
                t4 = time.perf_counter()
                timings["neighbours"] += t2 - t
                fit_s += t3 - t2
                timings["update"] += t4 - t3
                gi = g.cpu().numpy()
                for name in res:
                    res[name][gi] = r[name]
        timings["fit"] += fit_s
        h = dict(sweep=k, converged=int(np.sum(res["status"] == cb.CONVERGED)),
                 iters_mean=float(np.mean(res["iters"])), elbo_sum=float(np.sum(res["elbo"])), fit_s=fit_s)
        if field_pixels is not None:
            t = time.perf_counter()
            ctx.render_fields(base, theta, img_field, n_fields, H, W, out=fields)
            timings["render"] += time.perf_counter() - t
            h["joint_elbo"] = joint(k)
        history.append(h)
        if log:
            log(f"sweep {k} ({schedule}): fit {fit_s:.2f} s, converged {h['converged']}, "
                f"iterations {h['iters_mean']:.2f}" +
                (f", joint ELBO {h['joint_elbo']:.6e}" if "joint_elbo" in h else ""))
        if until_rtol is not None:
            prev = start_elbo if k == 0 else history[-2]["joint_elbo"]
            if h["joint_elbo"] - prev <= until_rtol * abs(h["joint_elbo"]):
                stopped = "stationary"
                break
    else:
        stopped = "sweeps"
    return theta, res, dict(timings=timings, history=history, nbr=(nbr_mean, nbr_var, nbr_off), fields=fields,
                            start_joint_elbo=start_elbo, stopped=stopped)
