"""Block coordinate ascent over a crowded field (argument marshalling around libceleste).

Section III-B optimises each source with the others held fixed.  In a crowded field the
fixed neighbours enter each source's pixel rates: every sweep renders all sources' expected
counts and variances into the field images at the current estimates, forms each source's
neighbour arrays (field totals minus its own contribution) and fits all sources at once with
those arrays held fixed (Jacobi: every source sees the previous sweep's estimates).
"""
from __future__ import annotations

import time

import numpy as np

from . import celeste as cb


def bca(ctx, batch_arrays, fields_meta, sweeps=3, start_mode=cb.INIT_SURROGATE, log=None):
    """batch_arrays: object with the SoA fields of Batch.from_synth (device pixels);
    fields_meta: (img_field, n_fields, height, width).  Returns theta, last results, timings."""
    import torch
    img_field, n_fields, H, W = fields_meta
    base = cb.Batch.from_synth(batch_arrays)
    S = base.n_sources
    th0 = np.zeros((S, cb.NP))
    th0[:, 0:2] = batch_arrays.u_cat
    timings = {"start": 0.0, "render": 0.0, "neighbours": 0.0, "fit": 0.0}
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
    res = None
    history = []
    for k in range(sweeps):
        t = time.perf_counter()
        ctx.render_fields(base, theta, img_field, n_fields, H, W, out=fields)
        t1 = time.perf_counter()
        ctx.neighbour_arrays(base, theta, img_field, n_fields, H, W, fields, nbr_off, nbr_mean, nbr_var)
        t2 = time.perf_counter()
        bk = cb.Batch.from_synth(batch_arrays, nbr=(nbr_mean, nbr_var, nbr_off))
        theta, res = ctx.batch_fit(bk, theta, cb.default_opts(init_mode=cb.INIT_AS_GIVEN))
        t3 = time.perf_counter()
        timings["render"] += t1 - t
        timings["neighbours"] += t2 - t1
        timings["fit"] += t3 - t2
        history.append(dict(sweep=k, converged=int(np.sum(res["status"] == cb.CONVERGED)),
                            iters_mean=float(np.mean(res["iters"])), elbo_sum=float(np.sum(res["elbo"])),
                            fit_s=t3 - t2, render_s=t1 - t))
        if log:
            log(f"sweep {k}: fit {t3 - t2:.2f} s, render {t1 - t:.2f} s, neighbours {t2 - t1:.2f} s, "
                f"converged {history[-1]['converged']}, iterations {history[-1]['iters_mean']:.2f}")
    return theta, res, dict(timings=timings, history=history, nbr=(nbr_mean, nbr_var, nbr_off), fields=fields)
