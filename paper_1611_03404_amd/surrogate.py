"""Training driver of the surrogate initialiser (argument marshalling around libceleste).

Labels are the plain method's own converged fits: every training source is fitted
on the device from the plain start (celeste_batch_fit), and the converged
parameters, in the fits' unconstrained coordinates with the position box centred
on the catalog position, are standardised per coordinate.  The network is then
trained on the device by the library's own forward/backward kernels and Adam.
Initial weights and minibatch orders are inputs (seeded by the caller).
"""
from __future__ import annotations

import time

import numpy as np

from . import celeste as cb


def fit_labels(ctx, batch, u_cat, max_iter=50):
    """Plain-start fits of all sources; returns (theta, results)."""
    th0 = np.zeros((batch.n_sources, cb.NP))
    th0[:, 0:2] = u_cat
    th, res = ctx.batch_fit(batch, th0, cb.default_opts(init_mode=cb.INIT_PLAIN, max_iter=max_iter))
    if not isinstance(th, np.ndarray):
        th = th.cpu().numpy()
    return th, res


def standardise(psi, std_floor=1e-3):
    mean = psi.mean(axis=0)
    sd = np.maximum(psi.std(axis=0), std_floor)
    return mean, sd


def train(ctx, batch, u_cat, init_params, orders_fn, epochs=20, minibatch=256, lr=1e-3, log=None):
    """Label, standardise and train.  orders_fn(n, epochs) gives the (epochs, n) int32 orders.

    Returns (net, info) with the per-epoch losses and the label statistics."""
    import torch
    t0 = time.perf_counter()
    th, res = fit_labels(ctx, batch, u_cat)
    keep = np.nonzero(res["status"] == cb.CONVERGED)[0]
    t1 = time.perf_counter()
    psi = cb.theta_to_psi(th, u_cat)
    mean, sd = standardise(psi[keep])
    target = ((psi - mean) / sd).astype(np.float32)
    th_cat = np.zeros((batch.n_sources, cb.NP))
    th_cat[:, 0:2] = u_cat
    x_all = ctx.make_patches(batch, th_cat)
    idx = torch.from_numpy(keep).to(x_all.device)
    x = x_all.index_select(0, idx).contiguous()
    del x_all
    t = torch.from_numpy(target[keep]).to(x.device).contiguous()
    orders = torch.from_numpy(orders_fn(len(keep), epochs)).to(x.device).contiguous()
    net = cb.Net(ctx, init_params, mean, sd)
    t2 = time.perf_counter()
    losses = net.train(x, t, orders, batch=minibatch, lr=lr)
    t3 = time.perf_counter()
    info = dict(n_sources=batch.n_sources, n_labels=int(len(keep)), label_fit_s=t1 - t0, prep_s=t2 - t1,
                train_s=t3 - t2, epoch_loss=losses.tolist(), psi_mean=mean.tolist(), psi_std=sd.tolist())
    if log:
        log(f"surrogate: {len(keep)} labels in {t1 - t0:.1f} s, trained {epochs} epochs in {t3 - t2:.1f} s, "
            f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    return net, info
