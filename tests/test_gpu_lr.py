"""GPU parity of the linear-response covariance (celeste_lr_covariance_from_hessian and
celeste_lr_covariance) against the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from oracle import init as oinit
from oracle import lr, model, newton, transforms

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


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
def fitted():
    """Oracle fits of three bright sources (one interior, two with q(star) at its lower edge)
    and the oracle's gradient and Hessian there."""
    full = synth.make_config(1, n_sources=4, bright=True)
    pick = [0, 1, 3]
    sb = full.subset(pick)
    th, u0, g, H = [], [], [], []
    for k in range(sb.n_sources):
        imgs = model.source_images(sb, k)
        st = oinit.plain_init(sb.u_cat[k], imgs, sb.prior)
        res = newton.fit(st, imgs, sb.prior, sb.profiles)
        _, gk, Hk = model.elbo(res.theta, imgs, sb.prior, sb.profiles)
        th.append(res.theta)
        u0.append(st[0:2])
        g.append(gk)
        H.append(Hk)
        _say("fitted source", k, "status", res.status, "a", res.theta[2])
    return sb, np.array(th), np.array(u0), np.array(g), np.array(H)


def _psi_parts(theta, u0, g, H, box=3.0):
    """Oracle-side D, Sigma_psi and the condition number of -H_psi."""
    psi = transforms.to_psi(theta, u0, box)
    _, d1, d2 = transforms.to_theta(psi, u0, box)
    _, Hp = transforms.grad_hess_psi(g, H, d1, d2)
    Hp = 0.5 * (Hp + Hp.T)
    ev = np.linalg.eigvalsh(-Hp)
    return d1, d2, -np.linalg.inv(Hp), ev.max() / ev.min()


def _assert_inverse_close(cov, theta, u0, g, H, what):
    """GPU Cholesky against the oracle's inverse: elementwise within 64 eps kappa of the
    scale of Sigma_psi, mapped through D."""
    ref = lr.lr_covariance(theta, g, H, u0)
    assert ref is not None
    d1, _, Sp, kappa = _psi_parts(theta, u0, g, H)
    tol = 64 * EPS * kappa * np.outer(np.abs(d1), np.abs(d1)) * np.max(np.abs(Sp))
    err = np.abs(cov - ref)
    _say(what, "kappa", f"{kappa:.3e}", "max err / tol", np.max(err / tol))
    assert np.all(err <= tol), f"{what}: max err/tol {np.max(err / tol):.3e}"
    assert np.array_equal(cov, cov.T)


def test_from_hessian_oracle_inputs_host_and_device(cb, ctx, fitted):
    import torch
    sb, th, u0, g, H = fitted
    cov, st = ctx.lr_covariance_from_hessian(th, u0, g, H)
    assert np.all(st == 0)
    for k in range(len(th)):
        _assert_inverse_close(cov[k], th[k], u0[k], g[k], H[k], f"host source {k}")
    dv = [torch.from_numpy(x).cuda() for x in (th, u0, g, H)]
    cov_d, st_d = ctx.lr_covariance_from_hessian(*dv)
    assert np.array_equal(st_d, st) and np.array_equal(cov_d.cpu().numpy(), cov)


def test_from_hessian_random_cases_and_statuses(cb, ctx):
    """Random interior points with random negative-definite Hessians of growing condition
    number and small gradients, one indefinite Hessian and one NaN."""
    rng = np.random.default_rng(17)
    n = 40
    base = synth.make_config(0).theta_truth[0]
    th = np.repeat(base[None, :], n, axis=0)
    th[:, 2] = rng.uniform(0.05, 0.95, n)
    th[:, 4] = rng.uniform(0.1, 0.9, n)
    th[:, 6] = rng.uniform(0.5, 5.0, n)
    u0 = th[:, 0:2] + rng.uniform(-2.5, 2.5, (n, 2))
    g = 1e-3 * rng.normal(size=(n, 27))
    H = np.empty((n, 27, 27))
    for k in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(27, 27)))
        lam = np.logspace(0, k / 5.0, 27)           # condition number up to 1e8
        H[k] = -(Q * lam) @ Q.T
    H[n - 2] = -H[n - 2]                            # positive definite: no maximum
    g[n - 1, 5] = np.nan
    cov, st = ctx.lr_covariance_from_hessian(th, u0, g, H)
    assert st[n - 2] == 1 and st[n - 1] == 2
    assert np.all(np.isnan(cov[n - 2])) and np.all(np.isnan(cov[n - 1]))
    assert lr.lr_covariance(th[n - 2], g[n - 2], H[n - 2], u0[n - 2]) is None
    for k in range(n - 2):
        assert st[k] == 0
        _assert_inverse_close(cov[k], th[k], u0[k], g[k], H[k], f"random case {k}")


def test_invalid_arguments(cb, ctx):
    th = np.zeros((2, 27))
    u0 = np.zeros((2, 2))
    g = np.zeros((2, 27))
    H = np.zeros((2, 27, 27))
    with pytest.raises(cb.CelesteError) as ei:
        ctx.lr_covariance_from_hessian(th, u0, g, H, u_box=0.0)
    assert ei.value.code == cb.E_INVALID
    lib = cb.load()
    st = np.zeros(2, np.int32)
    rc = lib.celeste_lr_covariance_from_hessian(ctx._h, 2, cb.MEM_HOST, th.ctypes.data, None, 3.0, g.ctypes.data,
                                                H.ctypes.data, H.ctypes.data, st.ctypes.data, None)
    assert rc == cb.E_INVALID
    rc = lib.celeste_lr_covariance_from_hessian(ctx._h, 2, 7, th.ctypes.data, u0.ctypes.data, 3.0, g.ctypes.data,
                                                H.ctypes.data, H.ctypes.data, st.ctypes.data, None)
    assert rc == cb.E_INVALID


def test_end_to_end_against_oracle_hessian_bound(cb, ctx, fitted):
    """celeste_lr_covariance evaluates the gradient and Hessian itself (FP32 pixel sums); its
    result is compared with the oracle's covariance within the first-order effect of the
    Hessian difference, which this test measures (GPU Hessian from celeste_elbo_eval)."""
    import torch
    sb, th, u0, _, _ = fitted
    b = cb.Batch.from_synth(sb)
    cov, st = ctx.lr_covariance(b, th, u0)
    _, g_gpu, H_gpu = ctx.elbo_eval(b, th)
    dev = synth.make_config(1, n_sources=4, bright=True).subset([0, 1, 3])
    dev.pixels = torch.from_numpy(sb.pixels).cuda()
    cov_d, st_d = ctx.lr_covariance(cb.Batch.from_synth(dev), torch.from_numpy(th).cuda(),
                                    torch.from_numpy(u0).cuda())
    assert np.array_equal(st_d, st) and np.array_equal(cov_d.cpu().numpy(), cov)
    for k in range(sb.n_sources):
        imgs = model.source_images(sb, k)
        _, go, Ho = model.elbo(th[k], imgs, sb.prior, sb.profiles)
        ref = lr.lr_covariance(th[k], go, Ho, u0[k])
        assert ref is not None and st[k] == 0
        d1, d2, Sp, kappa = _psi_parts(th[k], u0[k], go, Ho)
        dHp = d1[:, None] * (0.5 * (H_gpu[k] + H_gpu[k].T) - 0.5 * (Ho + Ho.T)) * d1[None, :] \
            + np.diag(d2 * (g_gpu[k] - go))
        first = np.abs(Sp) @ np.abs(dHp) @ np.abs(Sp)
        tol = 2 * np.outer(np.abs(d1), np.abs(d1)) * first + 1e-9 * np.max(np.abs(ref))
        err = np.abs(cov[k] - ref)
        _say(f"source {k}: kappa {kappa:.3e}, max err/tol {np.max(err / tol):.3e}, "
             f"LR var u_x {ref[0, 0]:.3e} (gpu {cov[k][0, 0]:.3e})")
        assert np.all(err <= tol), f"source {k}: max err/tol {np.max(err / tol):.3e}"


def test_full_size_after_batched_fit(cb, ctx):
    """Config 2 at full size: batched fit from the plain start, then the covariance of every
    source on device memory; exact symmetry and positive semi-definiteness wherever the status
    is 0, and a sample of sources against the oracle (first-order Hessian-difference bound)."""
    import torch
    sb = synth.make_config(2, device="cuda")
    b = cb.Batch.from_synth(sb)
    theta0 = np.zeros((sb.n_sources, 27))
    theta0[:, 0:2] = sb.u_cat
    th, res = ctx.batch_fit(b, theta0, cb.default_opts(init_mode=cb.INIT_PLAIN))
    u0 = torch.from_numpy(sb.u_cat.astype(np.float64)).cuda()
    cov, st = ctx.lr_covariance(b, th, u0)
    covh = cov.cpu().numpy()
    thh = th.cpu().numpy()
    ok = st == 0
    _say("full size: status counts", np.bincount(st, minlength=3), "of", sb.n_sources)
    assert ok.mean() > 0.5
    assert np.all(np.isnan(covh[~ok]))
    assert np.array_equal(covh[ok], np.transpose(covh[ok], (0, 2, 1)))
    rng = np.random.default_rng(5)
    for s in rng.choice(np.flatnonzero(ok), 200, replace=False):
        ev = np.linalg.eigvalsh(covh[s])
        assert ev.min() >= -1e-9 * ev.max(), (s, ev.min(), ev.max())
    npx = np.array([np.sum(sb.img_h[sb.src_img_off[s]:sb.src_img_off[s + 1]].astype(np.int64) ** 2)
                    for s in range(sb.n_sources)])
    cand = np.flatnonzero(ok & (npx < 40000))
    pick = [int(x) for x in rng.choice(cand, 3, replace=False)]
    sub = sb.subset(pick)
    el, g_gpu, H_gpu = ctx.elbo_eval(b, th)
    g_gpu, H_gpu = g_gpu.cpu().numpy(), H_gpu.cpu().numpy()
    for k, s in enumerate(pick):
        imgs = model.source_images(sub, k)
        _, go, Ho = model.elbo(thh[s], imgs, sub.prior, sub.profiles)
        ref = lr.lr_covariance(thh[s], go, Ho, sb.u_cat[s])
        if ref is None:
            _say("source", s, "oracle: -H_psi not positive definite; skipped")
            continue
        d1, d2, Sp, kappa = _psi_parts(thh[s], sb.u_cat[s], go, Ho)
        dHp = d1[:, None] * (0.5 * (H_gpu[s] + H_gpu[s].T) - 0.5 * (Ho + Ho.T)) * d1[None, :] \
            + np.diag(d2 * (g_gpu[s] - go))
        tol = 2 * np.outer(np.abs(d1), np.abs(d1)) * (np.abs(Sp) @ np.abs(dHp) @ np.abs(Sp)) \
            + 1e-9 * np.max(np.abs(ref))
        err = np.abs(covh[s] - ref)
        _say(f"full-size source {s} ({npx[s]} px): kappa {kappa:.3e}, max err/tol {np.max(err / tol):.3e}")
        assert np.all(err <= tol)
