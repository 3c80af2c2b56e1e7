"""Shared helpers for the parity tests (comparison rules and oracle calls)."""
import numpy as np

from oracle import model

ELBO_RTOL = 1e-5        # relative error on the ELBO
DERIV_RTOL = 1e-4       # relative error on gradient / Hessian entries
DERIV_FLOOR = 1e-3      # ... relative to max(|e*|, DERIV_FLOOR * max|array*|)


def oracle_eval(sb, s, theta, nbr=None, want="hess"):
    imgs = model.source_images(sb, s, nbr=nbr)
    if want == "hess":
        return model.elbo(theta, imgs, sb.prior, sb.profiles)
    return model.elbo_value(theta, imgs, sb.prior, sb.profiles), None, None


def assert_elbo_close(got, ref, rtol=ELBO_RTOL, what=""):
    err = abs(got - ref) / max(abs(ref), 1e-300)
    assert err <= rtol, f"{what} ELBO rel err {err:.3e} (got {got!r}, oracle {ref!r})"


def deriv_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), DERIV_FLOOR * np.max(np.abs(ref)))
    return np.max(np.abs(got - ref) / scale)


def assert_derivs_close(g, H, gref, Href, rtol=DERIV_RTOL, what=""):
    eg = deriv_err(g, gref)
    eh = deriv_err(H, Href)
    assert eg <= rtol, f"{what} gradient err {eg:.3e}"
    assert eh <= rtol, f"{what} Hessian err {eh:.3e}"
