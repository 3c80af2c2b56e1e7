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


def structural_zeros():
    """(i, j) Hessian entries that are exactly zero by the model's structure: a colour index
    j in {0, 1} (u-g, g-r: bands u, g) and one in {2, 3} (r-i, i-z: bands i, z) enter no band
    together, so the pixel sum couples them nowhere; the prior couples colour means only with
    colour means of the same type (full covariance) and keeps colour variances separable.
    Pairs of same-type colour means are left out (their prior coupling is an entry of the
    inverse prior covariance that is zero only up to rounding)."""
    c1 = {"s": 11, "g": 15}
    c2 = {"s": 19, "g": 23}
    bases = [("c1", t, c1[t]) for t in "sg"] + [("c2", t, c2[t]) for t in "sg"]
    out = set()
    for ka, ta, a in bases:
        for kb, tb, b in bases:
            if ka == kb == "c1" and ta == tb:
                continue
            for j in (0, 1):
                for k in (2, 3):
                    out.add((a + j, b + k))
                    out.add((b + k, a + j))
    return sorted(out)


def assert_structural_zeros(H, what=""):
    H = np.asarray(H)
    bad = [(i, j, float(H[..., i, j].flat[np.argmax(np.abs(H[..., i, j]))]))
           for i, j in structural_zeros() if np.any(H[..., i, j] != 0.0)]
    assert not bad, f"{what} structural zeros not exactly 0: {bad[:5]}"
