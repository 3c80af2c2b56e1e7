"""Fit the galaxy-profile prototype mixtures used by the Celeste model.

The model renders a galaxy as a mixture of an exponential (Sersic n=1) and a
de Vaucouleurs (Sersic n=4) profile, each approximated by a small mixture of
isotropic, zero-mean bivariate Gaussians (section III-A: the non-random
galaxy vector holds shape, scale and morphology).  The paper gives neither the
mixture sizes nor their coefficients; this script fits our own: 6 components
for the exponential and 8 for the de Vaucouleurs profile, by weighted least
squares of the normalised 2-D surface brightness on a log-spaced radial grid.

Radii are in units of the half-light radius r_e, so a component's covariance
is  var_j * r_e^2 * I  before the axis-ratio/angle transform.  Amplitudes are
normalised to sum to one (each prototype carries unit flux).

Run:  python synth/fit_profiles.py   (writes synth/galaxy_profiles.json)
"""
import json
import os

import numpy as np
from scipy.optimize import least_squares
from scipy.special import gammaincinv, gamma


def sersic_profile(r, n):
    """Unit-flux 2-D Sersic surface brightness at radius r (units of r_e)."""
    b = gammaincinv(2 * n, 0.5)          # half of the light inside r_e
    k = b ** (2 * n) / (2 * np.pi * n * gamma(2 * n))
    return k * np.exp(-b * r ** (1.0 / n)), b


def mog_profile(r, amp, var):
    return np.sum(amp[None, :] / (2 * np.pi * var[None, :])
                  * np.exp(-0.5 * r[:, None] ** 2 / var[None, :]), axis=1)


def fit(n, ncomp, rmax, seed=0):
    r = np.logspace(-3, np.log10(rmax), 400)
    target, b = sersic_profile(r, n)
    # flux-weighted residual: weight by r (area element) on a log grid -> r^2
    wts = r ** 1.0

    def unpack(x):
        la, lv = x[:ncomp], x[ncomp:]
        amp = np.exp(la - la.max())
        amp = amp / amp.sum()
        return amp, np.exp(np.clip(lv, -20.0, 10.0))

    def resid(x):
        amp, var = unpack(x)
        return wts * (mog_profile(r, amp, var) - target) / target.max()

    rng = np.random.default_rng(seed)
    best = None
    for trial in range(40):
        lv0 = np.sort(rng.uniform(np.log(1e-4 if n == 4 else 1e-3), np.log(rmax ** 2 / 4), ncomp))
        la0 = rng.normal(0, 1, ncomp)
        sol = least_squares(resid, np.concatenate([la0, lv0]), method="lm", max_nfev=20000)
        if best is None or sol.cost < best.cost:
            best = sol
    amp, var = unpack(best.x)
    order = np.argsort(var)
    amp, var = amp[order], var[order]
    # diagnostics: fraction of light within r_e and max relative flux error
    rr = np.linspace(0, rmax, 20001)
    enclosed = lambda prof: np.cumsum(prof * 2 * np.pi * rr) * (rr[1] - rr[0])
    ser, _ = sersic_profile(rr, n)
    mog = mog_profile(rr, amp, var)
    i_e = np.searchsorted(rr, 1.0)
    diag = {
        "b_n": float(b),
        "cost": float(best.cost),
        "sersic_frac_within_re": float(enclosed(ser)[i_e]),
        "mog_frac_within_re": float(enclosed(mog)[i_e]),
        "max_abs_cumflux_diff": float(np.max(np.abs(enclosed(ser) - enclosed(mog)))),
    }
    return amp, var, diag


def main():
    out = {}
    for name, n, k, rmax in (("exp", 1, 6, 8.0), ("dev", 4, 8, 16.0)):
        amp, var, diag = fit(n, k, rmax)
        out[name] = {"amp": [float(a) for a in amp], "var": [float(v) for v in var],
                     "sersic_n": n, "fit": diag}
        print(name, diag)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "galaxy_profiles.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
