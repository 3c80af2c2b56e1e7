"""Plain initialisation of a source (oracle).

The paper starts each source from an existing catalog's estimate (sections
III-B/C).  With no catalog, the plain start used here is:
  u      = catalog position (patch centre)
  a      = 0.5, e_dev = 0.5, e_axis = 0.7, e_angle = 0, e_scale = 1.5 px
  r1     = log(max(F_ap, 1 nMgy)) for both types, F_ap the mean over the source's
           r-band images of sum (x - sky) / calib over pixels within 3 px of the
           source's catalog position in that image
  r2     = prior variance of log brightness, c1 = prior colour mean,
  c2     = diagonal of the prior colour covariance.
Parity: pinned by a brute-force loop over pixels on a tiny patch in the tests.
"""
from __future__ import annotations

import math

import numpy as np

APERTURE_PX = 3.0
MIN_FLUX = 1.0
REF_BAND = 2


def plain_init(u_cat, images, prior):
    th = np.zeros(27)
    th[0:2] = u_cat
    th[2] = 0.5
    th[3] = 0.5
    th[4] = 0.7
    th[5] = 0.0
    th[6] = 1.5
    fluxes = []
    for img in images:
        if img["band"] != REF_BAND:
            continue
        A = np.array([[img["wcs"][0], img["wcs"][1]], [img["wcs"][2], img["wcs"][3]]])
        p = A @ np.asarray(u_cat) + img["wcs"][4:6]
        x = np.asarray(img["pixels"], dtype=np.float64)
        tot = 0.0
        for r in range(img["h"]):
            for c in range(img["w"]):
                px = img["origin"][0] + c
                py = img["origin"][1] + r
                if (px - p[0]) ** 2 + (py - p[1]) ** 2 <= APERTURE_PX ** 2:
                    tot += (x[r, c] - img["sky"]) / img["calib"]
        fluxes.append(tot)
    f = np.mean(fluxes) if fluxes else MIN_FLUX
    r1 = math.log(max(f, MIN_FLUX))
    th[7] = th[8] = r1
    th[9] = prior["r_var"][0]
    th[10] = prior["r_var"][1]
    th[11:15] = prior["c_mean"][0]
    th[15:19] = prior["c_mean"][1]
    th[19:23] = np.diag(prior["c_cov"][0])
    th[23:27] = np.diag(prior["c_cov"][1])
    return th
