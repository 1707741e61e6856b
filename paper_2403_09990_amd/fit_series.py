"""Coefficients of the arctangent polynomial in csrc/purse_geodesic.hpp.

    python -m paper_2403_09990_amd.fit_series

atan w = w + w^3 P(w^2) on 0 <= w <= tan(pi/8), P of degree 4, fitted to
(atan w - w) / w^3 by Lawson's algorithm (iteratively reweighted least squares
converging to the minimax fit of the absolute error of atan) on 4000 Chebyshev
points.  Prints the coefficients as float32 literals and the maximum error, in
exact arithmetic and with float32 Horner evaluation.
"""
import numpy as np


def fit(deg=4, iters=30, npts=4000):
    zmax = np.tan(np.pi / 8) ** 2
    z = (1 - np.cos(np.linspace(0, np.pi, npts))) / 2 * zmax
    z[0] = 1e-12
    w = np.sqrt(z)
    f = (np.arctan(w) - w) / w ** 3
    V = np.vander(z, deg + 1, increasing=True)
    wt = np.ones_like(z)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(V * wt[:, None], f * wt, rcond=None)
        err = np.abs((V @ c - f) * w ** 3)
        wt = wt * (err / err.max() + 1e-3) ** 0.5
    return c, float(np.abs((V @ c - f) * w ** 3).max())


def float32_error(c):
    zmax = np.tan(np.pi / 8) ** 2
    zz = np.linspace(0, zmax, 200001).astype(np.float32)
    ww = np.sqrt(zz.astype(np.float64)).astype(np.float32)
    cf = c.astype(np.float32)
    p = np.full_like(zz, cf[-1])
    for k in range(len(cf) - 2, -1, -1):
        p = (p * zz + cf[k]).astype(np.float32)
    approx = (ww + ww * (p * zz)).astype(np.float32)
    return float(np.abs(approx.astype(np.float64) - np.arctan(ww.astype(np.float64))).max())


if __name__ == "__main__":
    c, e = fit()
    for k, v in enumerate(c):
        print("c%d = %.9ef" % (k, np.float32(v)))
    print("max |error|: %.2e exact, %.2e float32 Horner" % (e, float32_error(c)))
