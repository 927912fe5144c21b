"""Coefficients of the odd polynomial used for the BF16 GELU epilogue.

Phi(x) - 1/2 (Phi = standard normal CDF) is approximated on [-C, C] by
x * P(x^2), P of degree DEG, fitted by iteratively reweighted least squares
towards equal-ripple error (on s = x / C for conditioning); outside the
interval the argument is clamped to +-C, where 1/2 - Phi(C) = 3.4e-6.
Prints the coefficients (x basis) and the maximum error of an FP32 Horner
evaluation over a dense grid.  Run once; the printed values are pasted into
common.hpp.
"""
import numpy as np
from scipy.special import erf

C, DEG = 4.5, 8


def half_centered_cdf(x):
    return 0.5 * erf(x / np.sqrt(2.0))


def fit(c, deg, iters=60):
    s = np.linspace(1e-7, 1.0, 40001)
    a = np.stack([s * (s * s) ** k for k in range(deg + 1)], 1)
    y = half_centered_cdf(c * s)
    w = np.ones_like(s)
    for _ in range(iters):
        q, *_ = np.linalg.lstsq(a * w[:, None], y * w, rcond=None)
        err = np.abs(a @ q - y)
        w = w * (err / err.max() + 1e-4) ** 0.5
        w /= w.max()
    return np.array([q[k] / c ** (2 * k + 1) for k in range(deg + 1)])


def fp32_eval(coef, x):
    xf = np.clip(x.astype(np.float32), -C, C)
    u = xf * xf
    p = np.float32(coef[-1])
    for k in range(len(coef) - 2, -1, -1):
        p = (p * u + np.float32(coef[k])).astype(np.float32)
    return (xf * p).astype(np.float64)


if __name__ == "__main__":
    coef = fit(C, DEG)
    x = np.linspace(-8.0, 8.0, 400001)
    err = np.abs(fp32_eval(coef, x) - half_centered_cdf(x)).max()
    for k, v in enumerate(coef):
        print(f"c{k} = {np.float32(v).item():.9e}f")
    print(f"max |error| of Phi - 1/2 on [-8, 8]: {err:.3e}")
