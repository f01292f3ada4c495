"""Fits the polynomial the HOG kernel uses for atan, in units of orientation
bins: atan(r) * 9 / pi ~= r * P(r^2) on [0, 1], degree 7 in r^2, by
iteratively reweighted least squares towards the minimax error (Lawson).

    python fit_atan.py    # prints the coefficients and the float32 error
"""
import numpy as np


def fit(deg=7, n=20000, iters=300):
    r = np.sort(np.concatenate([np.linspace(0, 1, n), np.cos(np.linspace(0, np.pi / 2, n))]))
    f = np.arctan(r) * 9 / np.pi
    A = np.stack([r ** (2 * k + 1) for k in range(deg + 1)], 1)
    w = np.ones_like(r)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], f * sw, rcond=None)
        e = np.abs(A @ c - f)
        w = w * e
        w /= w.sum()
    c32 = c.astype(np.float32)
    r32 = r.astype(np.float32)
    s = r32 * r32
    p = np.float32(c32[-1])
    for k in range(deg - 1, -1, -1):
        p = (p * s + c32[k]).astype(np.float32)
    err = np.abs((p * r32).astype(np.float64) - f).max()
    return c32, err


if __name__ == "__main__":
    c, err = fit()
    print("coefficients (r^1 .. r^15):", [float(x) for x in c])
    print(f"max |error| in float32 Horner: {err:.3g} bins")
