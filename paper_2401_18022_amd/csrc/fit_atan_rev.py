"""Coefficients of atan_rev32 (isrsgn_adjoint.hip): atan(t) / (2 pi) ~ t P(t^2) on t in [0, 1], P of
degree 7, fitted for the smallest largest absolute error by Lawson's iteration (iteratively
reweighted least squares) and checked in FP32 Horner evaluation.  Prints the coefficients and
the error bound.  Run: python paper_2401_18022_amd/csrc/fit_atan_rev.py"""
import numpy as np

DEG = 7


def fit(deg=DEG, iters=200):
    t = np.concatenate([np.cos(np.linspace(0.0, np.pi / 2, 4000)), np.linspace(0.0, 1.0, 4000)])
    A = np.vstack([t * (t * t) ** k for k in range(deg + 1)]).T
    f = np.arctan(t) / (2.0 * np.pi)
    w = np.ones_like(t)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], f * sw, rcond=None)
        w = w * (np.abs(A @ c - f) + 1e-30)
        w /= w.sum()
    return c.astype(np.float32)


def eval32(c, t):
    """t P(t^2) in FP32 Horner order, as the kernel evaluates it."""
    t = np.asarray(t, dtype=np.float32)
    u = (t * t).astype(np.float32)
    p = np.float32(c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p * u + np.float32(c[k])).astype(np.float32)
    return (p * t).astype(np.float32)


if __name__ == "__main__":
    c = fit()
    t = np.linspace(0.0, 1.0, 200001, dtype=np.float32)
    err = np.abs(eval32(c, t).astype(np.float64) - np.arctan(t.astype(np.float64)) / (2.0 * np.pi))
    print("coefficients (t^1, t^3, ...):", ", ".join(f"{float(x):.9g}f" for x in c))
    print(f"max |error| on [0, 1]: {err.max():.3g} revolutions")
