"""Coefficients of the march's small optical-depth polynomial.

For x < 1/8 the march needs 1 - phi(x) = x q(x), q(x) = (x - 1 + e^{-x}) / x^2,
without cancellation.  It evaluates x q(x) = y R(y) in y = -x log2(e) with a
degree-2 polynomial R fitted here for the least maximum relative error over
x in [0, 1/8] (a linear program over a dense grid, the reference values in
40-digit arithmetic).  Prints the coefficients and the relative error of the
float32 evaluation (about 1.2e-6).  Run: python fit_small_x.py
"""
import mpmath as mp
import numpy as np
from scipy.optimize import linprog

mp.mp.dps = 40
LN2 = mp.log(2)


def r_exact(y):
    if y == 0:
        return -LN2 / 2
    x = -LN2 * mp.mpf(y)
    return (x - 1 + mp.e ** (-x)) / x / mp.mpf(y)


def fit(deg=2, n=4001):
    ys = np.linspace(-0.125 / float(LN2), 0.0, n)
    rv = np.array([float(r_exact(y)) for y in ys])
    V = np.vstack([ys ** k for k in range(deg + 1)]).T
    w = np.abs(rv)[:, None]
    A = np.vstack([np.hstack([V, -w]), np.hstack([-V, -w])])
    b = np.concatenate([rv, -rv])
    res = linprog(np.r_[np.zeros(deg + 1), 1.0], A_ub=A, b_ub=b,
                  bounds=[(None, None)] * (deg + 1) + [(0, None)], method="highs")
    c = res.x[:deg + 1]
    c32 = c.astype(np.float32)
    y32 = ys.astype(np.float32)
    p = np.zeros_like(y32)
    for k in range(deg, -1, -1):
        p = p * y32 + c32[k]
    return c, res.x[-1], float(np.max(np.abs(p.astype(np.float64) - rv) / np.abs(rv)))


if __name__ == "__main__":
    c, err, err32 = fit()
    print("R(y) = " + " + ".join(f"{float(v)!r} y^{k}" for k, v in enumerate(c)))
    print(f"max relative error {err:.3e} (exact arithmetic), {err32:.3e} (float32 evaluation)")
