"""Writes the constants of sincos.hpp (run: python gen_sincos.py).

sin r = r + r^3 (s0 + s1 r^2 + s2 r^4 + s3 r^6) and
cos r = 1 + r^2 (c0 + c1 r^2 + c2 r^4 + c3 r^6) on |r| <= pi/4, fitted by
least squares in FP64 on 4001 Chebyshev nodes of [0, pi/4] (relative weight
for sin), then rounded to FP32; pi/2 split into three FP32 parts for the
Cody-Waite reduction.  Prints the constants and the worst absolute error of
an FP32 evaluation over [-pi/4, pi/4].
"""
import numpy as np


def fit():
    r = np.cos(np.linspace(0.0, np.pi, 4001)) * (np.pi / 8) + np.pi / 8
    r = r[r > 1e-4]
    a = np.stack([r ** (3 + 2 * k) for k in range(4)], 1)
    w = 1.0 / np.abs(np.sin(r))
    s = np.linalg.lstsq(a * w[:, None], (np.sin(r) - r) * w, rcond=None)[0]
    a = np.stack([r ** (2 + 2 * k) for k in range(4)], 1)
    c = np.linalg.lstsq(a, np.cos(r) - 1.0, rcond=None)[0]
    return s.astype(np.float32), c.astype(np.float32)


def split_pio2():
    p = np.pi / 2
    hi = np.float32(p)
    mid = np.float32(p - float(hi))
    lo = np.float32(p - float(hi) - float(mid))
    return hi, mid, lo


def worst_error(s, c):
    rr = np.linspace(-np.pi / 4, np.pi / 4, 200001).astype(np.float32)
    r2 = rr * rr
    ps, pc = s[3], c[3]
    for k in (2, 1, 0):
        ps = ps * r2 + s[k]
        pc = pc * r2 + c[k]
    sv = rr + rr * r2 * ps
    cv = np.float32(1.0) + r2 * pc
    x = rr.astype(np.float64)
    return float(np.abs(sv - np.sin(x)).max()), float(np.abs(cv - np.cos(x)).max())


if __name__ == "__main__":
    s, c = fit()
    print("sin", [repr(float(v)) for v in s])
    print("cos", [repr(float(v)) for v in c])
    print("pi/2", [repr(float(v)) for v in split_pio2()])
    print("worst abs error sin %.3g cos %.3g" % worst_error(s, c))
