"""Derive the polynomial coefficients of the fp32 sincospi used for recurrence seeds (kernels_bf16.hip).

On f in [-1/4, 1/4]:  sin(pi f) ~ f (s1 + s3 x + s5 x^2 + s7 x^3),  cos(pi f) ~ 1 + c2 x + c4 x^2 + c6 x^3 + c8 x^4,
x = f^2.  Coefficients: least-squares fit in double precision on 4001 Chebyshev points of x in [0, 1/16],
weighted to equalise the relative error.  Prints the coefficients and the worst errors of an fp32 evaluation.
"""
import numpy as np


def fit():
    t = np.cos(np.pi * (np.arange(4001) + 0.5) / 4001)
    f = 0.125 + 0.125 * t                      # f in (0, 1/4)
    x = f * f
    As = np.stack([x ** k for k in range(4)], axis=1)
    bs = np.sin(np.pi * f) / f
    s = np.linalg.lstsq(As / bs[:, None], np.ones_like(bs), rcond=None)[0]
    Ac = np.stack([x ** k for k in range(1, 5)], axis=1)
    bc = np.cos(np.pi * f) - 1.0
    c = np.linalg.lstsq(Ac, bc, rcond=None)[0]
    return s, c


def check(s, c):
    f32 = np.float32
    fs = np.linspace(-0.25, 0.25, 200001)
    fv = fs.astype(f32)
    x = fv * fv
    sp = fv * (f32(s[0]) + x * (f32(s[1]) + x * (f32(s[2]) + x * f32(s[3]))))
    cp = f32(1) + x * (f32(c[0]) + x * (f32(c[1]) + x * (f32(c[2]) + x * f32(c[3]))))
    es = np.abs(sp.astype(np.float64) - np.sin(np.pi * fv.astype(np.float64))).max()
    ec = np.abs(cp.astype(np.float64) - np.cos(np.pi * fv.astype(np.float64))).max()
    return es, ec


if __name__ == "__main__":
    s, c = fit()
    print("sin:", ", ".join(f"{v:.9e}f" for v in s))
    print("cos:", ", ".join(f"{v:.9e}f" for v in c))
    print("max abs err (fp32 eval): sin %.2e cos %.2e" % check(s, c))
