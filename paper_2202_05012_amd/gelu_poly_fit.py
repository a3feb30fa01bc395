"""Coefficients of the GELU polynomial of the fused forward pass.

GELU(a) = a Phi(a).  The kernel evaluates Phi(a) - 1/2 = c P(c^2) with c = a
clamped to [-C, C] and P of degree N - 1 in c^2.  The fit minimises the
largest error of c P(c^2) against Phi(c) - 1/2 on (0, C]: weighted least
squares in a Chebyshev basis of t = 2 c^2 / C^2 - 1, the weights multiplied
by the current errors each round (Lawson's iteration, which tends to the
equal-ripple fit), then the series rewritten as powers of c^2.  The clamp
makes Phi constant beyond C; the fit's ripple and the tail Phi(-C) share the
error budget, so C is chosen with N to minimise the largest error over all a
(evaluated in float32 the way the kernel does it).

Run to print the coefficients, lowest power first, and the float32 error:

    python -m paper_2202_05012_amd.gelu_poly_fit
"""
import numpy as np
from numpy.polynomial import chebyshev as cheb
from numpy.polynomial import polynomial as poly
from scipy.special import ndtr

N = 7          # coefficients (degree 6 in c^2)
C = 3.7        # clamp


def fit(c_max: float, n: int, iters: int = 60) -> np.ndarray:
    """Coefficients of P in powers of c^2 (float64, lowest first)."""
    a = np.linspace(1e-6, c_max, 20001)
    t = 2.0 * a * a / (c_max * c_max) - 1.0
    target = ndtr(a) - 0.5
    V = cheb.chebvander(t, n - 1) * a[:, None]
    w = np.ones_like(a)
    for _ in range(iters):
        sw = np.sqrt(w)
        coef, *_ = np.linalg.lstsq(V * sw[:, None], target * sw, rcond=None)
        err = np.abs(V @ coef - target)
        w = w * (err + 1e-30)
        w /= w.sum()
    in_t = cheb.cheb2poly(coef)                  # powers of t
    in_s = np.zeros(n)                           # powers of s = c^2
    lin = np.array([-1.0, 2.0 / (c_max * c_max)])
    term = np.array([1.0])
    for k in range(n):
        in_s[:len(term)] += in_t[k] * term
        term = poly.polymul(term, lin)
    return in_s


def phi_f32(a: np.ndarray, c_max: float, coef) -> np.ndarray:
    """Phi as the kernel computes it: float32 operations, each multiply-add
    rounded once."""
    c = np.clip(a.astype(np.float32), np.float32(-c_max), np.float32(c_max))
    s = (c * c).astype(np.float32)
    p32 = np.asarray(coef, dtype=np.float32)
    acc = np.full_like(s, p32[-1])
    for k in range(len(p32) - 2, -1, -1):
        acc = (acc.astype(np.float64) * s + np.float64(p32[k])).astype(np.float32)
    return (c.astype(np.float64) * acc + 0.5).astype(np.float32)


if __name__ == "__main__":
    coef = fit(C, N)
    a = np.linspace(-12.0, 12.0, 600001)
    err = np.abs(phi_f32(a, C, coef).astype(np.float64) - ndtr(a)).max()
    print("coefficients (powers of c^2):", ", ".join(repr(float(v)) for v in coef.astype(np.float32)))
    print(f"largest |Phi error| in float32 over [-12, 12]: {err:.3e}")
