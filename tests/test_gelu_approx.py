"""The erfc approximation the fused forward pass evaluates GELU with
(Abramowitz & Stegun 7.1.26): its coefficients, as typed into the kernel,
against scipy's erfc, within the published absolute error 1.5e-7."""
import numpy as np
from scipy.special import erfc

P = 0.3275911
A = (0.254829592, -0.284496736, 1.421413741, -1.453152027, 1.061405429)


def erfc_as(x):
    t = 1.0 / (1.0 + P * x)
    poly = t * (A[0] + t * (A[1] + t * (A[2] + t * (A[3] + t * A[4]))))
    return poly * np.exp(-x * x)


def test_as_7_1_26_error_bound():
    x = np.linspace(0.0, 12.0, 200001)
    err = np.abs(erfc_as(x) - erfc(x))
    assert err.max() <= 1.5e-7, err.max()
    # GELU from it: a Phi(a), Phi(-|a|) = erfc(|a| / sqrt 2) / 2
    a = np.linspace(-12.0, 12.0, 100001)
    h = 0.5 * erfc_as(np.abs(a) / np.sqrt(2.0))
    gelu = a * np.where(a >= 0, 1.0 - h, h)
    exact = 0.5 * a * erfc(-a / np.sqrt(2.0))
    assert (np.abs(gelu - exact) <= 0.75e-7 * np.abs(a) + 1e-300).all()
