"""The GELU the fused forward pass evaluates: Phi(a) - 1/2 = c P(c^2), c = a
clamped to [-3.7, 3.7], P of degree 6.  Its coefficients, read from the
kernel source, against scipy's normal distribution function in float32
arithmetic as the kernel does it, and against the fitting script."""
import os
import re

import numpy as np
from scipy.special import ndtr

from paper_2202_05012_amd import gelu_poly_fit as G

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2202_05012_amd", "csrc", "supa_mlp.hip")
BOUND = 5.9e-5           # |Phi error|, the figure the kernel comment and the GPU bound use


def kernel_poly():
    """(clamp, coefficients lowest power first) as typed in gelu_poly."""
    src = open(SRC).read()
    body = src[src.index("float gelu_poly(float a)"):]
    body = body[:body.index("\n}\n")]
    clamp = float(re.search(r"fmed3f\(a, -([0-9.]+)f, ([0-9.]+)f\)", body).group(1))
    first = float(re.search(r"float p = ([-0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"p = fmaf\(p, s, ([-0-9.e]+)f\)", body)]
    return clamp, np.array(([first] + rest)[::-1])


def test_phi_error_bound_everywhere():
    clamp, coef = kernel_poly()
    assert clamp == G.C and len(coef) == G.N
    a = np.linspace(-40.0, 40.0, 800001)
    err = np.abs(G.phi_f32(a, clamp, coef).astype(np.float64) - ndtr(a))
    assert err.max() <= BOUND, err.max()
    # GELU = a Phi(a): off by at most BOUND |a|
    gelu = a * G.phi_f32(a, clamp, coef).astype(np.float64)
    assert (np.abs(gelu - a * ndtr(a)) <= BOUND * np.abs(a) + 1e-300).all()


def test_phi_shape():
    """Odd about 1/2, slope 1/sqrt(2 pi) at 0, constant beyond the clamp."""
    clamp, coef = kernel_poly()
    a = np.linspace(0.0, 10.0, 10001)
    up = G.phi_f32(a, clamp, coef).astype(np.float64)
    down = G.phi_f32(-a, clamp, coef).astype(np.float64)
    assert np.abs(up + down - 1.0).max() <= 2.4e-7          # float32 rounding only
    assert abs(coef[0] - 1.0 / np.sqrt(2.0 * np.pi)) <= 1e-3
    beyond = G.phi_f32(np.array([clamp, 5.0, 50.0]), clamp, coef)
    assert beyond[0] == beyond[1] == beyond[2]


def test_script_reproduces_the_kernel_coefficients():
    clamp, coef = kernel_poly()
    fitted = G.fit(clamp, len(coef))
    np.testing.assert_allclose(fitted, coef, rtol=1e-6, atol=0)
