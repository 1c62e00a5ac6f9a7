"""The closure kernel's forward GELU (a polynomial of Phi(-|a|), see
paper_1808_04406_amd/gelu_poly.py) against the exact GELU a Phi(a): the
coefficients compiled into the kernel are the generator's, and their FP32
evaluation stays within the 5e-6 |a| that the closure parity bound assumes
(ERR_MODEL[1] in test_gpu_closure.py)."""
import os
import re

import numpy as np
from scipy.special import ndtr

from paper_1808_04406_amd import gelu_poly

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_1808_04406_amd", "csrc", "closure.hpp")


def kernel_coefficients():
    src = open(HEADER).read()
    body = re.search(r"kGeluPoly\[(\d+)\]\s*=\s*\{([^}]*)\}", src)
    assert body, "kGeluPoly not found"
    vals = [float(v.strip().rstrip("f")) for v in body.group(2).split(",") if v.strip()]
    assert len(vals) == int(body.group(1))
    return np.array(vals)


def test_kernel_coefficients_are_the_generators():
    c = gelu_poly.coefficients()
    k = kernel_coefficients()
    assert len(k) == gelu_poly.DEG + 1
    assert np.allclose(k, c, rtol=2e-9, atol=1e-12)


def test_fp32_gelu_within_error_model():
    k = kernel_coefficients()
    a = np.concatenate([np.linspace(-30.0, 30.0, 600001), np.geomspace(1e-6, 30.0, 20001),
                        -np.geomspace(1e-6, 30.0, 20001)])
    a = a[a != 0.0]
    g = gelu_poly.gelu_poly_f32(a, k).astype(np.float64)
    a32 = a.astype(np.float32).astype(np.float64)
    exact = a32 * ndtr(a32)
    rel = np.abs(g - exact) / np.abs(a32)
    assert rel.max() <= 5e-6, rel.max()
    assert gelu_poly.gelu_poly_f32(np.zeros(1), k)[0] == 0.0
    # the clamp: beyond 4.5 the correction keeps its value at 4.5; large and
    # infinite inputs stay within the model (GELU(+inf) = +inf)
    big = np.array([4.5, 6.0, 1e3, 3e38, -6.0, -1e3], np.float32)
    gb = gelu_poly.gelu_poly_f32(big, k).astype(np.float64)
    b64 = big.astype(np.float64)
    assert np.all(np.abs(gb - b64 * ndtr(b64)) <= 5e-6 * np.abs(b64))
    with np.errstate(invalid="ignore"):
        assert gelu_poly.gelu_poly_f32(np.array([np.inf], np.float32), k)[0] == np.inf


def test_polynomial_tracks_phi_not_a_constant():
    """A dropped or permuted coefficient shows: each single-coefficient
    change of 1 % of its size moves the error past the model."""
    k = kernel_coefficients()
    a = np.linspace(-6.0, 6.0, 200001)
    for j in range(len(k)):
        kk = k.copy()
        kk[j] *= 1.01
        g = gelu_poly.gelu_poly_f32(a, kk).astype(np.float64)
        rel = np.abs(g - a * ndtr(a)) / np.maximum(np.abs(a), 1e-30)
        assert rel.max() > 5e-6, j
