"""CPU check of cis_quarter (csrc/fft.hip), the float32 cos/sin of the dispersive phase's
remainder after whole quarter turns: its constants are the output of fit_cis_quarter.py, and
the polynomials meet the stated error bounds, exactly and in emulated float32 evaluation."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_constants():
    src = open(os.path.join(ROOT, "paper_2508_04951_amd", "csrc", "fft.hip")).read()
    body = src[src.index("__device__ __forceinline__ float2 cis_quarter"):]
    body = body[:body.index("}")]
    v = [float.fromhex(h) for h in re.findall(r"(-?0x[0-9a-fA-F.]+p[+-]?\d+)f", body)]
    # order in the source: S3, S2, S1, S0, C3, C2, C1, C0
    return [v[3], v[2], v[1], v[0]], [v[7], v[6], v[5], v[4]]


def test_constants_are_the_fit():
    from paper_2508_04951_amd.fit_cis_quarter import coefficients

    S, C = coefficients()
    kS, kC = kernel_constants()
    assert kS == S and kC == C
    assert all(float(np.float32(c)) == c for c in S + C)


def test_exact_polynomial_error_bounds():
    from paper_2508_04951_amd.fit_cis_quarter import errors

    es, ec = errors(*kernel_constants())
    assert es < 5.1e-9 and ec < 4.1e-10, (es, ec)


def _fmaf(a, b, c):
    # float32 fused multiply-add: the float64 product of two float32 values is exact, so one
    # float64 sum and a rounding to float32 (double rounding aside) model it
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def test_float32_evaluation_error():
    """Within 7e-8 of the true values (about one float32 ulp of 1) and within 2 ulp of each."""
    S, C = kernel_constants()
    w = np.float32(np.linspace(-0.5, 0.5, 200001))
    u = np.float32(w * w)
    ps = _fmaf(u, np.float32(S[3]), np.float32(S[2]))
    ps = _fmaf(u, ps, np.float32(S[1]))
    ps = _fmaf(u, ps, np.float32(S[0]))
    pc = _fmaf(u, np.float32(C[3]), np.float32(C[2]))
    pc = _fmaf(u, pc, np.float32(C[1]))
    pc = _fmaf(u, pc, np.float32(C[0]))
    c = _fmaf(u, pc, np.float32(1.0))
    s = np.float32(w * ps)
    wd = np.float64(w)
    tc, ts = np.cos(np.pi * wd / 2), np.sin(np.pi * wd / 2)
    ulp_c = np.spacing(np.float32(np.abs(tc))).astype(np.float64)
    ulp_s = np.spacing(np.maximum(np.float32(np.abs(ts)), np.float32(1e-30))).astype(np.float64)
    assert np.max(np.abs(c - tc)) < 7e-8 and np.max(np.abs(s - ts)) < 7e-8
    assert np.max(np.abs(c - tc) / ulp_c) <= 2.0
    assert np.max(np.abs(s - ts) / ulp_s) <= 2.0
