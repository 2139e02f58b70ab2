"""GPU parity of the paper's other Doppler resampling methods (App. C Alg. 1-3; Sec. I and
Table I linear interpolation and frequency conversion; Sec. III-A FFT P/Q resampling) against
the oracle's float64 definitions of the same methods, through the C ABI.

Bar: relative L2 <= 1e-5 with every element within 20 tol rms (tests/parity.py).  The Alg. 1
and Alg. 3 kernels compute the same sum in the same order and are compared bit for bit.
"""
from fractions import Fraction

import numpy as np
import pytest

import waveforms as wf
from parity import check

pytestmark = pytest.mark.gpu

C = 299792458


def alpha_exact(v):
    return float(Fraction(C + Fraction(v)) / Fraction(C - Fraction(v)))


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2508_04951_amd as rc

    return rc.Context(0)


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


ALPHAS = [1.0, 2.0, alpha_exact(-8000.0), alpha_exact(7500.0), alpha_exact(1000.0), 0.7654321, 1.37]


# --- App. C: the paper's sinc kernels ------------------------------------------------------

@pytest.mark.parametrize("n", [1, 7, 300, 5001])
@pytest.mark.parametrize("n_window", [1, 3, 25, 41])
@pytest.mark.parametrize("blocks", [0, 3])
def test_paper_direct_and_tiled_match_the_oracle(torch, ctx, orc, n, n_window, blocks):
    x = wf.bandlimited_noise(n, wf.rng_for(501, n))
    xd = dev(torch, x)
    h = (n_window - 1) // 2
    for a in ALPHAS:
        for n_out in (n, n + 37):
            if h > 0:
                ref = orc.doppler(x, a, h, "paper", n_out=n_out)
            else:
                # one tap at the nearest input: sinc(t - c) x[c] (half width 0 is the full sum there)
                t = a * np.arange(n_out)
                c = np.floor(t + 0.5).astype(np.int64)
                ok = (c >= 0) & (c < n)
                ref = np.where(ok, x.astype(np.complex128)[np.clip(c, 0, n - 1)] * np.sinc(t - c), 0)
            yd = host(ctx.correct_doppler_paper(xd, a, n_window, "direct", blocks=blocks, n_out=n_out))
            yt = host(ctx.correct_doppler_paper(xd, a, n_window, "tiled", blocks=blocks, n_out=n_out))
            assert np.array_equal(yd, yt), (n, n_window, a)
            if np.linalg.norm(ref) == 0:
                assert np.all(yd == 0)
            else:
                check(yd, ref, what=(n, n_window, a, n_out))


def test_paper_direct_matches_the_production_paper_window(torch, ctx):
    """Alg. 1 and correct_doppler with RC_WIN_PAPER compute the same operator."""
    import paper_2508_04951_amd as rc

    n = 1 << 19
    x = dev(torch, wf.bandlimited_noise(n, wf.rng_for(502, 0)))
    for v in (-8000.0, 1000.0, 7999.0):
        a = alpha_exact(v)
        y1 = host(ctx.correct_doppler_paper(x, a, 25, "direct"))
        y2 = host(ctx.correct_doppler(x, a, rc.Sinc(12, "paper")))
        check(y1, y2.astype(np.complex128), tol=1e-6, what=v)


@pytest.mark.parametrize("lut_size", [2, 300, 1251, 3000, 16384])
@pytest.mark.parametrize("n_window", [25, 41])
def test_paper_lut_matches_the_oracle(torch, ctx, orc, lut_size, n_window):
    n = 6007
    x = wf.bandlimited_noise(n, wf.rng_for(503, n))
    xd = dev(torch, x)
    h = (n_window - 1) // 2
    for a in ALPHAS:
        for blocks in (0, 2):
            y = host(ctx.correct_doppler_paper(xd, a, n_window, "lut", lut_size=lut_size, blocks=blocks))
            check(y, orc.doppler_lut(x, a, h, lut_size), what=(lut_size, n_window, a, blocks))


def test_paper_kernels_on_the_paper_setup_sampled(torch, ctx, orc):
    """2^19 samples, 25 taps (Fig 7, Fig 9 setup): every variant on sampled outputs."""
    n = 1 << 19
    x = wf.lfm_rf(n, 2.048e9, 413e6, 18e6)
    xd = dev(torch, x)
    a = alpha_exact(1000.0)
    idx = np.unique(np.concatenate([np.arange(64), np.linspace(0, n - 1, 3000).astype(np.int64), n - 1 - np.arange(64)]))
    ref = orc.doppler_at(x, idx, a, 12, "paper")
    for variant in ("direct", "tiled"):
        for blocks in (0, 32):
            y = host(ctx.correct_doppler_paper(xd, a, 25, variant, blocks=blocks))
            check(y[idx], ref, what=(variant, blocks))
    for lut_size in (300, 3000):
        full = orc.doppler_lut(x, a, 12, lut_size)
        for blocks in (0, 32):
            check(host(ctx.correct_doppler_paper(xd, a, 25, "lut", lut_size=lut_size, blocks=blocks)), full,
                  what=(lut_size, blocks))


# --- linear interpolation and frequency conversion -------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 999, 65536, 100003])
def test_linear_matches_the_oracle(torch, ctx, orc, n):
    x = wf.bandlimited_noise(n, wf.rng_for(504, n))
    xd = dev(torch, x)
    for a in ALPHAS:
        for n_out in (n, 2 * n + 3):
            check(host(ctx.correct_doppler_linear(xd, a, n_out=n_out)), orc.doppler_linear(x, a, n_out=n_out),
                  what=(n, a, n_out))


@pytest.mark.parametrize("n", [1, 1000, 1 << 20, (1 << 24) + 3])
def test_tone_matches_the_oracle_and_runs_in_place(torch, ctx, orc, n):
    x = (wf.rng_for(505, n).standard_normal((n, 2)) @ np.array([1.0, 1j])).astype(np.complex64)
    xd = dev(torch, x)
    for v, fr in ((-8000.0, 413e6), (7500.0, -2.5e6), (0.0, 1e9)):
        a = alpha_exact(v)
        ref = orc.doppler_tone(x, 10e6, a, fr)
        check(host(ctx.correct_doppler_tone(xd, 10e6, a, fr)), ref, what=(n, v))
    y = xd.clone()
    ctx.correct_doppler_tone(y, 10e6, alpha_exact(3000.0), 450e6, out=y)
    check(host(y), orc.doppler_tone(x, 10e6, alpha_exact(3000.0), 450e6))


# --- FFT P/Q resampling -------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 64, 1000, 4096, 65536, 102400, 300001])
def test_fft_pq_matches_the_oracle(torch, ctx, orc, n):
    x = wf.bandlimited_noise(n, wf.rng_for(506, n))
    xd = dev(torch, x)
    removes = [0, 2, 3, -2, -5, 6]
    for r in removes:
        if n - r < 2:
            continue
        a = n / (n - r) if r else 1.0
        for tone in (False, True):
            for n_out in (n, max(1, n - 7)):
                y = host(ctx.correct_doppler_fft_pq(xd, 200e6, a, f_ref=40e6, tone=tone, n_out=n_out))
                ref = orc.doppler_pq(x, 200e6, a, f_ref=40e6, tone=tone, n_out=n_out)
                check(y, ref, what=(n, r, tone, n_out))
    import paper_2508_04951_amd as rc

    for v in (-8000.0, 4000.0):
        assert rc.pq_length(n, alpha_exact(v)) == orc.pq_length(n, alpha_exact(v))


def test_methods_reject_bad_arguments(torch, ctx):
    import paper_2508_04951_amd as rc

    x = dev(torch, np.ones(100, np.complex64))
    with pytest.raises(ValueError):
        ctx.correct_doppler_paper(x, 1.1, 24)  # even window
    with pytest.raises(ValueError):
        ctx.correct_doppler_paper(x, 1.1, 25, "lut", lut_size=1)
    with pytest.raises(ValueError):
        ctx.correct_doppler_paper(x, -1.0, 25)
    with pytest.raises(rc.RcError):
        ctx.correct_doppler_paper(x, 50.0, 25, "tiled")  # span beyond 64 KiB of LDS
    with pytest.raises(ValueError):
        ctx.correct_doppler_linear(x, float("nan"))
    with pytest.raises(ValueError):
        ctx.correct_doppler_tone(x, 10e6, 1.0, float("inf"))
    with pytest.raises(rc.RcError):
        ctx.correct_doppler_fft_pq(dev(torch, np.ones(1, np.complex64)), 10e6, 1.0)
