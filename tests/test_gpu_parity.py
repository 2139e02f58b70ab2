"""GPU parity: the HIP path (through the C ABI) against the float64 oracle on the same
seeded complex64 inputs.

Tolerance: relative L2 error <= 1e-5 per pulse for the float32 paths (the accuracy bar of
the correction path; the float32 kernels land near 1e-7).  Exact special cases (alpha = 1,
integer alpha) are compared bit for bit.  Every alpha is the correctly rounded
(c + v)/(c - v), computed here with exact rationals and handed to both sides.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import waveforms as wf
from parity import TOL, check, rel_l2

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


def sinc(hw, window="kaiser", beta=8.0):
    import paper_2508_04951_amd as rc

    return rc.Sinc(hw, window, beta)


# --- Doppler --------------------------------------------------------------------------------

@pytest.mark.parametrize("n,hw,window", [(65536, 64, "kaiser"), (5000, 20, "paper"), (300, 0, "kaiser"),
                                         (777, 16, "rect")])
def test_doppler_alpha_one_is_bit_exact(torch, ctx, n, hw, window):
    x = wf.bandlimited_noise(n, wf.rng_for(101, n))
    y = host(ctx.correct_doppler(dev(torch, x), 1.0, sinc(hw, window)))
    assert np.array_equal(y, x)


@pytest.mark.parametrize("alpha", [2.0, 3.0])
def test_doppler_integer_alpha_is_bit_exact(torch, ctx, alpha):
    x = wf.bandlimited_noise(999, wf.rng_for(102, 0))
    y = host(ctx.correct_doppler(dev(torch, x), alpha, sinc(16)))
    a = int(alpha)
    exp = np.zeros(999, np.complex64)
    exp[: 998 // a + 1] = x[::a]
    assert np.array_equal(y, exp)


ALPHAS = [alpha_exact(8000.0), alpha_exact(-8000.0), alpha_exact(7500.0), 1 + 1e-6, 1 - 3e-7, 1.3, 0.77]
SINCS = [(64, "kaiser", 8.0), (128, "kaiser", 8.0), (8, "kaiser", 5.0), (16, "rect", 0.0), (20, "paper", 0.0),
         (0, "kaiser", 8.0)]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1000, 1025, 4096, 5000])
@pytest.mark.parametrize("sk", SINCS, ids=lambda s: f"{s[1]}{s[0]}")
def test_doppler_parity_grid(torch, ctx, orc, n, sk):
    hw, window, beta = sk
    x = wf.bandlimited_noise(n, wf.rng_for(103, n)) if n > 8 else \
        (wf.rng_for(103, n).standard_normal(n) + 1j).astype(np.complex64)
    xd = dev(torch, x)
    for alpha in ALPHAS:
        for n_out in sorted({n, n + 37, max(1, n // 2)}):
            y = host(ctx.correct_doppler(xd, alpha, sinc(hw, window, beta), n_out=n_out))
            ref = orc.doppler(x, alpha, hw, window, beta, n_out=n_out)
            check(y, ref, what=(n, n_out, alpha, sk))


@pytest.fixture
def engine(ctx, request):
    ctx.set_sinc_engine(request.param)
    yield request.param
    ctx.set_sinc_engine("auto")


@pytest.mark.parametrize("engine", ["auto", "valu"], indirect=True)
@pytest.mark.parametrize("v", [8000.0, -8000.0, 5000.0, -2500.0, 1e-3, -7.7, 9000.0, 14000.0])
@pytest.mark.parametrize("hw", [64, 128])
def test_doppler_fast_paths_at_pulse_length(torch, ctx, orc, engine, v, hw):
    """The matrix-core ("auto") and vector tile kernels at the batch pulse length 65536, with a
    ragged tail; 9 and 14 km/s leave the matrix-core range and take the vector kernel."""
    x = wf.batch_pulse(3)
    alpha = alpha_exact(v)
    for n_out in (65536, 65536 - 333, 70000):
        y = host(ctx.correct_doppler(dev(torch, x), alpha, sinc(hw), n_out=n_out))
        ref = orc.doppler(x, alpha, hw, "kaiser", 8.0, n_out=n_out)
        check(y, ref, what=(engine, v, hw, n_out))
        assert np.max(np.abs(y - ref)) <= 20 * TOL * np.sqrt(np.mean(np.abs(ref) ** 2))


def white(n, rng):
    """Full-band complex white noise (every DFT bin occupied, unit mean power)."""
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) * np.sqrt(0.5)).astype(np.complex64)


@pytest.mark.parametrize("engine", ["auto", "valu"], indirect=True)
@pytest.mark.parametrize("hw", [64, 128])
@pytest.mark.parametrize("kind", ["white", "tone+0.49", "tone-0.49", "tone+0.5"])
def test_doppler_full_band_inputs(torch, ctx, orc, engine, hw, kind):
    """The matrix-core and vector tile kernels on inputs that are not band-limited: full-band
    white noise and tones at +/-0.49 fs and at Nyquist (the drift polynomial's higher orders
    carry the most weight there)."""
    n = 65536
    if kind == "white":
        x = white(n, wf.rng_for(112, hw))
    else:
        x = np.exp(2j * np.pi * float(kind[4:]) * np.arange(n)).astype(np.complex64)
    xd = dev(torch, x)
    for v in (8000.0, -8000.0, 2345.0):
        alpha = alpha_exact(v)
        y = host(ctx.correct_doppler(xd, alpha, sinc(hw)))
        ref = orc.doppler(x, alpha, hw, "kaiser", 8.0)
        check(y, ref, what=(engine, hw, kind, v))


@pytest.mark.parametrize("engine", ["auto", "valu", "direct"], indirect=True)
@pytest.mark.parametrize("sk", SINCS + [(128, "kaiser", 8.0), (12, "paper", 0.0)], ids=lambda s: f"{s[1]}{s[0]}")
def test_doppler_impulse_response(torch, ctx, orc, engine, sk):
    """A unit impulse at n0: every output is the kernel itself at t - n0 (the oracle's tap sets
    are pinned by the same case against the definitions); impulses at the record's two ends
    and in the middle, at the bench's range rates and at a large dilation."""
    hw, window, beta = sk
    n = 4096
    for n0 in (0, 5, 2047, n - 1):
        x = np.zeros(n, np.complex64)
        x[n0] = 1 - 0.5j
        xd = dev(torch, x)
        for alpha in (alpha_exact(8000.0), alpha_exact(-5000.0), 1.0 + 1e-6, 1.37):
            y = host(ctx.correct_doppler(xd, alpha, sinc(hw, window, beta)))
            ref = orc.doppler(x, alpha, hw, window, beta)
            check(y, ref, what=(engine, sk, n0, alpha))


@pytest.mark.parametrize("engine", ["auto", "valu", "direct"], indirect=True)
def test_doppler_engines_on_small_and_scaled_inputs(torch, ctx, orc, engine):
    """Every engine on short pulses (a partial workgroup tile) and on inputs scaled far from
    unit power (the matrix-core path rescales by powers of two before its fp16 split)."""
    a = alpha_exact(-7000.0)
    for n, scale in [(100, 1.0), (1023, 1.0), (1025, 3e-9), (5000, 7e5), (3000, 0.0), (5000, 1e-30), (5000, 1e30)]:
        x = (wf.bandlimited_noise(n, wf.rng_for(110, n)) * np.float32(scale)).astype(np.complex64)
        y = host(ctx.correct_doppler(dev(torch, x), a, sinc(64)))
        ref = orc.doppler(x, a, 64, "kaiser", 8.0)
        if scale == 0.0:
            assert not np.any(y)
        else:
            check(y, ref, what=(engine, n, scale))


def test_doppler_long_pulse_sampled(torch, ctx, orc):
    """2^24 samples at +/-8 km/s (895 samples of accumulated shift, float64 positions):
    sampled outputs, including the far end, against the oracle."""
    n = 1 << 24
    x = wf.bandlimited_noise(n, wf.rng_for(104, 0))
    xd = dev(torch, x)
    idx = np.concatenate([np.arange(0, 2000), np.arange(n - 4000, n),
                          wf.rng_for(104, 1).integers(0, n, 4000)])
    for v in (8000.0, -8000.0):
        alpha = alpha_exact(v)
        y = host(ctx.correct_doppler(xd, alpha, sinc(128)))
        ref = orc.doppler_at(x, idx, alpha, 128, "kaiser", 8.0)
        check(y[idx], ref)


# --- Ionosphere -----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 256, 1024, 4096, 8192, 65536, 1 << 20])
@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_iono_parity(torch, ctx, orc, n, direction):
    x = wf.bandlimited_noise(n, wf.rng_for(105, n)) if n > 2 else np.array([1 + 2j, -0.5j][:n], np.complex64)
    for tec_tecu, fc, fs in [(50.0, 450e6, 10e6), (100.0, 450e6, 10e6), (5.0, 150e6, 10e6), (0.0, 450e6, 10e6),
                             (100.0, 0.0, 2.048e9)]:
        y = host(ctx.correct_ionosphere(dev(torch, x), fs, fc, tec_tecu * wf.TECU, direction))
        ref = orc.ionosphere(x, fs, fc, tec_tecu * wf.TECU, direction, naive=False)
        check(y, ref, what=(n, direction, tec_tecu, fc))


@pytest.mark.parametrize("n", [3, 5, 7, 12, 48, 1000, 4095, 4097, 5000, 65537, 100003, 300001])
@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_iono_parity_any_length(torch, ctx, orc, n, direction):
    """Lengths that are not powers of two (Bluestein at the power of two >= 2n - 1) against
    the oracle's N-point operator."""
    x = wf.bandlimited_noise(n, wf.rng_for(117, n))
    for tec_tecu, fc, fs in [(50.0, 450e6, 10e6), (5.0, 150e6, 10e6), (0.0, 450e6, 10e6), (100.0, 0.0, 2.048e9)]:
        y = host(ctx.correct_ionosphere(dev(torch, x), fs, fc, tec_tecu * wf.TECU, direction))
        ref = orc.ionosphere(x, fs, fc, tec_tecu * wf.TECU, direction, naive=n <= 5000)
        check(y, ref, what=(n, direction, tec_tecu, fc))


@pytest.mark.parametrize("n", [65536, 70001])
@pytest.mark.parametrize("scale", [1e-30, 1e30])
def test_iono_scaled_inputs(torch, ctx, orc, n, scale):
    """The float32 transforms keep their relative accuracy far from unit power (powers of two
    and Bluestein)."""
    x = (wf.bandlimited_noise(n, wf.rng_for(119, n)).astype(np.complex128) * scale).astype(np.complex64)
    y = host(ctx.correct_ionosphere(dev(torch, x), 10e6, 450e6, 60 * wf.TECU))
    ref = orc.ionosphere(x, 10e6, 450e6, 60 * wf.TECU, "correct", naive=False)
    check(y, ref, what=(n, scale))


def test_doppler_by_range_rate(torch, ctx):
    """correct_doppler(x, v_r=...) is correct_doppler(x, alpha_from_vr(v_r)), bit for bit."""
    import paper_2508_04951_amd as rc

    x = dev(torch, wf.bandlimited_noise(5000, wf.rng_for(121, 0)))
    a = host(ctx.correct_doppler(x, rc.alpha_from_vr(-6500.0), sinc(64)))
    b = host(ctx.correct_doppler(x, sinc=sinc(64), v_r=-6500.0))
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 1.0, sinc(64), v_r=10.0)


def test_memory_budget_caps_the_workspace(torch, orc):
    """A context capped at 1 MiB of workspace refuses a Bluestein transform that needs 4 MiB
    (RC_ERR_OUT_OF_MEMORY), still runs a power of two, and runs the Bluestein call once the
    cap is lifted."""
    import paper_2508_04951_amd as rc

    c = rc.Context(0)
    with pytest.raises(ValueError):
        c.set_mem_budget(-1)
    c.set_mem_budget(1 << 20)
    x = wf.bandlimited_noise(70001, wf.rng_for(120, 0))  # M = 2^18: 2 M complex64 = 4 MiB
    with pytest.raises(rc.RcError) as ei:
        c.correct_ionosphere(dev(torch, x), 10e6, 450e6, 60 * wf.TECU)
    assert ei.value.status == 3
    p2 = wf.bandlimited_noise(4096, wf.rng_for(120, 1))
    y2 = host(c.correct_ionosphere(dev(torch, p2), 10e6, 450e6, 60 * wf.TECU))
    check(y2, orc.ionosphere(p2, 10e6, 450e6, 60 * wf.TECU))
    c.set_mem_budget(0)
    y = host(c.correct_ionosphere(dev(torch, x), 10e6, 450e6, 60 * wf.TECU))
    check(y, orc.ionosphere(x, 10e6, 450e6, 60 * wf.TECU, naive=False))


def test_iono_any_length_in_place_and_round_trip(torch, ctx, orc):
    """Bluestein in place equals out of place bit for bit; at 2^22 + 12345 (the longest serving
    lengths) distort then correct is the identity and the norm is kept."""
    x = wf.bandlimited_noise(70001, wf.rng_for(118, 0))
    xd = dev(torch, x)
    y = host(ctx.correct_ionosphere(xd, 10e6, 450e6, 60 * wf.TECU))
    ctx.correct_ionosphere(xd, 10e6, 450e6, 60 * wf.TECU, out=xd)
    assert np.array_equal(host(xd), y)
    n = (1 << 22) + 12345
    x = wf.bandlimited_noise(n, wf.rng_for(118, 1))
    xd = dev(torch, x)
    d = ctx.correct_ionosphere(xd, 10e6, 450e6, 90 * wf.TECU, "distort")
    z = host(ctx.correct_ionosphere(d, 10e6, 450e6, 90 * wf.TECU, "correct"))
    check(z, x, tol=2 * TOL)
    assert abs(np.linalg.norm(host(d)) / np.linalg.norm(x) - 1) <= 1e-5


def test_iono_in_place(torch, ctx, orc):
    x = wf.bandlimited_noise(65536, wf.rng_for(106, 0))
    xd = dev(torch, x)
    ctx.correct_ionosphere(xd, 10e6, 450e6, 70 * wf.TECU, "correct", out=xd)
    ref = orc.ionosphere(x, 10e6, 450e6, 70 * wf.TECU, "correct", naive=False)
    check(host(xd), ref)


CARRIER_ZERO = [(1 << 16, 10e6, 100.0), (1 << 22, 10e6, 100.0), (1 << 22, 10e6, 5.0), (1 << 21, 2.048e9, 100.0),
                (70001, 10e6, 100.0), (4097, 10e6, 100.0)]


@pytest.mark.parametrize("n,fs,tec_tecu", CARRIER_ZERO, ids=lambda v: str(v))
@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_iono_carrier_zero(torch, ctx, orc, n, fs, tec_tecu, direction):
    """A carrier of 0 Hz (the RF-sampled setup of Sec. II-C) puts bins within a few hertz of
    f = 0, where the phase 4 pi K2 / (c f) reaches ~1e12 rad: the quarter-turn count must be
    taken exactly and the quotient carried to float64 accuracy.  White noise (every bin
    occupied) and a tone in the lowest positive bin."""
    x = (wf.rng_for(171, n).standard_normal((n, 2)) @ np.array([1.0, 1j])).astype(np.complex64)
    y = host(ctx.correct_ionosphere(dev(torch, x), fs, 0.0, tec_tecu * wf.TECU, direction))
    ref = orc.ionosphere(x, fs, 0.0, tec_tecu * wf.TECU, direction, naive=False)
    check(y, ref, what=(n, fs, tec_tecu, direction))
    tone = np.exp(2j * np.pi * np.arange(n) / n).astype(np.complex64)
    y = host(ctx.correct_ionosphere(dev(torch, tone), fs, 0.0, tec_tecu * wf.TECU, direction))
    ref = orc.ionosphere(tone, fs, 0.0, tec_tecu * wf.TECU, direction, naive=False)
    check(y, ref, what=(n, fs, tec_tecu, direction, "tone"))


def test_iono_at_2_24_against_the_oracle(torch, ctx, orc):
    """The long-dwell length 2^24 against the oracle's float64 FFT path, at a 450 MHz carrier
    and at carrier 0 (10 MHz sampling: the lowest bin at 0.6 Hz)."""
    n = 1 << 24
    x = wf.bandlimited_noise(n, wf.rng_for(107, 1))
    xd = dev(torch, x)
    for fc in (450e6, 0.0):
        y = host(ctx.correct_ionosphere(xd, 10e6, fc, 100 * wf.TECU, "correct"))
        ref = orc.ionosphere(x, 10e6, fc, 100 * wf.TECU, "correct", naive=False)
        check(y, ref, what=fc)


def test_iono_round_trip_and_norm_at_2_24(torch, ctx):
    """Full long-dwell length: distort then correct returns the input; the operator is unitary."""
    n = 1 << 24
    x = wf.bandlimited_noise(n, wf.rng_for(107, 0))
    xd = dev(torch, x)
    d = ctx.correct_ionosphere(xd, 10e6, 450e6, 100 * wf.TECU, "distort")
    dn = host(d)
    back = host(ctx.correct_ionosphere(d, 10e6, 450e6, 100 * wf.TECU, "correct"))
    check(back, x)
    assert np.linalg.norm(dn.astype(np.complex128)) == pytest.approx(np.linalg.norm(x.astype(np.complex128)), rel=1e-5)


def test_iono_sampled_bins_at_2_22(torch, ctx, orc):
    """2^22 samples against the oracle's float64 FFT path."""
    n = 1 << 22
    x = wf.bandlimited_noise(n, wf.rng_for(108, 0))
    y = host(ctx.correct_ionosphere(dev(torch, x), 10e6, 450e6, 60 * wf.TECU, "correct"))
    ref = orc.ionosphere(x, 10e6, 450e6, 60 * wf.TECU, "correct", naive=False)
    check(y, ref)


# --- Whole path -----------------------------------------------------------------------------

def test_c1_single_lfm_pulse(torch, ctx, orc):
    """Single LFM pulse, N = 4096, fs = 10 MHz, B = 5 MHz, v_r = +7.5 km/s, full sinc,
    then ionospheric correction at 50 TECU, carrier 450 MHz."""
    import paper_2508_04951_amd as rc

    c = wf.SINGLE_LFM
    x = wf.lfm(c["n"], c["fs"], c["bandwidth"])
    alpha = alpha_exact(c["v_r"])
    ref = orc.correct_pulse(x, c["fs"], alpha, c["tec"], c["carrier"], half_width=0, naive=True)
    xd = dev(torch, x)
    r = ctx.correct_doppler(xd, alpha, rc.Sinc(0))
    y1 = host(ctx.correct_ionosphere(r, c["fs"], c["carrier"], c["tec"], "correct"))
    check(y1, ref)
    yd = torch.empty_like(xd)
    ctx.correct_pulse_batch(xd, yd, [dict(off_in=0, n_in=4096, off_out=0, n_out=4096, fs=c["fs"], alpha=alpha,
                                          tec=c["tec"], carrier=c["carrier"])], rc.Sinc(0))
    assert np.array_equal(host(yd), y1)


def _ragged_batch():
    """Pulses of mixed length, alpha, TEC, flags and direction, packed with gaps."""
    rng = wf.rng_for(109, 0)
    specs = [(65536, 3), (4096, 3), (8192, 1), (1000, 1), (65536, 2), (256, 3), (1 << 17, 3), (4096, 2),
             (3000, 1), (16, 3), (5000, 3), (70001, 2), (12, 3), (70001, 3)]
    pulses, xs = [], []
    off_in = off_out = 5
    for i, (n, flags) in enumerate(specs):
        x = wf.bandlimited_noise(n, wf.rng_for(109, i + 1))
        v = rng.uniform(-8000, 8000) if i != 7 else 1.2e6  # one pulse off the fast path
        p = dict(off_in=off_in, n_in=n, off_out=off_out, n_out=n, fs=10e6, alpha=alpha_exact(v),
                 tec=rng.uniform(5, 100) * wf.TECU, carrier=450e6, flags=flags,
                 direction="distort" if i % 4 == 3 else "correct")
        pulses.append(p)
        xs.append(x)
        off_in += n + 3
        off_out += n + 11
    return pulses, xs, off_in, off_out


def test_batch_matches_oracle_and_single_calls(torch, ctx, orc):
    import paper_2508_04951_amd as rc

    pulses, xs, x_len, y_len = _ragged_batch()
    xp = np.zeros(x_len, np.complex64)
    for p, x in zip(pulses, xs):
        xp[p["off_in"]:p["off_in"] + p["n_in"]] = x
    xd = dev(torch, xp)
    yd = torch.full((y_len,), complex("nan"), dtype=torch.complex64, device="cuda")
    ctx.correct_pulse_batch(xd, yd, pulses, rc.Sinc(64))
    yb = host(yd)
    for i, (p, x) in enumerate(zip(pulses, xs)):
        got = yb[p["off_out"]:p["off_out"] + p["n_out"]]
        assert not np.isnan(got).any(), i
        ref = orc.correct_pulse(x, p["fs"], p["alpha"], p["tec"], p["carrier"], n_out=p["n_out"],
                                doppler_on=bool(p["flags"] & 1), iono_on=bool(p["flags"] & 2),
                                direction=p["direction"], half_width=64)
        check(got, ref, what=(i))
        # the same pulse alone, through the single-pulse entry points: bit-identical
        xi = dev(torch, x)
        r = ctx.correct_doppler(xi, p["alpha"], rc.Sinc(64)) if p["flags"] & 1 else xi
        if p["flags"] & 2:
            r = ctx.correct_ionosphere(r, p["fs"], p["carrier"], p["tec"], p["direction"])
        assert np.array_equal(host(r), got), i
    gaps = np.ones(y_len, bool)
    for p in pulses:
        gaps[p["off_out"]:p["off_out"] + p["n_out"]] = False
    assert np.isnan(yb[gaps]).all()  # nothing written outside the pulses


def test_batch_bluestein_chunks(torch, ctx, orc):
    """Ionosphere-only pulses whose lengths are not powers of two: five that share the 2^23
    convolution length (128 MiB of workspace each, so the batch runs them as chunks of two,
    two and one) and three that share 2^13, in one call.  Each against the oracle and, bit
    for bit, against the single-pulse entry point."""
    import paper_2508_04951_amd as rc

    lens = [4194303, 4100000, 4194000, 4150001, 4194301, 4097, 4100, 6000]
    rng = wf.rng_for(131, 0)
    pulses, xs, off = [], [], 0
    for i, n in enumerate(lens):
        xs.append(wf.bandlimited_noise(n, wf.rng_for(131, i + 1)))
        pulses.append(dict(off_in=off, n_in=n, off_out=off, n_out=n, fs=10e6, alpha=1.0,
                           tec=float(rng.uniform(5, 100)) * wf.TECU, carrier=450e6, flags=rc.DO_IONO,
                           direction="distort" if i % 3 == 2 else "correct"))
        off += n + 64
    xp = np.zeros(off, np.complex64)
    for p, x in zip(pulses, xs):
        xp[p["off_in"]:p["off_in"] + p["n_in"]] = x
    xd = dev(torch, xp)
    yd = torch.full((off,), complex("nan"), dtype=torch.complex64, device="cuda")
    ctx.correct_pulse_batch(xd, yd, pulses, rc.Sinc(64))
    yb = host(yd)
    for i, (p, x) in enumerate(zip(pulses, xs)):
        got = yb[p["off_out"]:p["off_out"] + p["n_out"]]
        ref = orc.ionosphere(x, p["fs"], p["carrier"], p["tec"], p["direction"])
        check(got, ref, what=(i))
        one = host(ctx.correct_ionosphere(dev(torch, x), p["fs"], p["carrier"], p["tec"], p["direction"]))
        assert np.array_equal(one, got), i


def test_batch_from_a_pulse_table_is_bit_identical(torch, ctx):
    """The same ragged batch described by a pulse_table array instead of dicts."""
    import paper_2508_04951_amd as rc

    pulses, xs, x_len, y_len = _ragged_batch()
    xp = np.zeros(x_len, np.complex64)
    for p, x in zip(pulses, xs):
        xp[p["off_in"]:p["off_in"] + p["n_in"]] = x
    xd = dev(torch, xp)
    col = lambda k: np.array([p[k] for p in pulses])
    table = rc.pulse_table(col("off_in"), col("n_in"), col("off_out"), col("n_out"), col("fs"), alpha=col("alpha"),
                           tec=col("tec"), carrier=col("carrier"), flags=col("flags"),
                           direction=np.array([rc.DIRECTIONS[d] for d in col("direction")]))
    outs = []
    for desc in (pulses, table):
        yd = torch.full((y_len,), complex("nan"), dtype=torch.complex64, device="cuda")
        ctx.correct_pulse_batch(xd, yd, desc, rc.Sinc(64))
        outs.append(host(yd))
    assert np.array_equal(outs[0], outs[1], equal_nan=True)


def test_batch_c2_full_size_sampled(torch, ctx, orc):
    """The full batch workload (1024 pulses x 65536, Kaiser H = 64, beta = 8) in one call;
    four seeded pulses compared in full against the oracle, all pulses finite."""
    import paper_2508_04951_amd as rc

    c = wf.BATCH
    n, P = c["n"], c["pulses"]
    v, e = wf.batch_params()
    x = np.empty(P * n, np.complex64)
    for p in range(P):
        x[p * n:(p + 1) * n] = wf.batch_pulse(p)
    pulses = [dict(off_in=p * n, n_in=n, off_out=p * n, n_out=n, fs=c["fs"], alpha=alpha_exact(v[p]),
                   tec=e[p], carrier=c["carrier"]) for p in range(P)]
    xd = dev(torch, x)
    yd = torch.empty_like(xd)
    ctx.correct_pulse_batch(xd, yd, pulses, rc.Sinc(64, "kaiser", 8.0))
    y = host(yd)
    assert np.isfinite(y.view(np.float32)).all()
    for p in (0, 1, 511, 1023):
        ref = orc.correct_pulse(x[p * n:(p + 1) * n], c["fs"], pulses[p]["alpha"], e[p], c["carrier"],
                                half_width=64, beta=8.0)
        check(y[p * n:(p + 1) * n], ref, what=p)


def test_batch_tile_list_matches_single_calls(torch, ctx, orc):
    """A ragged batch with more 2048-output matrix-core tiles than resident workgroups (the
    persistent path over the tile list sorted by phase): every pulse equals, bit for bit, its
    single-pulse call (one workgroup per tile), and sampled pulses match the oracle."""
    import paper_2508_04951_amd as rc

    rng = wf.rng_for(131, 0)
    lens = [int(n) for n in rng.integers(1, 120000, size=40)] + [1, 2047, 2048, 2049, 1 << 17]
    pulses, xs = [], []
    off_in = off_out = 3
    for i, n in enumerate(lens):
        v = rng.uniform(-8800, 8800) if i % 9 else rng.uniform(9000, 12000)  # a few off the matrix cores
        pulses.append(dict(off_in=off_in, n_in=n, off_out=off_out, n_out=n, fs=10e6, alpha=alpha_exact(v),
                           tec=0.0, carrier=450e6, flags=1))
        xs.append(wf.bandlimited_noise(n, wf.rng_for(131, i + 1)) if n > 1 else np.ones(1, np.complex64))
        off_in += n + 7
        off_out += n + 1
    assert sum((n + 2047) // 2048 for n in lens) > 1100  # above any resident grid of 256 CUs x 4
    xp = np.zeros(off_in, np.complex64)
    for p, x in zip(pulses, xs):
        xp[p["off_in"]:p["off_in"] + p["n_in"]] = x
    xd = dev(torch, xp)
    yd = torch.full((off_out,), complex("nan"), dtype=torch.complex64, device="cuda")
    k = rc.Sinc(64, "kaiser", 8.0)
    ctx.correct_pulse_batch(xd, yd, pulses, k)
    yb = host(yd)
    gaps = np.ones(off_out, bool)
    for i, (p, x) in enumerate(zip(pulses, xs)):
        got = yb[p["off_out"]:p["off_out"] + p["n_out"]]
        gaps[p["off_out"]:p["off_out"] + p["n_out"]] = False
        single = host(ctx.correct_doppler(dev(torch, x), p["alpha"], k))
        assert np.array_equal(single, got), i
        if i in (0, 5, 40, 43, 44):
            ref = orc.doppler(x, p["alpha"], 64, "kaiser", 8.0)
            check(got, ref, what=(i))
    assert np.isnan(yb[gaps]).all()


def test_repeat_runs_are_bit_identical(torch, ctx):
    import paper_2508_04951_amd as rc

    x = dev(torch, wf.batch_pulse(7))
    a = alpha_exact(-6543.0)
    y1 = host(ctx.correct_ionosphere(ctx.correct_doppler(x, a, rc.Sinc(64)), 10e6, 450e6, 30 * wf.TECU))
    y2 = host(ctx.correct_ionosphere(ctx.correct_doppler(x, a, rc.Sinc(64)), 10e6, 450e6, 30 * wf.TECU))
    assert np.array_equal(y1, y2)


# --- Argument validation ---------------------------------------------------------------------

def test_invalid_arguments_are_rejected(torch, ctx):
    import paper_2508_04951_amd as rc

    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    y = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 0.0)
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, float("nan"))
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 1.0, rc.Sinc(-1))
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 1.0, fs=0.0)
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 1.0, out=x)  # x and y overlap
    with pytest.raises(ValueError):
        ctx.correct_ionosphere(x, 10e6, 450e6, -1.0)
    with pytest.raises(ValueError):
        ctx.correct_ionosphere(x[1:], 10e6, 450e6, 1e17, out=x[:-1])  # partial overlap
    big = torch.zeros((1 << 23) + 1, dtype=torch.complex64, device="cuda")
    with pytest.raises(rc.RcError) as ei:
        ctx.correct_ionosphere(big, 10e6, 450e6, 1e17)
    assert ei.value.status == 2  # RC_ERR_UNSUPPORTED (Bluestein would need m > 2^24)
    del big
    ok = dict(off_in=0, n_in=32, off_out=0, n_out=32, fs=10e6, alpha=1.0, tec=1e17, carrier=450e6)
    with pytest.raises(ValueError):
        ctx.correct_pulse_batch(x, y, [dict(ok, off_in=40)])  # past the end of x
    with pytest.raises(ValueError):
        ctx.correct_pulse_batch(x, y, [ok, dict(ok, off_out=16)])  # overlapping outputs
    with pytest.raises(ValueError):
        ctx.correct_pulse_batch(x, x, [ok])  # in-place batch
    with pytest.raises(ValueError):
        ctx.correct_pulse_batch(x, y, [dict(ok, flags=2, n_out=16)])  # length change without Doppler
    ctx.correct_pulse_batch(x, y, [ok])
    ctx.sync()


def test_empty_batches_and_zero_lengths(torch, ctx):
    """A batch of no pulses does nothing; a pulse or call of length 0 is an argument error."""
    import paper_2508_04951_amd as rc

    x = torch.ones(64, dtype=torch.complex64, device="cuda")
    y = torch.full((64,), complex("nan"), dtype=torch.complex64, device="cuda")
    ctx.correct_pulse_batch(x, y, [])
    ctx.correct_pulse_batch(x, y, rc.pulse_table([], [], [], [], []))
    assert torch.isnan(y).all().item()
    ok = dict(off_in=0, n_in=32, off_out=0, n_out=32, fs=10e6, alpha=1.0, tec=1e17, carrier=450e6)
    for bad in (dict(ok, n_in=0), dict(ok, n_out=0), dict(ok, n_in=0, n_out=0, flags=rc.DO_IONO)):
        with pytest.raises(ValueError):
            ctx.correct_pulse_batch(x, y, [bad])
    with pytest.raises(ValueError):
        ctx.correct_doppler(x[:0], 1.0)
    with pytest.raises(ValueError):
        ctx.correct_doppler(x, 1.0, n_out=0)
    with pytest.raises(ValueError):
        ctx.correct_ionosphere(x[:0], 10e6, 450e6, 1e17)
    ctx.sync()
    assert torch.isnan(y).all().item()
