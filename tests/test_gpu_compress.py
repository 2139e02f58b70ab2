"""GPU parity of pulse compression with the ionospheric correction in the same frequency-domain
pass (replica_spectrum + compress_pulse, through the C ABI) against the float64 oracle.

Tolerance: relative L2 error <= 1e-5 per pulse, as for the other float32 paths.
"""
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


@pytest.mark.parametrize("n,n_rep", [(16, 5), (256, 256), (4096, 1000), (8192, 3000), (65536, 20000),
                                     (1 << 19, 204800), (1 << 20, 1000),
                                     # other lengths: Bluestein, the correlation in its middle step
                                     (3, 2), (1000, 300), (3001, 3001), (65537, 20000), (300001, 100000)])
@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_compress_matches_oracle(torch, ctx, orc, n, n_rep, direction):
    x = wf.bandlimited_noise(n, wf.rng_for(161, n))
    r = wf.lfm(n_rep, 10e6, 5e6)
    spec = ctx.replica_spectrum(dev(torch, r), n)
    for tec_tecu, fc, fs in [(50.0, 450e6, 10e6), (0.0, 450e6, 10e6), (100.0, 0.0, 2.048e9)]:
        y = host(ctx.compress_pulse(dev(torch, x), spec, fs, fc, tec_tecu * wf.TECU, direction))
        ref = orc.compress(x, r, fs, fc, tec_tecu * wf.TECU, direction, naive=n <= 4096)
        check(y, ref, what=(n, n_rep, direction, tec_tecu))


@pytest.mark.parametrize("n,n_rep", [(1 << 16, 5000), (70001, 3000)])
@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_compress_carrier_zero(torch, ctx, orc, n, n_rep, direction):
    """Carrier 0 Hz at 10 MHz sampling: bins a few hundred hertz from f = 0 carry phases of
    ~1e10 rad, in the row pass (2^16) and in Bluestein's middle step (70001)."""
    x = (wf.rng_for(164, n).standard_normal((n, 2)) @ np.array([1.0, 1j])).astype(np.complex64)
    r = wf.lfm(n_rep, 10e6, 5e6)
    spec = ctx.replica_spectrum(dev(torch, r), n)
    y = host(ctx.compress_pulse(dev(torch, x), spec, 10e6, 0.0, 100 * wf.TECU, direction))
    ref = orc.compress(x, r, 10e6, 0.0, 100 * wf.TECU, direction, naive=False)
    check(y, ref, what=(n, direction))


def test_unit_replica_without_ionosphere_is_identity(torch, ctx):
    n = 1 << 16
    x = dev(torch, wf.bandlimited_noise(n, wf.rng_for(162, 0)))
    spec = ctx.replica_spectrum(dev(torch, np.ones(1, np.complex64)), n)
    y = host(ctx.compress_pulse(x, spec, 10e6, 450e6, 0.0))
    assert rel_l2(y, host(x)) <= 1e-6


def test_in_place_and_one_spectrum_for_many_pulses(torch, ctx, orc):
    n = 1 << 16
    r = wf.lfm(5000, 10e6, 5e6)
    spec = ctx.replica_spectrum(dev(torch, r), n)
    for p in range(3):
        x = wf.bandlimited_noise(n, wf.rng_for(163, p))
        tec = (20.0 + 30 * p) * wf.TECU
        xd = dev(torch, x)
        y = ctx.compress_pulse(xd, spec, 10e6, 450e6, tec, out=xd)
        assert y.data_ptr() == xd.data_ptr()
        check(host(y), orc.compress(x, r, 10e6, 450e6, tec), what=p)


def test_replica_from_correct_doppler(torch, ctx, orc):
    """The paper's chain: the replica is the transmitted LFM dilated by correct_doppler; the
    received echo is that replica delayed and dispersed by the ionosphere; compressing with the
    correction puts the peak back at the delay."""
    import paper_2508_04951_amd as rc

    n, n_rep, fs, fc, tec, delay = 1 << 18, 60000, 10e6, 150e6, 100 * wf.TECU, 12345
    tx = dev(torch, wf.lfm(n_rep, fs, 5e6))
    rep = ctx.correct_doppler(tx, alpha_exact(6000.0), rc.Sinc(64))
    rep_h = host(rep)
    echo = np.zeros(n, np.complex64)
    echo[delay:delay + n_rep] = rep_h
    rx = host(ctx.correct_ionosphere(dev(torch, echo), fs, fc, tec, "distort"))
    spec = ctx.replica_spectrum(rep, n)
    y = host(ctx.compress_pulse(dev(torch, rx), spec, fs, fc, tec, "correct"))
    ref = orc.compress(rx, rep_h, fs, fc, tec, "correct")
    check(y, ref)
    assert int(np.argmax(np.abs(y))) == delay
    uncorrected = host(ctx.compress_pulse(dev(torch, rx), spec, fs, fc, 0.0))
    assert np.abs(y).max() > 1.5 * np.abs(uncorrected).max()  # dispersion smears the peak


def test_compress_argument_errors(torch, ctx):
    import paper_2508_04951_amd as rc

    r = torch.ones(16, dtype=torch.complex64, device="cuda")
    with pytest.raises(rc.RcError) as ei:
        ctx.replica_spectrum(r, (1 << 23) + 1)  # other lengths stop at 2^23
    assert ei.value.status == 2
    with pytest.raises(ValueError):
        ctx.replica_spectrum(r, 8)  # replica longer than n
    spec = ctx.replica_spectrum(r, 1024)
    x = torch.zeros(1024, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ctx.compress_pulse(x, spec, 10e6, 450e6, 1e17, out=spec)  # y overlaps the spectrum
    with pytest.raises(ValueError):
        ctx.compress_pulse(x, spec, 0.0, 450e6, 1e17)
    with pytest.raises(ValueError):
        ctx.compress_pulse(x, spec, 10e6, 450e6, -1.0)
    ctx.sync()
