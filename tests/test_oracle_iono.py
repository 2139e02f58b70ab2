"""Pins of the float64 oracle's ionospheric operator and transforms against facts the
paper and the mathematics fix (no GPU).

Delay model: Eq (3) with App. A (tau(f) = K2/(c f^2), K2 = e^2 E/(8 pi^2 m_e eps0));
operator: Eq (15) (distortion, +) and Eq (16) (correction, -); Fourier convention of
Sec. II-B (g_hat(f) = int g(t) exp(-2 pi i t f) dt, so a delay t0 multiplies by
exp(-2 pi i t0 f)).
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

import waveforms as wf

FS = 10e6
FC = 450e6


def _phi(tec):
    """4 pi K2 / c with K2 from scipy's CODATA constants (independent of the oracle)."""
    k2 = sc.e ** 2 / (8 * math.pi ** 2 * sc.m_e * sc.epsilon_0) * tec
    return 4 * math.pi * k2 / sc.c


def test_k2_constant_vs_scipy(orc):
    ref = sc.e ** 2 / (8 * math.pi ** 2 * sc.m_e * sc.epsilon_0)
    assert orc.k2_per_tec() == pytest.approx(ref, rel=1e-13)
    assert orc.k2_per_tec() == pytest.approx(40.308, rel=1e-4)  # the textbook 40.3 m^3/s^2


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 100, 1000])
def test_naive_dft_vs_numpy(orc, n):
    rng = wf.rng_for(21, n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = orc.dft(x)
    np.testing.assert_allclose(X, np.fft.fft(x), rtol=0, atol=1e-12 * max(1, np.abs(X).max()))
    np.testing.assert_allclose(orc.dft(x, +1), np.fft.ifft(x) * n, rtol=0,
                               atol=1e-12 * max(1, np.abs(X).max()))


@pytest.mark.parametrize("n", [1, 2, 5, 12, 64, 97, 1000, 4096, 3 * 1024])
def test_fft_vs_dft_and_numpy(orc, n):
    rng = wf.rng_for(22, n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = orc.fft(x)
    scale = max(1.0, np.abs(X).max())
    np.testing.assert_allclose(X, np.fft.fft(x), rtol=0, atol=1e-12 * scale)
    if n <= 1000:
        np.testing.assert_allclose(X, orc.dft(x), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(orc.fft(x, +1), np.fft.ifft(x) * n, rtol=0, atol=1e-12 * scale)


def test_parseval(orc):
    x = wf.bandlimited_noise(1000, wf.rng_for(23, 0)).astype(np.complex128)
    X = orc.fft(x)
    assert np.sum(np.abs(x) ** 2) == pytest.approx(np.sum(np.abs(X) ** 2) / x.size, rel=1e-13)


@pytest.mark.parametrize("n", [1, 2, 7, 8, 4096, 4097])
def test_bin_frequency_is_numpy_fftfreq(orc, n):
    ks = sorted({0, 1, n // 2, (n + 1) // 2, n - 1} & set(range(n)))
    ref = FC + FS * np.fft.fftfreq(n)
    for k in ks:
        assert orc.bin_frequency(k, n, FS, FC) == pytest.approx(ref[k], rel=1e-15)


@pytest.mark.parametrize("n,k0", [(4096, 0), (4096, 5), (4096, 2048), (4096, 4093), (1000, 501), (97, 48)])
@pytest.mark.parametrize("direction,sign", [("correct", -1.0), ("distort", +1.0)])
def test_single_bin_tone_gets_exact_phase(orc, n, k0, direction, sign):
    """A tone on bin k0 passes through Eq (15)/(16) as y = exp(+/- i 4 pi K2/(c f_k0)) x,
    f_k0 the RF frequency of that bin (negative and Nyquist bins included)."""
    tec = 50 * wf.TECU
    x = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    f = FC + FS * np.fft.fftfreq(n)[k0]
    expected = np.exp(1j * sign * _phi(tec) / f) * x
    y = orc.ionosphere(x, FS, FC, tec, direction)
    np.testing.assert_allclose(y, expected, rtol=0, atol=1e-11)


CODATA = dict(e="1.602176634e-19", m_e="9.1093837139e-31", eps0="8.8541878188e-12", c="299792458")


@pytest.mark.parametrize("n,fs,carrier,tec_tecu", [(1 << 22, 10e6, 0.0, 100.0), (1 << 24, 10e6, 0.0, 100.0),
                                                   (70001, 10e6, 0.0, 100.0), ((1 << 22) + 12345, 10e6, 0.0, 5.0),
                                                   (1 << 21, 2.048e9, 0.0, 100.0), (4096, 10e6, 4.99e6, 100.0),
                                                   (1 << 16, 10e6, 450e6, 50.0)])
def test_large_phases_against_multiprecision(orc, n, fs, carrier, tec_tecu):
    """With the carrier below fs/2 the lowest bins sit a few hertz from f = 0 and the phase
    4 pi K2/(c f) of Eq (15)/(16) reaches ~1e12 rad.  The oracle's response there matches the
    same formula evaluated with 50-digit arithmetic (mpmath) on the same double inputs and the
    CODATA decimal constants, reduced mod 2 pi, to 1e-6 rad; a float64 quotient would miss by
    ~1e-4 rad at the largest of these phases."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    tec = tec_tecu * wf.TECU
    H = orc.iono_response(n, fs, carrier, tec, "correct")
    k2 = mp.mpf(CODATA["e"]) ** 2 / (8 * mp.pi ** 2 * mp.mpf(CODATA["m_e"]) * mp.mpf(CODATA["eps0"])) * mp.mpf(tec)
    worst = 0.0
    for k in sorted({1, 2, 3, n // 2 - 1, n // 2, n - 1, n - 2, n // 3}):
        kk = k if k < (n + 1) // 2 else k - n
        f = mp.mpf(carrier) + mp.mpf(fs) * kk / n
        phi = -4 * mp.pi * k2 / (mp.mpf(CODATA["c"]) * f)
        ref = float(phi - 2 * mp.pi * mp.nint(phi / (2 * mp.pi)))
        got = float(np.angle(H[k]))
        d = abs((got - ref + np.pi) % (2 * np.pi) - np.pi)
        worst = max(worst, d)
        assert abs(abs(H[k]) - 1.0) < 1e-15
    assert worst <= 1e-6, worst


def test_zero_frequency_bin_is_left_alone(orc):
    """With the carrier at 0 (RF-sampled data) the DC bin has f = 0; its response is 1."""
    n = 64
    x = np.ones(n, dtype=np.complex128)
    y = orc.ionosphere(x, 2.048e9, 0.0, 1e18, "correct")
    np.testing.assert_allclose(y, x, atol=1e-13)


def test_distort_then_correct_is_identity(orc):
    x = wf.bandlimited_noise(4096, wf.rng_for(24, 0)).astype(np.complex128)
    tec = 100 * wf.TECU
    back = orc.ionosphere(orc.ionosphere(x, FS, FC, tec, "distort"), FS, FC, tec, "correct")
    assert np.linalg.norm(back - x) / np.linalg.norm(x) < 1e-13


def test_norm_is_preserved(orc):
    x = wf.bandlimited_noise(3000, wf.rng_for(25, 0)).astype(np.complex128)
    y = orc.ionosphere(x, FS, FC, 73 * wf.TECU, "correct")
    assert np.linalg.norm(y) == pytest.approx(np.linalg.norm(x), rel=1e-13)


def test_zero_tec_is_identity(orc):
    x = wf.bandlimited_noise(512, wf.rng_for(26, 0)).astype(np.complex128)
    np.testing.assert_allclose(orc.ionosphere(x, FS, FC, 0.0), x, atol=1e-14)


def test_tec_is_additive(orc):
    x = wf.bandlimited_noise(2048, wf.rng_for(27, 0)).astype(np.complex128)
    e1, e2 = 20 * wf.TECU, 35 * wf.TECU
    two = orc.ionosphere(orc.ionosphere(x, FS, FC, e1), FS, FC, e2)
    one = orc.ionosphere(x, FS, FC, e1 + e2)
    # the phases are ~2000 rad, whose float64 spacing is 4.5e-13 rad
    assert np.linalg.norm(two - one) / np.linalg.norm(one) < 2e-12


@pytest.mark.parametrize("f1", [0.0, 2e6, -3e6])
def test_distortion_delays_envelope_by_two_way_group_delay(orc, f1):
    """Eq (3) and the two-way factor: a narrowband Gaussian pulse at RF frequency
    f = carrier + f1 comes out of Eq (15) delayed by 2 tau(f) = 2 K2/(c f^2)
    (6.6 samples at 50 TECU, 450 MHz, 10 MHz sampling)."""
    n, tec = 4096, 50 * wf.TECU
    k = np.arange(n)
    x = np.exp(-0.5 * ((k - 1500.0) / 120.0) ** 2) * np.exp(2j * np.pi * f1 / FS * k)
    y = orc.ionosphere(x, FS, FC, tec, "distort", naive=False)
    k2 = sc.e ** 2 / (8 * math.pi ** 2 * sc.m_e * sc.epsilon_0) * tec
    expected = 2 * k2 / (sc.c * (FC + f1) ** 2) * FS
    shift = np.sum(k * np.abs(y) ** 2) / np.sum(np.abs(y) ** 2) - 1500.0
    assert shift == pytest.approx(expected, rel=2e-3)


def test_naive_and_fast_transforms_agree(orc):
    x = wf.bandlimited_noise(1536, wf.rng_for(28, 0)).astype(np.complex128)
    a = orc.ionosphere(x, FS, FC, 42 * wf.TECU, naive=True)
    b = orc.ionosphere(x, FS, FC, 42 * wf.TECU, naive=False)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def test_pulse_is_doppler_then_ionosphere(orc):
    """Batch reading: Doppler first, then the ionosphere on the resampled samples.  The two
    orders differ by far more than the parity tolerance, so the order is part of the contract."""
    x = wf.bandlimited_noise(2048, wf.rng_for(29, 0))
    a, tec = orc.alpha_from_vr(7500.0), 80 * wf.TECU
    got = orc.correct_pulse(x, FS, a, tec, FC, half_width=64)
    ref = orc.ionosphere(orc.doppler(x, a, 64), FS, FC, tec, naive=False)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13
    swapped = orc.doppler(orc.ionosphere(x, FS, FC, tec, naive=False), a, 64)
    assert np.linalg.norm(swapped - ref) / np.linalg.norm(ref) > 1e-3


# --- pulse compression with the ionospheric operator in the same pass (Sec. II-B, II-D) --------

def _xcorr(x, r):
    """Circular cross-correlation by brute force: y[m] = sum_j x[(j + m) mod n] conj(r[j])."""
    n = x.size
    return np.array([sum(x[(j + m) % n] * np.conj(r[j]) for j in range(r.size)) for m in range(n)])


@pytest.mark.parametrize("n,n_rep", [(1, 1), (7, 3), (16, 16), (31, 5), (64, 20)])
def test_compress_is_circular_cross_correlation(orc, n, n_rep):
    rng = wf.rng_for(151, n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = rng.standard_normal(n_rep) + 1j * rng.standard_normal(n_rep)
    y = orc.compress(x, r, FS, FC, 0.0)
    ref = _xcorr(x, r)
    assert np.abs(y - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("d", [0, 1, 17, 63])
def test_compress_with_a_unit_replica_shifts(orc, d):
    rng = wf.rng_for(152, d)
    n = 64
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = np.zeros(d + 1, complex)
    r[d] = 1.0
    np.testing.assert_allclose(orc.compress(x, r, FS, FC, 0.0), np.roll(x, -d), rtol=0, atol=1e-13)


@pytest.mark.parametrize("direction", ["correct", "distort"])
def test_compress_applies_the_ionosphere_in_the_same_pass(orc, direction):
    """The phase commutes with the matched filter: compressing x at TEC E equals correlating the
    ionosphere-corrected x (the separately pinned operator) with the replica."""
    rng = wf.rng_for(153, 0)
    n = 256
    x = wf.bandlimited_noise(n, rng)
    r = wf.lfm(40, FS, 5e6)
    tec = 60 * wf.TECU
    y = orc.compress(x, r, FS, FC, tec, direction)
    ref = _xcorr(orc.ionosphere(x, FS, FC, tec, direction), r)
    assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max()


def test_compress_autocorrelation_peak_is_the_energy(orc):
    rng = wf.rng_for(154, 0)
    x = wf.lfm(512, FS, 5e6) * np.exp(2j * np.pi * rng.uniform())
    y = orc.compress(x, x, FS, FC, 0.0)
    assert y[0].real == pytest.approx(np.vdot(x, x).real, rel=1e-12)
    assert abs(y[0].imag) <= 1e-9 * abs(y[0])
    assert np.abs(y[1:]).max() <= np.abs(y[0]) * (1 + 1e-12)  # Cauchy-Schwarz


@pytest.mark.parametrize("n", [4096, 3001])  # the radix-2 and the Bluestein transforms
def test_compress_naive_and_fast_agree(orc, n):
    rng = wf.rng_for(155, 0)
    x = wf.bandlimited_noise(n, rng)
    r = wf.lfm(1000, FS, 5e6)
    a = orc.compress(x, r, FS, FC, 80 * wf.TECU, naive=True)
    b = orc.compress(x, r, FS, FC, 80 * wf.TECU, naive=False)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()


def test_compress_rejects_a_replica_longer_than_the_pulse(orc):
    with pytest.raises(Exception):
        orc.compress(np.ones(8, complex), np.ones(9, complex), FS, FC, 0.0)
