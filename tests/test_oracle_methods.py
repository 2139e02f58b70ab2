"""Pins of the oracle's references for the paper's other resampling methods (no GPU):
FFT P/Q resampling (Sec. I, Sec. III-A, Table I), frequency conversion and linear
interpolation (Sec. I, Table I), and the sinc lookup table of App. C (Alg. 2).

Each is pinned by a library routine, a closed form, or a convergence rate, never by a
re-transcription of its own formula.
"""
import numpy as np
import pytest
import scipy.signal as ss

import waveforms as wf

C = 299792458.0


def alpha(v):
    return (1 + v / C) / (1 - v / C)


# --- FFT P/Q resampling ------------------------------------------------------------------------

@pytest.mark.parametrize("n_in,n_out", [(64, 60), (64, 70), (63, 60), (63, 70), (64, 64), (65, 64), (100, 37),
                                        (37, 100), (64, 32), (32, 64), (1, 5), (5, 1), (4096, 4094), (4095, 4097)])
def test_resample_fft_is_scipy_resample(orc, n_in, n_out):
    """The bin removal / zero padding, Nyquist bins included, is scipy.signal.resample's."""
    rng = wf.rng_for(401, n_in * 7 + n_out)
    x = rng.standard_normal(n_in) + 1j * rng.standard_normal(n_in)
    np.testing.assert_allclose(orc.resample_fft(x, n_out), ss.resample(x, n_out), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n_in,n_out", [(1000, 998), (1000, 1004), (999, 995), (4096, 4000)])
def test_resample_fft_is_exact_for_periodic_band_limited_signals(orc, n_in, n_out):
    """Sum of tones on bins |k| < min(n_in, n_out)/2: the output samples are the signal itself
    at t = m n_in / n_out (the method is exact for Nyquist-limited periodic signals)."""
    rng = wf.rng_for(402, n_in)
    K = min(n_in, n_out)
    ks = rng.integers(-(K // 2) + 1, K // 2, size=12)
    amps = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    n = np.arange(n_in)
    x = (amps[None, :] * np.exp(2j * np.pi * np.outer(n, ks) / n_in)).sum(axis=1)
    m = np.arange(n_out)
    t = m * n_in / n_out
    ref = (amps[None, :] * np.exp(2j * np.pi * np.outer(t, ks) / n_in)).sum(axis=1)
    np.testing.assert_allclose(orc.resample_fft(x, n_out), ref, rtol=0, atol=1e-10)


def test_pq_length_removes_an_even_number_of_samples(orc):
    n = 102400  # the Fig 5 record: T = 500 us at 200 MHz... here 512 us at 200 MHz
    for v in np.linspace(-8000, 8000, 41):
        ni = orc.pq_length(n, alpha(v))
        assert (n - ni) % 2 == 0
        assert abs(ni - n / alpha(v)) <= 1.0 + 1e-9
    assert orc.pq_length(n, 1.0) == n


def test_doppler_pq_exact_at_even_whole_removals_and_harmonic_between(orc):
    """Table I, Fig 5: P/Q is exact when the dilation removes an even whole number of samples and
    worst halfway between (odd numbers).  A periodic band-limited multitone, where the only
    error is the rounding of the dilation to an even removal."""
    n = 8192
    rng = wf.rng_for(403, 0)
    ks = rng.integers(-400, 400, size=16)
    amps = rng.standard_normal(16) + 1j * rng.standard_normal(16)

    def sig(t):
        return (amps[None, :] * np.exp(2j * np.pi * np.outer(t, ks) / n)).sum(axis=1)

    x = sig(np.arange(n))
    errs = {}
    for removed in (2, 3, 4, 5, 6):
        a = n / (n - removed)  # alpha whose dilated record is exactly n - removed samples
        y = orc.doppler_pq(x, 10e6, a, n_out=n - 6)
        ref = sig(a * np.arange(n - 6))
        errs[removed] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert errs[2] < 1e-11 and errs[4] < 1e-11 and errs[6] < 1e-11, errs
    assert errs[3] > 1e-3 and errs[5] > 1e-3, errs


def test_doppler_pq_with_tone_beats_pq_alone_at_odd_removals(orc):
    """P/Q to the nearest even removal, then frequency conversion of the rest (Sec. III-A):
    for a narrowband signal around f_ref the remaining error drops."""
    n, fs, f0 = 8192, 10e6, 1.5e6
    t = np.arange(n) / fs
    x = np.exp(2j * np.pi * f0 * t) * np.exp(-((t - t.mean()) / (0.2 * n / fs)) ** 2)
    a = n / (n - 3)
    ref_t = a * np.arange(n - 8) / fs
    ref = np.exp(2j * np.pi * f0 * ref_t) * np.exp(-((ref_t - t.mean()) / (0.2 * n / fs)) ** 2)
    e_pq = np.linalg.norm(orc.doppler_pq(x, fs, a, n_out=n - 8) - ref) / np.linalg.norm(ref)
    e_tone = np.linalg.norm(orc.doppler_pq(x, fs, a, f_ref=f0, tone=True, n_out=n - 8) - ref) / np.linalg.norm(ref)
    assert e_tone < 0.1 * e_pq, (e_pq, e_tone)


# --- frequency conversion --------------------------------------------------------------------

@pytest.mark.parametrize("v", [-8000.0, 1000.0, 7500.0])
def test_tone_is_exact_for_a_tone_at_the_reference_frequency(orc, v):
    """The frequency shift is exact at one frequency (Sec. I): a complex tone at f_ref becomes
    the dilated tone exp(2 pi i f_ref alpha m / fs)."""
    n, fs, fr = 100000, 10e6, 3.3e6
    m = np.arange(n)
    x = np.exp(2j * np.pi * fr * m / fs)
    a = alpha(v)
    ref = np.exp(2j * np.pi * fr * a * m / fs)
    np.testing.assert_allclose(orc.doppler_tone(x, fs, a, fr), ref, rtol=0, atol=1e-9)


def test_tone_loss_grows_as_bandwidth_squared_for_lfms(orc):
    """Table I: for LFMs the frequency-conversion error is O(B^2), read (as for the sinc window's
    O(N_window^-2)) as the SNR loss against the analytic dilated LFM, which goes as the square of
    the phase error; the phase error itself grows as B.  LFM centred on f_ref = 0; doubling B
    quadruples the loss and doubles the relative L2 error."""
    fs, T = 200e6, 500e-6
    n = int(T * fs)
    t = np.arange(n) / fs
    a = alpha(5000.0)
    keep = slice(0, n - 100)  # clear of the dilated record's end

    def lfm(tt, B):
        return np.exp(2j * np.pi * (-B / 2 * tt + B / (2 * T) * tt ** 2))

    losses, errs = [], []
    for B in (0.5e6, 1e6, 2e6):
        y = orc.doppler_tone(lfm(t, B), fs, a, 0.0)[keep]
        ref = lfm(a * t, B)[keep]
        rho = abs(np.vdot(ref, y)) / (np.linalg.norm(ref) * np.linalg.norm(y))
        losses.append(-20 * np.log10(rho))
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    for i in range(2):
        assert 3.6 < losses[i + 1] / losses[i] < 4.4, losses
        assert 1.8 < errs[i + 1] / errs[i] < 2.2, errs


# --- linear interpolation --------------------------------------------------------------------

def test_linear_is_numpy_interp_inside_the_record(orc):
    rng = wf.rng_for(404, 0)
    n = 5000
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for v in (-7000.0, 333.0, 8000.0):
        a = alpha(v)
        m = np.arange(int((n - 1) / a))
        ref = np.interp(a * m, np.arange(n), x.real) + 1j * np.interp(a * m, np.arange(n), x.imag)
        np.testing.assert_allclose(orc.doppler_linear(x, a, n_out=m.size), ref, rtol=0, atol=1e-12)


def test_linear_is_exact_for_straight_lines_and_zero_past_the_end(orc):
    n = 1000
    x = (3.0 - 2.0j) + (0.25 + 0.5j) * np.arange(n)
    a = 1.75
    y = orc.doppler_linear(x, a, n_out=700)
    m = np.arange(700)
    inside = a * m <= n - 1
    np.testing.assert_allclose(y[inside], (3.0 - 2.0j) + (0.25 + 0.5j) * a * m[inside], rtol=0, atol=1e-10)
    assert np.all(y[a * m >= n] == 0)


# --- the sinc lookup table (App. C, Alg. 2) -------------------------------------------------

def test_lut_converges_to_the_paper_window_at_first_order(orc):
    """Nearest-entry lookup leaves a tap error of at most |sinc'| dx / 2: the table operator
    approaches the exact 25-tap paper window as the table grows, halving its error each time
    the table spacing halves."""
    n = 4000
    x = wf.bandlimited_noise(n, wf.rng_for(405, 0)).astype(np.complex128)
    a = 0.7654321  # positions spread over every fraction of a sample (a physical alpha barely moves them)
    exact = orc.doppler(x, a, 12, "paper")
    errs = []
    for s in (101, 201, 401, 801, 1601):
        y = orc.doppler_lut(x, a, 12, s)
        errs.append(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(1.6 < r < 2.5 for r in ratios), (errs, ratios)
    assert errs[-1] < 5e-3


def test_lut_at_exact_instants_with_a_hundredth_sample_spacing(orc):
    """With dx = 1/100 (lut_size = 1251 for 25 taps: the spacing of Fig 5) every tap of an
    exact sample instant falls on a table node sinc(k) = 0, k != 0, or sinc(0) = 1."""
    n = 300
    x = wf.bandlimited_noise(n, wf.rng_for(406, 0)).astype(np.complex128)
    y = orc.doppler_lut(x, 2.0, 12, 1251, n_out=150)
    np.testing.assert_allclose(y, x[::2], rtol=0, atol=1e-14)
