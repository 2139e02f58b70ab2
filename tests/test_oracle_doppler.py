"""Pins of the float64 oracle's Doppler resampling against facts the paper and the
mathematics fix (no GPU; nothing here touches the HIP library).

Doppler model: Eq (1)-(2) (alpha, S(alpha t)); resampling: Eq (17), Sec. III-B,
App. C (windowed Whittaker-Shannon sum); accuracy claims: Table I, Fig. 6.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

import waveforms as wf

C = 299792458


# --- Eq (1): alpha -------------------------------------------------------------------------

@pytest.mark.parametrize("v", [-8000.0, -1.0, 0.0, 1.0, 1000.0, 7500.0, 8000.0, 1.0e8, -2.5e8])
def test_alpha_matches_exact_rational(orc, v):
    """alpha = (1 + v/c)/(1 - v/c) = (c + v)/(c - v) exactly; the oracle must be within 2 ulp."""
    exact = Fraction(C) + Fraction(v)
    exact /= Fraction(C) - Fraction(v)
    a = orc.alpha_from_vr(v)
    assert abs(Fraction(a) - exact) <= 2 * Fraction(math.ulp(float(exact)))


@pytest.mark.parametrize("v", [3.0, 1000.0, 7500.0, 8000.0, 1.0e7])
def test_alpha_reciprocal(orc, v):
    """alpha(-v) = 1/alpha(v): receding and approaching dilations undo each other."""
    assert orc.alpha_from_vr(v) * orc.alpha_from_vr(-v) == pytest.approx(1.0, abs=4e-16)
    assert orc.alpha_from_vr(v) > 1.0 > orc.alpha_from_vr(-v)


@pytest.mark.parametrize("v", [C, -C, 2.0 * C, float("inf"), float("nan")])
def test_alpha_rejects_superluminal(orc, v):
    assert math.isnan(orc.alpha_from_vr(v))


# --- kernel pieces against library routines ------------------------------------------------

@pytest.mark.parametrize("z", [0.0, 1e-3, 0.5, 3.0, 8.0, 12.0, 25.0])
def test_bessel_i0_vs_scipy(orc, z):
    assert orc.bessel_i0(z) == pytest.approx(float(scipy.special.i0(z)), rel=1e-14)


@pytest.mark.parametrize("m", [9, 65, 129])
@pytest.mark.parametrize("beta", [0.0, 5.0, 8.0, 12.0])
def test_kaiser_vs_numpy_window(orc, m, beta):
    """numpy.kaiser(M, beta)[n] samples the same taper at x = 2n/(M-1) - 1."""
    ref = np.kaiser(m, beta)
    got = np.array([orc.kaiser(2.0 * n / (m - 1) - 1.0, beta) for n in range(m)])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
    assert orc.kaiser(1.0 + 1e-12, beta) == 0.0 and orc.kaiser(-1.5, beta) == 0.0


def test_sinc_vs_numpy(orc):
    u = np.concatenate([np.linspace(-70.3, 70.3, 1001), [0.0, 1.0, -3.0, 1e-9]])
    got = np.array([orc.sinc(v) for v in u])
    np.testing.assert_allclose(got, np.sinc(u), rtol=1e-12, atol=1e-16)


# --- D1 / D2: exact special cases ----------------------------------------------------------

@pytest.mark.parametrize("hw,window", [(64, "kaiser"), (3, "rect"), (5, "paper"), (0, "kaiser")])
def test_alpha_one_is_identity_bit_exact(orc, hw, window):
    """alpha = 1 samples every input at its own instant: y = x exactly (sinc(0)=1, sinc(k)=0)."""
    x = wf.bandlimited_noise(777, wf.rng_for(11, 0))
    y = orc.doppler(x, 1.0, hw, window)
    assert np.array_equal(y, x.astype(np.complex128))


@pytest.mark.parametrize("alpha", [2.0, 3.0])
def test_integer_alpha_is_exact_decimation(orc, alpha):
    """Integer alpha lands on input samples: y[m] = x[alpha m], zero past the end."""
    x = wf.bandlimited_noise(500, wf.rng_for(12, 0))
    y = orc.doppler(x, alpha, 16)
    a = int(alpha)
    exp = np.zeros(500, dtype=np.complex128)
    exp[: (499 // a) + 1] = x[::a]
    assert np.array_equal(y, exp)


# --- D3: multitone closed form -------------------------------------------------------------

def _multitone_case(n=4096, seed=13):
    rng = wf.rng_for(seed, 0)
    freqs = rng.uniform(-0.4, 0.4, 8)
    amps = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    return wf.multitone(n, freqs, amps), freqs, amps


@pytest.mark.parametrize("alpha", [1.0000500358660425, 0.99995, 1.37, 0.8])
def test_multitone_matches_closed_form(orc, alpha):
    """A sum of tones inside +/-0.4 fs resampled to S(alpha t) is the same tones at
    frequencies alpha f_j (Eq 2).  The Kaiser-windowed sum (H=64) approximates it to a few
    1e-6 at beta=8 and ~1e-7 at beta=12; dropping the taper costs three orders."""
    x, freqs, amps = _multitone_case()
    n = x.size
    t = alpha * np.arange(n)
    exact = (amps[None, :] * np.exp(2j * np.pi * freqs[None, :] * t[:, None])).sum(1)
    # the input the oracle sees is the complex64 rounding of the tones; compare against the
    # closed form only in the interior, where the window sees no edge
    sel = (t >= 64) & (t <= n - 65)

    def rel(y):
        return np.linalg.norm(y[sel] - exact[sel]) / np.linalg.norm(exact[sel])

    assert rel(orc.doppler(x, alpha, 64, "kaiser", 12.0)) < 3e-7
    assert rel(orc.doppler(x, alpha, 64, "kaiser", 8.0)) < 1.5e-5
    assert rel(orc.doppler(x, alpha, 64, "rect")) > 1e-3


# --- D4: analytic LFM (the paper's "DIR" control case) -------------------------------------

def test_lfm_matches_analytic_resampling(orc):
    """The single-LFM workload pulse resampled numerically equals the LFM regenerated at alpha t: start frequency
    scaled by alpha, chirp rate by alpha^2 (Eq 2; analytic resampling, Sec. I / Table I)."""
    c = wf.SINGLE_LFM
    n, fs, B = c["n"], c["fs"], c["bandwidth"]
    alpha = orc.alpha_from_vr(c["v_r"])
    x = wf.lfm(n, fs, B)
    exact = np.exp(1j * wf.lfm_phase(alpha * np.arange(n) / fs, fs, n, B))

    def rel(y, lo):
        s = slice(lo, n - lo)
        return np.linalg.norm(y[s] - exact[s]) / np.linalg.norm(exact[s])

    assert rel(orc.doppler(x, alpha, 64, "kaiser", 8.0), 64) < 1e-5
    full = orc.doppler(x, alpha, 0)
    assert rel(full, 256) < 3e-4  # full sum: error is the rectangular truncation at the pulse ends


def _snr_loss_db(a, b, max_lag=3):
    """-20 log10 of the peak normalised cross-correlation |sum a conj(b_lag)| / (|a||b|)."""
    best = 0.0
    for lag in range(-max_lag, max_lag + 1):
        if lag >= 0:
            c = np.vdot(b[lag:], a[: a.size - lag])
        else:
            c = np.vdot(b[:lag], a[-lag:])
        best = max(best, abs(c))
    return -20 * np.log10(best / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_window_convergence_is_inverse_square_in_snr_loss(orc):
    """Table I: windowed Whittaker-Shannon accuracy O(N_window^-2) for LFMs (found numerically
    by the authors).  Read as the SNR loss, which goes as the square of the sample error."""
    c = wf.SINGLE_LFM
    n, fs, B = c["n"], c["fs"], c["bandwidth"]
    alpha = orc.alpha_from_vr(c["v_r"])
    x = wf.lfm(n, fs, B)
    exact = np.exp(1j * wf.lfm_phase(alpha * np.arange(n) / fs, fs, n, B))
    s = slice(256, n - 256)
    hws = [8, 16, 32, 64]
    loss = [_snr_loss_db(orc.doppler(x, alpha, h, "rect")[s], exact[s]) for h in hws]
    slope = np.polyfit(np.log(2 * np.array(hws)), np.log(loss), 1)[0]
    assert -2.3 < slope < -1.7, (loss, slope)


def _read_golden(name):
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_paper_fig6_snr_loss_order_of_magnitude(orc):
    """Fig. 6: N_window = 41 sinc interpolation of the paper's LFM loses about 1e-4 dB of SNR
    against analytic resampling.  The caption's figure is approximate and the taper is
    unstated, so only the order of magnitude is pinned (paper mode: 41 taps centred on the
    nearest input, no taper)."""
    g = _read_golden("fig6_sinc_snr_loss.txt")
    fs, T, fc, B = g["fs_hz"], g["pulse_width_s"], g["center_hz"], g["bandwidth_hz"]
    n = int(round(T * fs))
    f0 = fc - B / 2
    alpha = orc.alpha_from_vr(g["v_r_mps"])

    def ph(t):
        return 2 * np.pi * (f0 * t + B / (2 * T) * t * t)

    t = np.arange(n) / fs
    x = np.exp(1j * ph(t))
    exact = np.exp(1j * ph(alpha * t))
    hw = int(g["n_window"]) // 2
    loss = _snr_loss_db(orc.doppler(x, alpha, hw, "paper"), exact)
    assert g["snr_loss_db"] / 10 < loss < g["snr_loss_db"] * 10, loss


# --- D5: brute force on tiny inputs, D8: approximate inverse, edges --------------------------

def _brute(x, alpha, hw, window, beta):
    """Direct transcription on tiny inputs with math.sin and scipy's I0 (cross-check of the C
    loops' bounds and index arithmetic)."""
    n_in = len(x)
    out = []
    for m in range(n_in):
        t = alpha * m
        if t == math.floor(t):
            k = int(t)
            out.append(complex(x[k]) if k < n_in else 0j)
            continue
        if hw == 0:
            taps = range(0, n_in)
        elif window == "paper":
            c = math.floor(t + 0.5)
            taps = range(c - hw, c + hw + 1)
        else:
            f = math.floor(t)
            taps = range(f - hw + 1, f + hw + 1)
        acc = 0j
        for k in taps:
            if 0 <= k < n_in:
                u = t - k
                w = math.sin(math.pi * u) / (math.pi * u)
                if hw and window == "kaiser":
                    r = u / hw
                    w *= scipy.special.i0(beta * math.sqrt(max(0.0, 1 - r * r))) / scipy.special.i0(beta)
                acc += complex(x[k]) * w
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
@pytest.mark.parametrize("alpha", [0.5, 0.999999, 1.000001, 1.00005, 1.3, 2.5])
def test_brute_force_tiny(orc, n, alpha):
    rng = wf.rng_for(14, n)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    for hw in sorted({0, 1, 2, max(1, n // 2), n}):
        for window in ("kaiser", "rect", "paper"):
            got = orc.doppler(x, alpha, hw, window, 8.0)
            ref = _brute(x, alpha, hw, window, 8.0)
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_resample_then_inverse_recovers_interior(orc):
    """alpha(-v) = 1/alpha(v): resampling by alpha and then by 1/alpha returns a band-limited
    input in the interior, to the windowed-sum accuracy (beta = 12)."""
    x = wf.bandlimited_noise(4096, wf.rng_for(15, 0), 0.6)
    a = orc.alpha_from_vr(8000.0)
    back = orc.doppler(orc.doppler(x, a, 64, "kaiser", 12.0), 1.0 / a, 64, "kaiser", 12.0)
    s = slice(200, 3800)
    assert np.linalg.norm(back[s] - x[s]) / np.linalg.norm(x[s]) < 1e-6


def test_outputs_past_the_input_are_zero(orc):
    """x[n] = 0 outside [0, N): an output whose whole window lies past the end is 0."""
    x = wf.bandlimited_noise(256, wf.rng_for(16, 0))
    y = orc.doppler(x, 1.5, 8, "kaiser", 8.0, n_out=256)
    t = 1.5 * np.arange(256)
    assert np.all(y[t > 255 + 8] == 0)
    assert np.all(np.abs(y[t < 200]) > 0)


def test_doppler_at_matches_full(orc):
    x = wf.bandlimited_noise(2048, wf.rng_for(17, 0))
    a = orc.alpha_from_vr(-6000.0)
    idx = np.array([0, 1, 5, 700, 2047, 1500])
    np.testing.assert_array_equal(orc.doppler_at(x, idx, a, 64), orc.doppler(x, a, 64)[idx])


# --- Impulse responses: the tap sets of Eq (17) / App. C written from the definitions ---------

def _impulse_expected(n, n0, alpha, hw, window, beta):
    """Output of a unit impulse at n0, from the definitions alone: numpy's sinc and I0.

    full sum (hw = 0): sinc(t - n0);
    Kaiser: sinc(t - n0) K((t - n0)/H) when |t - n0| < H (the 2H inputs floor(t)-H+1 ..
      floor(t)+H are exactly those within H of t), else 0;
    rect: sinc(t - n0) on the same 2H inputs;
    paper mode (App. C, Fig. 10: N_w = 2H+1 inputs centred on the nearest sample c = floor(t + 1/2)):
      sinc(t - n0) when |c - n0| <= H, else 0.
    An exact sample instant t = n0 gives 1, any other integer t gives 0."""
    y = np.zeros(n)
    for m in range(n):
        t = alpha * m
        if t == math.floor(t):
            y[m] = 1.0 if t == n0 else 0.0
            continue
        u = t - n0
        if hw == 0:
            y[m] = np.sinc(u)
        elif window == "paper":
            y[m] = np.sinc(u) if abs(math.floor(t + 0.5) - n0) <= hw else 0.0
        elif abs(u) < hw:
            w = np.sinc(u)
            if window == "kaiser":
                w *= np.i0(beta * math.sqrt(1.0 - (u / hw) ** 2)) / np.i0(beta)
            y[m] = w
    return y


IMPULSE_KERNELS = [(0, "kaiser"), (1, "kaiser"), (3, "kaiser"), (8, "kaiser"), (1, "rect"), (2, "rect"),
                   (5, "rect"), (1, "paper"), (2, "paper"), (3, "paper"), (12, "paper")]
IMPULSE_ALPHAS = [1.3, 0.77, 1.00005, 2.5, 0.999]


def _impulse_deviation(doppler):
    """Largest |oracle - definition| over every kernel, alpha and impulse position."""
    n, worst = 64, 0.0
    for hw, window in IMPULSE_KERNELS:
        for alpha in IMPULSE_ALPHAS:
            for n0 in (0, 1, 20, 41, 62, 63):
                x = np.zeros(n, np.complex128)
                x[n0] = 1.0
                got = doppler(x, alpha, hw, window, 6.0)
                exp = _impulse_expected(n, n0, alpha, hw, window, 6.0)
                worst = max(worst, float(np.max(np.abs(got - exp))))
    return worst


def test_impulse_response_is_the_kernel(orc):
    """Every output of a unit impulse is the kernel of Eq (17) at t - n0, with the tap set of
    its window (2H inputs around t; 2H + 1 around the nearest input in paper mode)."""
    assert _impulse_deviation(lambda x, a, h, w, b: orc.doppler(x, a, h, w, b)) <= 1e-13


def _mutant_doppler(tmp_path, old, new):
    """The oracle's C with one planted mistake, built on the CPU into a private library."""
    import ctypes
    import os
    import subprocess

    import oracle

    src = open(os.path.join(os.path.dirname(oracle.__file__), "rc_oracle.c")).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so),
                    str(path), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    p, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.rco_doppler.restype = i32
    lib.rco_doppler.argtypes = [p, i64, p, i64, d, i32, i32, d]

    def doppler(x, alpha, hw, window, beta):
        xin = np.ascontiguousarray(x, np.complex128)
        y = np.zeros(xin.size, np.complex128)
        assert lib.rco_doppler(xin.ctypes.data, xin.size, y.ctypes.data, y.size, alpha, hw,
                               oracle.WINDOWS[window], beta) == 0
        return y

    return doppler


@pytest.mark.parametrize("old,new", [
    ("(int64_t)floor(t + 0.5); /* nearest input sample */",
     "(int64_t)floor(t); /* nearest input sample */"),          # paper-mode centre at floor(t)
    ("lo = c - half_width;", "lo = c - half_width + 1;"),       # paper mode one tap short
    ("lo = (int64_t)f - half_width + 1;", "lo = (int64_t)f - half_width;"),  # 2H+1 taps
    ("hi = (int64_t)f + half_width;", "hi = (int64_t)f + half_width - 1;"),  # 2H-1 taps
])
def test_impulse_pin_catches_planted_tap_set_mistakes(tmp_path, old, new):
    """The impulse pin fails for an oracle with a planted one-tap mistake in its tap sets."""
    assert _impulse_deviation(_mutant_doppler(tmp_path, old, new)) > 1e-3
