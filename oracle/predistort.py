"""LFM predistortion for the two-way ionospheric delay: an analytic cross-check of the FFT
phase operator of Eq (15)/(16).

TEST INFRASTRUCTURE ONLY, under the same rules as the rest of this package: only ``tests/``
may use it, and it shares nothing with the product library.  Plain numpy in float64.

The paper compares its FFT correction with two ways of predistorting a linear FM pulse so that
the ionosphere turns it back into the intended LFM (Sec. II-A, II-C; App. B):

* CUBIC: the instantaneous frequency f(t) that arrives at the right time is the real root of
  the cubic Eq (4), written in closed form by Eq (9)-(12); the phase is the trapezoidal
  integral of 2 pi f(t) over the sample grid.
* POLY: the pseudo-Chebyshev quadratic of Eq (5)-(8) with the node times of Eq (10)/(11), in
  the corrected form (2 K2 / c) or the original one (4 K2 / c, App. B Eq (13)/(14)).

The comparison measure is the SNR loss of a normalised cross-correlation peak.

Readings where the text is silent or inconsistent:

* Frames.  The received LFM has f_r(t_r) = f0 + B t_r / T on t_r in [0, T).  A component of
  frequency f reaches the receiver 2 tau(f) = 2 K2 / (c f^2) after it is sent.  Eq (4) carries
  the term -2 K2 B / (c f0^2 T), which puts t = 0 where f0 is sent ("paper frame").  Eq (16)
  applied to the LFM advances each component by 2 tau(f) ("FFT frame"), so t_paper = t_fft +
  2 tau(f0).  The predistorted pulse lasts from f0 to f0 + B, i.e. t_paper in
  [0, T - 2 tau(f0 + B) + 2 tau(f0)).
* Pseudo-Chebyshev nodes.  The quadratic passes through the three frequencies f0 + B/2 and
  f0 + B (1 -/+ a) / 2 (a = sqrt(3)/2), at their transmit times relative to the centre one:
  T1 (lower, Eq (10)), 0 and T3 (upper).  T3 is not printed; it is the mirror image of T1,
  T3 = a T / 2 + (2 K2 / c) [(f0 + B/2)^-2 - (f0 + B (1 + a) / 2)^-2], and T1 + T3 equals the
  printed T2 of Eq (11).
* Slope.  Through those nodes the slope is mu0 + dmu = (a B / 2) (T1^2 + T3^2) /
  (-T1 T3 (T3 - T1)).  The printed denominator of Eq (7) has T1 T2; that is read as a
  misprint, because T2 vanishes with K2 while the slope must tend to B / T.  The curvature of
  Eq (8) agrees with the three-node fit as printed.
* Constant term.  Eq (5) is taken around the centre node: f(t) = fc + (mu0 + dmu) u + gamma u^2,
  with fc = f0 + B/2 and u = t - tc, where tc is the transmit time of fc.
* SNR loss.  loss = -20 log10( max over lags |sum a[n] conj(b[n + lag])| / (|a| |b|) ) in dB.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
# CODATA 2022 values (e exact in the SI), the same physical constants the C oracle uses
_E_CHARGE = 1.602176634e-19
_M_E = 9.1093837139e-31
_EPS0 = 8.8541878188e-12

A_NODE = np.sqrt(3.0) / 2.0  # a of Eq (7)-(11): the outer Chebyshev nodes of degree 3


def k2_from_tec(tec: float) -> float:
    """K2 = e^2 E / (8 pi^2 m_e eps0) of Eq (3) / App. A (m^3 s^-2), E in electrons / m^2."""
    return _E_CHARGE ** 2 / (8.0 * np.pi ** 2 * _M_E * _EPS0) * tec


def two_way_delay(f, k2: float):
    """2 tau(f) = 2 K2 / (c f^2), Eq (3) taken both ways."""
    f = np.asarray(f, dtype=np.float64)
    return 2.0 * k2 / (C_LIGHT * f * f)


def cubic_coefficients(t, f0: float, B: float, T: float, k2: float):
    """(p, q) of Eq (4) written as f^3 - p f^2 - q = 0 (paper frame)."""
    t = np.asarray(t, dtype=np.float64)
    p = f0 + B * t / T - 2.0 * k2 * B / (C_LIGHT * f0 * f0 * T)
    q = 2.0 * k2 * B / (C_LIGHT * T)
    return p, q


def cubic_frequency(t, f0: float, B: float, T: float, k2: float):
    """The real root of Eq (4) at paper-frame times t, by the closed form of Eq (9)-(12)."""
    p, q = cubic_coefficients(t, f0, B, T, k2)
    chi = p * p                                      # Eq (10)
    psi = -2.0 * p ** 3 - 27.0 * q                   # Eq (11)
    # psi^2 - 4 chi^3 = 108 p^3 q + 729 q^2 >= 0 for q >= 0; without an ionosphere (q = 0) it is
    # zero and rounding may leave it a hair below
    disc = np.maximum(psi * psi - 4.0 * chi ** 3, 0.0)
    omega = np.cbrt((psi + np.sqrt(disc)) / 2.0)     # Eq (12), the real cube root
    return (p - omega - chi / omega) / 3.0           # Eq (9)


def chebyshev_node_times(f0: float, B: float, T: float, k2: float, original: bool = False):
    """(T1, T2, T3) of Eq (10)/(11) (original=True: the 4 K2 / c forms of Eq (13)/(14)).

    T1 and T3 are the transmit times of the lower and upper node relative to the centre node;
    T2 = T1 + T3.
    """
    a = A_NODE
    g = (4.0 if original else 2.0) * k2 / C_LIGHT
    fc = f0 + B / 2.0
    flo = f0 + B * (1.0 - a) / 2.0
    fhi = f0 + B * (1.0 + a) / 2.0
    T1 = -a * T / 2.0 + g * (fc ** -2 - flo ** -2)
    T2 = g * (2.0 * fc ** -2 - flo ** -2 - fhi ** -2)
    T3 = a * T / 2.0 + g * (fc ** -2 - fhi ** -2)
    return T1, T2, T3


def poly_coefficients(f0: float, B: float, T: float, k2: float, original: bool = False):
    """Pseudo-Chebyshev quadratic, Eq (5)-(8): returns (fc, tc, slope, gamma).

    f(t) = fc + slope (t - tc) + gamma (t - tc)^2 in the paper frame, with slope = mu0 + dmu.
    """
    a = A_NODE
    T1, T2, T3 = chebyshev_node_times(f0, B, T, k2, original)
    slope = (a * B / 2.0) * (T1 * T1 + T3 * T3) / (-T1 * T3 * (T3 - T1))
    gamma = (a * B / 2.0) * T2 / (T1 * T3 * (T3 - T1))
    fc = f0 + B / 2.0
    # the centre frequency is received at T/2 and sent 2 tau(fc) earlier; the paper frame puts
    # the start frequency's transmission at 0
    tc = T / 2.0 - float(two_way_delay(fc, k2)) + float(two_way_delay(f0, k2))
    return fc, tc, slope, gamma


def poly_frequency(t, f0: float, B: float, T: float, k2: float, original: bool = False):
    fc, tc, slope, gamma = poly_coefficients(f0, B, T, k2, original)
    u = np.asarray(t, dtype=np.float64) - tc
    return fc + slope * u + gamma * u * u


def sample_times(n: int, n0: int, fs: float) -> np.ndarray:
    """t_n = (n - n0) / fs: sample n0 is time 0 of the FFT frame (where the LFM starts)."""
    return (np.arange(n, dtype=np.float64) - n0) / fs


def lfm(n: int, n0: int, fs: float, f0: float, B: float, T: float) -> np.ndarray:
    """The intended received pulse: exp(2 pi i (f0 t + B t^2 / (2T))) on [0, T), else 0."""
    t = sample_times(n, n0, fs)
    inside = (t >= 0.0) & (t < T)
    return np.where(inside, np.exp(2j * np.pi * (f0 * t + B * t * t / (2.0 * T))), 0.0)


def _paper_support(n: int, n0: int, fs: float, f0: float, B: float, T: float, k2: float):
    t_fft = sample_times(n, n0, fs)
    t_paper = t_fft + float(two_way_delay(f0, k2))
    t_end = T - float(two_way_delay(f0 + B, k2)) + float(two_way_delay(f0, k2))
    return t_paper, (t_paper >= 0.0) & (t_paper < t_end)


def cubic_waveform(n: int, n0: int, fs: float, f0: float, B: float, T: float, k2: float) -> np.ndarray:
    """CUBIC predistortion in the FFT frame: exp(i phi), phi the trapezoidal integral of 2 pi f."""
    t_paper, inside = _paper_support(n, n0, fs, f0, B, T, k2)
    f = cubic_frequency(t_paper, f0, B, T, k2)
    phi = np.zeros(n)
    phi[1:] = np.cumsum(np.pi * (f[1:] + f[:-1]) / fs)  # 2 pi * (f_i + f_{i+1}) / 2 * dt
    return np.where(inside, np.exp(1j * phi), 0.0)


def poly_waveform(n: int, n0: int, fs: float, f0: float, B: float, T: float, k2: float,
                  original: bool = False) -> np.ndarray:
    """POLY predistortion in the FFT frame: the quadratic frequency integrated in closed form."""
    t_paper, inside = _paper_support(n, n0, fs, f0, B, T, k2)
    fc, tc, slope, gamma = poly_coefficients(f0, B, T, k2, original)
    u = t_paper - tc
    phi = 2.0 * np.pi * (fc * u + slope * u * u / 2.0 + gamma * u ** 3 / 3.0)
    return np.where(inside, np.exp(1j * phi), 0.0)


def snr_loss_db(a, b) -> float:
    """-20 log10 of the peak of the normalised cross-correlation of a and b over all lags."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    m = 1 << int(np.ceil(np.log2(a.size + b.size)))
    cc = np.fft.ifft(np.fft.fft(a, m) * np.conj(np.fft.fft(b, m)))
    peak = np.abs(cc).max() / (np.linalg.norm(a) * np.linalg.norm(b))
    return float(-20.0 * np.log10(peak))
