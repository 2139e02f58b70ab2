"""Seeded synthetic waveforms and per-pulse parameter draws.

This module only *generates inputs*: it holds none of the correction arithmetic
(no resampling, no ionospheric phase, no Doppler factor).  Both the oracle-side
tests and the GPU-side tests / benchmark draw their inputs from here, so the two
sides see bit-identical complex64 samples.

Workload shapes follow the paper's synthetic test signals (LFM pulses, Sec. II-C
and III; no public dataset is used by the paper):

  SINGLE_LFM  single LFM pulse, N = 4096, fs = 10 MHz, B = 5 MHz, v_r = +7.5 km/s,
              full sinc + iono (E = 50 TECU, carrier 450 MHz)
  BATCH       1024 pulses x 65536 band-limited complex Gaussian noise (passband 0.8 fs),
              v_r ~ U[-8, 8] km/s, E ~ U[5, 100] TECU, Kaiser H = 64, beta = 8
  BANK        Doppler bank: one 2^20 polyphase-coded pulse, 256 v_r hypotheses in [-8, 8] km/s
  SERVING     serving stream: Poisson arrivals at 2000 pulses/s, lengths log-uniform 2^12..2^22
  LONG_DWELL  64 pulses x 2^24 band-limited noise, H = 128
"""
from __future__ import annotations

import numpy as np

TECU = 1e16  # electrons / m^2
FS_DEFAULT = 10e6
CARRIER_DEFAULT = 450e6


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (config seed, pulse index)."""
    return np.random.default_rng(np.random.PCG64(int(seed) * 1_000_003 + int(stream)))


def lfm(n: int, fs: float, bandwidth: float) -> np.ndarray:
    """Complex baseband up-chirp spanning [-B/2, +B/2] over the pulse, T = n/fs:
    x[k] = exp(2 pi i (-B/2 t + B/(2T) t^2)), t = k/fs (float64 phase, cast once)."""
    t = np.arange(n, dtype=np.float64) / fs
    T = n / fs
    return np.exp(2j * np.pi * (-0.5 * bandwidth * t + 0.5 * bandwidth / T * t * t)).astype(np.complex64)


def lfm_rf(n: int, fs: float, f0: float, bandwidth: float) -> np.ndarray:
    """Complex analytic up-chirp from f0 to f0 + B over the pulse, T = n/fs, sampled directly
    at RF (carrier 0): x[k] = exp(2 pi i (f0 t + B/(2T) t^2)), t = k/fs (float64, cast once)."""
    t = np.arange(n, dtype=np.float64) / fs
    T = n / fs
    return np.exp(2j * np.pi * (f0 * t + 0.5 * bandwidth / T * t * t)).astype(np.complex64)


def lfm_phase(t: np.ndarray, fs: float, n: int, bandwidth: float) -> np.ndarray:
    """Phase of the same chirp at arbitrary times t (seconds), float64."""
    T = n / fs
    return 2 * np.pi * (-0.5 * bandwidth * t + 0.5 * bandwidth / T * t * t)


def bandlimited_noise(n: int, rng: np.random.Generator, passband: float = 0.8) -> np.ndarray:
    """Complex Gaussian noise confined to |f| <= passband/2 * fs, unit mean power.

    Spectral construction: W_k ~ CN(0, 1) on the passband bins, zero elsewhere,
    x = IDFT(W) * sqrt(N / K_pass).  Returns complex64."""
    freqs = np.fft.fftfreq(n)
    mask = np.abs(freqs) <= 0.5 * passband
    k_pass = int(mask.sum())
    W = np.zeros(n, dtype=np.complex128)
    W[mask] = (rng.standard_normal(k_pass) + 1j * rng.standard_normal(k_pass)) * np.sqrt(0.5)
    x = np.fft.ifft(W) * np.sqrt(n / max(k_pass, 1)) * np.sqrt(n)
    return x.astype(np.complex64)


def multitone(n: int, freqs: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """Sum of complex tones a_j exp(2 pi i f_j k), f_j in cycles/sample (complex64)."""
    k = np.arange(n, dtype=np.float64)
    return (amps[None, :] * np.exp(2j * np.pi * freqs[None, :] * k[:, None])).sum(1).astype(np.complex64)


def polyphase_code(n: int, rng: np.random.Generator, phases: int = 64,
                   samples_per_chip: int = 4) -> np.ndarray:
    """Random-phase polyphase code: chip phases 2 pi p / P, p ~ U{0..P-1}, each chip
    held for ``samples_per_chip`` samples (complex64)."""
    chips = -(-n // samples_per_chip)
    p = rng.integers(0, phases, size=chips)
    x = np.exp(2j * np.pi * p / phases)
    return np.repeat(x, samples_per_chip)[:n].astype(np.complex64)


def draw_range_rates(count: int, rng: np.random.Generator, vmax: float = 8000.0) -> np.ndarray:
    """v_r ~ U[-vmax, vmax] m/s (positive when approaching)."""
    return rng.uniform(-vmax, vmax, size=count)


def draw_tec(count: int, rng: np.random.Generator, lo_tecu: float = 5.0,
             hi_tecu: float = 100.0) -> np.ndarray:
    """E ~ U[lo, hi] TECU, returned in electrons / m^2."""
    return rng.uniform(lo_tecu, hi_tecu, size=count) * TECU


def poisson_arrivals(rate_hz: float, count: int, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))


def loguniform_lengths(count: int, rng: np.random.Generator, lo_exp: float = 12.0,
                       hi_exp: float = 22.0) -> np.ndarray:
    """Pulse lengths floor(2^U), U ~ U[lo_exp, hi_exp]."""
    return np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)


# --- the workloads (seed 1 .. 5 in the order above) ----------------------------------------

SINGLE_LFM = dict(name="single_lfm_4096", seed=1, n=4096, fs=10e6, bandwidth=5e6, v_r=7500.0,
          tec=50 * TECU, carrier=450e6, half_width=0)
BATCH = dict(name="batch_1024x65536", seed=2, pulses=1024, n=65536, fs=FS_DEFAULT,
          carrier=CARRIER_DEFAULT, half_width=64, beta=8.0, passband=0.8)
BANK = dict(name="doppler_bank_256x2^20", seed=3, n=1 << 20, hypotheses=256, fs=FS_DEFAULT,
          half_width=64, beta=8.0)
SERVING = dict(name="serving_poisson_2000hz", seed=4, rate_hz=2000.0, lo_exp=12.0, hi_exp=22.0,
          fs=FS_DEFAULT, carrier=CARRIER_DEFAULT, half_width=64, beta=8.0)
LONG_DWELL = dict(name="long_dwell_64x2^24", seed=5, pulses=64, n=1 << 24, fs=FS_DEFAULT,
          carrier=CARRIER_DEFAULT, half_width=128, beta=8.0)
# the timing setup of the paper's ionospheric correction during pulse compression (Sec. II-D):
# 2^19 I/Q samples at 2.048 GHz, an LFM from 413 MHz over 18 MHz lasting 100 us, 100 TECU
COMPRESS = dict(name="pulse_compression_2^19", n=1 << 19, fs=2.048e9, f0=413e6, bandwidth=18e6,
                pulse_s=100e-6, tec=100 * TECU, carrier=0.0, delay=50000)
# The paper's sinc-resampler timing setup (Sec. III-B, Fig. 7; App. C, Fig. 9): 2^19 samples,
# a 25-sample window centred on the nearest input, no taper.  The waveform is not specified there:
# the Fig. 2 LFM band (413-431 MHz) over the whole record, sampled at 2.048 GHz, at v_r = 1 km/s.
PAPER_SINC = dict(name="paper_sinc_2^19", n=1 << 19, fs=2.048e9, f0=413e6, bandwidth=18e6,
                  half_width=12, window="paper", v_r=1000.0)
# The comparison of Doppler methods against velocity (Sec. III-A, Fig. 5): an LFM from 411 MHz
# over 18 MHz lasting 500 us.  Read here as complex samples taken at RF (carrier 0) at the
# original 2 GHz rate, so that resampling the record is the whole Doppler operator and frequency
# conversion shifts at the band centre; velocities 0 .. 5 km/s as in Fig. 4.
METHODS = dict(name="doppler_methods_fig5", fs=2e9, f0=411e6, bandwidth=18e6, pulse_s=500e-6,
               f_ref=420e6, v_max=5000.0, points=21, n_window=25, lut_size=1251)


def batch_pulse(p: int, n: int | None = None) -> np.ndarray:
    """Samples of pulse p of the batch workload (band-limited noise, passband 0.8 fs)."""
    return bandlimited_noise(BATCH["n"] if n is None else n, rng_for(BATCH["seed"], p + 1), BATCH["passband"])


def batch_params(pulses: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """(v_r [m/s], E [el/m^2]) for every pulse of the batch workload."""
    count = BATCH["pulses"] if pulses is None else pulses
    rng = rng_for(BATCH["seed"], 0)
    v = draw_range_rates(count, rng)
    e = draw_tec(count, rng)
    return v, e


def bank_range_rates(h: int = 256, vmax: float = 8000.0) -> np.ndarray:
    """Hypotheses v_h = -vmax + 2 vmax h / (H - 1), evenly spaced."""
    return -vmax + 2 * vmax * np.arange(h) / (h - 1)
