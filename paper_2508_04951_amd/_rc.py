"""ctypes binding of librc.so (include/rc.h).

Argument marshalling only: every step of the correction runs in the HIP kernels of the
library.  torch provides device memory and the stream (``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``, which are HIP objects on ROCm).  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librc.so")

RC_OK, RC_ERR_INVALID_ARG, RC_ERR_UNSUPPORTED, RC_ERR_OUT_OF_MEMORY, RC_ERR_DEVICE, RC_ERR_BUSY = range(6)
WINDOWS = {"kaiser": 0, "rect": 1, "paper": 2}
DIRECTIONS = {"correct": 0, "distort": 1}
DO_DOPPLER, DO_IONO = 1, 2

# exported symbols of include/rc.h
SYMBOLS = (
    "rc_create", "rc_destroy", "rc_status_string", "rc_last_error", "rc_alpha_from_vr",
    "rc_k2_per_tec", "rc_sync", "correct_doppler", "correct_ionosphere", "correct_ionosphere_noalloc",
    "correct_pulse_batch",
    "correct_doppler_bank", "rc_server_create", "rc_server_submit", "rc_server_poll", "rc_server_wait",
    "rc_server_stats", "rc_server_reset_stats", "rc_server_destroy", "rc_server_request_bytes",
    "rc_profile_enable", "rc_profile_read", "rc_set_sinc_engine", "rc_set_bank_engine", "rc_set_mem_budget",
    "replica_spectrum", "compress_pulse",
    "correct_doppler_paper", "correct_doppler_linear", "correct_doppler_tone", "rc_pq_length",
    "correct_doppler_fft_pq", "rc_batch_plan_create", "rc_batch_plan_launch", "rc_batch_plan_update",
    "rc_batch_plan_destroy", "rc_set_fft_levels", "rc_set_sinc_grid", "rc_set_bluestein_chunk", "rc_load_tuning",
)
KERNELS = ("k_sinc_mfma", "k_sinc_fast", "k_sinc_direct", "k_fft_strided_fwd", "k_fft_rows_iono",
           "k_fft_strided_inv", "k_mf_tile_list", "k_bluestein", "k_farrow_z", "k_farrow_bank",
           "k_paper_sinc", "k_linear", "k_tone", "k_pq")
PAPER_VARIANTS = {"direct": 0, "tiled": 1, "lut": 2}
# the autotuner's table for gfx950 (paper_2508_04951_amd/tune.py writes it)
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
BANK_PRECISIONS = {"fp16x3": 0, "bf16x3": 1, "fp32": 2}
BANK_ENGINES = {"auto": 0, "farrow": 1, "per_hypothesis": 2}
SINC_ENGINES = {"auto": 0, "valu": 1, "direct": 2}


class RcSinc(ctypes.Structure):
    _fields_ = [("half_width", ctypes.c_int32), ("window", ctypes.c_int32), ("kaiser_beta", ctypes.c_double)]


class RcPulse(ctypes.Structure):
    _fields_ = [
        ("off_in", ctypes.c_int64), ("n_in", ctypes.c_int64), ("off_out", ctypes.c_int64),
        ("n_out", ctypes.c_int64), ("fs_hz", ctypes.c_double), ("alpha", ctypes.c_double),
        ("tec_el_per_m2", ctypes.c_double), ("carrier_hz", ctypes.c_double),
        ("flags", ctypes.c_uint32), ("direction", ctypes.c_int32),
    ]


class RcRequest(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n_in", ctypes.c_int64), ("n_out", ctypes.c_int64),
        ("fs_hz", ctypes.c_double), ("alpha", ctypes.c_double), ("tec_el_per_m2", ctypes.c_double),
        ("carrier_hz", ctypes.c_double), ("flags", ctypes.c_uint32), ("direction", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class RcServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
        ("batches", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("latency_ms_p50", ctypes.c_double),
        ("latency_ms_p99", ctypes.c_double), ("latency_ms_max", ctypes.c_double),
        ("samples_per_s", ctypes.c_double),
    ]


class RcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librc.so (built by ``python -m paper_2508_04951_amd.build``)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2508_04951_amd.build`")
        # torch ships its own HIP runtime; loading it first makes librc.so bind to that same
        # runtime, so tensors and streams from torch are valid in the library's calls.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        c_i32, c_i64, c_d, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.rc_create.argtypes = [ctypes.c_int, ctypes.POINTER(p)]
        lib.rc_create.restype = c_i32
        lib.rc_destroy.argtypes = [p]
        lib.rc_destroy.restype = c_i32
        lib.rc_status_string.argtypes = [c_i32]
        lib.rc_status_string.restype = ctypes.c_char_p
        lib.rc_last_error.argtypes = [p]
        lib.rc_last_error.restype = ctypes.c_char_p
        lib.rc_alpha_from_vr.argtypes = [c_d]
        lib.rc_alpha_from_vr.restype = c_d
        lib.rc_k2_per_tec.argtypes = []
        lib.rc_k2_per_tec.restype = c_d
        lib.rc_sync.argtypes = [p, p]
        lib.rc_sync.restype = c_i32
        lib.correct_doppler.argtypes = [p, p, c_i64, p, c_i64, c_d, c_d, ctypes.POINTER(RcSinc), p]
        lib.correct_doppler.restype = c_i32
        lib.correct_doppler_bank.argtypes = [p, p, c_i64, p, c_i64, c_d, ctypes.POINTER(c_d), c_i32,
                                             ctypes.POINTER(RcSinc), c_i32, p]
        lib.correct_doppler_bank.restype = c_i32
        lib.correct_ionosphere.argtypes = [p, p, p, c_i64, c_d, c_d, c_d, c_i32, p]
        lib.correct_ionosphere.restype = c_i32
        lib.correct_ionosphere_noalloc.argtypes = [p, p, p, c_i64, c_d, c_d, c_d, c_i32, p]
        lib.correct_ionosphere_noalloc.restype = c_i32
        lib.correct_doppler_paper.argtypes = [p, p, c_i64, p, c_i64, c_d, c_d, c_i32, c_i32, c_i32, c_i32, p]
        lib.correct_doppler_paper.restype = c_i32
        lib.correct_doppler_linear.argtypes = [p, p, c_i64, p, c_i64, c_d, c_d, p]
        lib.correct_doppler_linear.restype = c_i32
        lib.correct_doppler_tone.argtypes = [p, p, p, c_i64, c_d, c_d, c_d, p]
        lib.correct_doppler_tone.restype = c_i32
        lib.rc_pq_length.argtypes = [c_i64, c_d]
        lib.rc_pq_length.restype = c_i64
        lib.correct_doppler_fft_pq.argtypes = [p, p, c_i64, p, c_i64, c_d, c_d, c_d, c_i32, p]
        lib.correct_doppler_fft_pq.restype = c_i32
        lib.replica_spectrum.argtypes = [p, p, c_i64, c_i64, p, p]
        lib.replica_spectrum.restype = c_i32
        lib.compress_pulse.argtypes = [p, p, p, c_i64, p, c_d, c_d, c_d, c_i32, p]
        lib.compress_pulse.restype = c_i32
        lib.correct_pulse_batch.argtypes = [p, p, c_i64, p, c_i64, ctypes.POINTER(RcPulse), c_i32,
                                            ctypes.POINTER(RcSinc), p]
        lib.correct_pulse_batch.restype = c_i32
        lib.rc_batch_plan_create.argtypes = [p, p, c_i64, p, c_i64, ctypes.POINTER(RcPulse), c_i32,
                                             ctypes.POINTER(RcSinc), ctypes.POINTER(p)]
        lib.rc_batch_plan_create.restype = c_i32
        lib.rc_batch_plan_launch.argtypes = [p, p]
        lib.rc_batch_plan_launch.restype = c_i32
        lib.rc_batch_plan_update.argtypes = [p, ctypes.POINTER(RcPulse), c_i32, p]
        lib.rc_batch_plan_update.restype = c_i32
        lib.rc_batch_plan_destroy.argtypes = [p]
        lib.rc_batch_plan_destroy.restype = c_i32
        lib.rc_profile_enable.argtypes = [p, ctypes.c_int]
        lib.rc_profile_enable.restype = c_i32
        lib.rc_profile_read.argtypes = [p, ctypes.c_char_p, ctypes.POINTER(c_d), ctypes.POINTER(c_i64)]
        lib.rc_profile_read.restype = c_i32
        lib.rc_set_sinc_engine.argtypes = [p, c_i32]
        lib.rc_set_sinc_engine.restype = c_i32
        lib.rc_set_bank_engine.argtypes = [p, c_i32]
        lib.rc_set_bank_engine.restype = c_i32
        lib.rc_set_fft_levels.argtypes = [p, c_i64, ctypes.POINTER(c_i32), c_i32]
        lib.rc_set_fft_levels.restype = c_i32
        lib.rc_set_sinc_grid.argtypes = [p, c_i32, c_i32]
        lib.rc_set_sinc_grid.restype = c_i32
        lib.rc_set_bluestein_chunk.argtypes = [p, c_i64]
        lib.rc_set_bluestein_chunk.restype = c_i32
        lib.rc_load_tuning.argtypes = [p, ctypes.c_char_p]
        lib.rc_load_tuning.restype = c_i32
        lib.rc_set_mem_budget.argtypes = [p, ctypes.c_int64]
        lib.rc_set_mem_budget.restype = c_i32
        lib.rc_server_create.argtypes = [p, ctypes.POINTER(RcSinc), c_i64, c_i32, ctypes.POINTER(p)]
        lib.rc_server_submit.argtypes = [p, ctypes.POINTER(RcRequest), ctypes.POINTER(c_i64)]
        lib.rc_server_request_bytes.argtypes = [p, ctypes.POINTER(RcRequest)]
        lib.rc_server_request_bytes.restype = c_i64
        lib.rc_server_poll.argtypes = [p, c_i64, ctypes.POINTER(c_i32)]
        lib.rc_server_wait.argtypes = [p, c_i64]
        lib.rc_server_stats.argtypes = [p, ctypes.POINTER(RcServerStats)]
        lib.rc_server_reset_stats.argtypes = [p]
        lib.rc_server_destroy.argtypes = [p]
        for f in ("rc_server_create", "rc_server_submit", "rc_server_poll", "rc_server_wait", "rc_server_stats",
                  "rc_server_reset_stats", "rc_server_destroy"):
            getattr(lib, f).restype = c_i32
        _lib = lib
        return lib


def alpha_from_vr(v_r: float) -> float:
    """Eq (1): alpha = (1 + v_r/c)/(1 - v_r/c), v_r positive when approaching (librc)."""
    return float(load_library().rc_alpha_from_vr(float(v_r)))


def _alpha_or_vr(alpha, v_r) -> float:
    if (alpha is None) == (v_r is None):
        raise ValueError("give exactly one of alpha and v_r")
    if alpha is None:
        alpha = alpha_from_vr(v_r)
        if alpha != alpha:  # NaN: |v_r| >= c
            raise ValueError("|v_r| must be below the speed of light")
    return float(alpha)


def pq_length(n_in: int, alpha: float) -> int:
    """Length of the FFT P/Q resampled record (an even number of samples removed or added)."""
    return int(load_library().rc_pq_length(int(n_in), float(alpha)))


def k2_per_tec() -> float:
    """Eq (3): K2/E = e^2/(8 pi^2 m_e eps0) in m^3 s^-2 (librc)."""
    return float(load_library().rc_k2_per_tec())


@dataclass
class Sinc:
    """Resampling kernel: half_width H (0 = full sum), window name, Kaiser beta."""
    half_width: int = 64
    window: str = "kaiser"
    beta: float = 8.0

    def c(self) -> RcSinc:
        if self.window not in WINDOWS:
            raise ValueError(f"unknown window {self.window!r}")
        return RcSinc(int(self.half_width), WINDOWS[self.window], float(self.beta))


def _torch():
    import torch

    return torch


def _check_samples(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.complex64:
        raise TypeError(f"{name} must be complex64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """An rc_context on one HIP device."""

    def __init__(self, device: int = 0, tuning: str | None = "default"):
        """tuning: "default" applies the autotuner's table shipped with the package (tuning.json
        beside this file) unless RC_TUNE_FILE names one, which rc_create then loads itself; a
        path applies that file; None applies nothing beyond RC_TUNE_FILE."""
        self._lib = load_library()
        self.device = int(device)
        h = ctypes.c_void_p()
        st = self._lib.rc_create(self.device, ctypes.byref(h))
        if st != RC_OK:
            raise RcError(st, f"rc_create({device}) failed: {self._lib.rc_status_string(st).decode()}")
        self._h = h
        if tuning == "default":
            tuning = None if os.environ.get("RC_TUNE_FILE") else (TUNING_PATH if os.path.exists(TUNING_PATH) else None)
        if tuning:
            self.load_tuning(tuning)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _raise(self, st: int, what: str):
        msg = self._lib.rc_last_error(self._h).decode()
        name = self._lib.rc_status_string(st).decode()
        if st == RC_ERR_INVALID_ARG:
            raise ValueError(f"{what}: {name}: {msg}")
        raise RcError(st, f"{what}: {name}: {msg}")

    def _stream(self, stream=None) -> int:
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return int(s.cuda_stream)

    def sync(self, stream=None):
        st = self._lib.rc_sync(self._h, self._stream(stream))
        if st != RC_OK:
            self._raise(st, "rc_sync")

    def set_mem_budget(self, nbytes: int = 0):
        """Cap the context's device workspace at nbytes (0: no cap); see rc_set_mem_budget."""
        st = self._lib.rc_set_mem_budget(self._h, int(nbytes))
        if st != RC_OK:
            self._raise(st, "rc_set_mem_budget")

    def set_fft_levels(self, n: int, levels=()):
        """Strided levels of the n-point transform before its 4096-point level (() = default)."""
        arr = (ctypes.c_int32 * max(1, len(levels)))(*[int(v) for v in levels])
        st = self._lib.rc_set_fft_levels(self._h, int(n), arr, len(levels))
        if st != RC_OK:
            self._raise(st, "rc_set_fft_levels")

    def set_sinc_grid(self, half_width: int, wg_per_cu: int = 0):
        """Workgroups per CU of the matrix-core resampler at half_width 64 or 128 (0 = all that fit)."""
        st = self._lib.rc_set_sinc_grid(self._h, int(half_width), int(wg_per_cu))
        if st != RC_OK:
            self._raise(st, "rc_set_sinc_grid")

    def set_bluestein_chunk(self, nbytes: int = 0):
        st = self._lib.rc_set_bluestein_chunk(self._h, int(nbytes))
        if st != RC_OK:
            self._raise(st, "rc_set_bluestein_chunk")

    def load_tuning(self, path: str):
        """Apply an autotuner table (JSON; see rc_load_tuning)."""
        st = self._lib.rc_load_tuning(self._h, os.fsencode(path))
        if st != RC_OK:
            self._raise(st, "rc_load_tuning")

    def set_sinc_engine(self, engine: str = "auto"):
        """Resampling engine for later calls: "auto" (matrix cores where eligible), "valu" or
        "direct" (the direct sum: float64 positions, float32 tap weights)."""
        if engine not in SINC_ENGINES:
            raise ValueError(f"engine must be one of {list(SINC_ENGINES)}")
        st = self._lib.rc_set_sinc_engine(self._h, SINC_ENGINES[engine])
        if st != RC_OK:
            self._raise(st, "rc_set_sinc_engine")

    def set_bank_engine(self, engine: str = "auto"):
        """Engine of later correct_doppler_bank calls: "auto" (the filter bank where it applies),
        "farrow" (always the filter bank; RcError where it does not apply) or "per_hypothesis"."""
        if engine not in BANK_ENGINES:
            raise ValueError(f"engine must be one of {list(BANK_ENGINES)}")
        st = self._lib.rc_set_bank_engine(self._h, BANK_ENGINES[engine])
        if st != RC_OK:
            self._raise(st, "rc_set_bank_engine")

    def profile(self, enable: bool = True):
        """Bracket every kernel launch with HIP events on its stream (for benchmarks)."""
        st = self._lib.rc_profile_enable(self._h, int(bool(enable)))
        if st != RC_OK:
            self._raise(st, "rc_profile_enable")

    def profile_read(self) -> dict:
        """{kernel: (total_ms, launches)} since the last read (waits for the recorded events)."""
        out = {}
        for name in KERNELS:
            ms, n = ctypes.c_double(), ctypes.c_int64()
            st = self._lib.rc_profile_read(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(n))
            if st != RC_OK:
                self._raise(st, "rc_profile_read")
            out[name] = (ms.value, n.value)
        return out

    def correct_doppler(self, x, alpha: float | None = None, sinc: Sinc | None = None, n_out: int | None = None,
                        fs: float = 1.0, out=None, stream=None, *, v_r: float | None = None):
        """y[m] = sum_n x[n] h(alpha m - n) (Eq 2 / Eq 17) for m < n_out.  Give alpha, or the range
        rate v_r in m/s (alpha from Eq (1) by rc_alpha_from_vr), not both."""
        torch = _torch()
        alpha = _alpha_or_vr(alpha, v_r)
        _check_samples(x, "x")
        n_out = x.numel() if n_out is None else int(n_out)
        if out is None:
            out = torch.empty(n_out, dtype=torch.complex64, device=x.device)
        _check_samples(out, "out")
        if out.numel() < n_out:
            raise ValueError("out is shorter than n_out")
        k = (sinc or Sinc()).c()
        st = self._lib.correct_doppler(self._h, x.data_ptr(), x.numel(), out.data_ptr(), n_out, float(fs),
                                       float(alpha), ctypes.byref(k), self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler")
        return out

    def correct_ionosphere(self, x, fs: float, carrier: float, tec: float, direction: str = "correct",
                           out=None, stream=None):
        """y = IDFT(DFT(x) exp(-/+ i 4 pi K2 / (c f_k))) (Eq 16 / Eq 15).  out may be x."""
        torch = _torch()
        _check_samples(x, "x")
        if out is None:
            out = torch.empty_like(x)
        _check_samples(out, "out")
        if out.numel() != x.numel():
            raise ValueError("out must have as many samples as x")
        if direction not in DIRECTIONS:
            raise ValueError(f"direction must be one of {list(DIRECTIONS)}")
        st = self._lib.correct_ionosphere(self._h, x.data_ptr(), out.data_ptr(), x.numel(), float(fs),
                                          float(carrier), float(tec), DIRECTIONS[direction],
                                          self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_ionosphere")
        return out

    def correct_ionosphere_noalloc(self, x, out, fs: float, carrier: float, tec: float,
                                   direction: str = "correct", stream=None):
        """correct_ionosphere into a caller-given `out` (may be x) through the entry point that
        allocates no device memory (lengths that are not powers of two: n <= 2^20)."""
        _check_samples(x, "x")
        _check_samples(out, "out")
        if out.numel() != x.numel():
            raise ValueError("out must have as many samples as x")
        if direction not in DIRECTIONS:
            raise ValueError(f"direction must be one of {list(DIRECTIONS)}")
        st = self._lib.correct_ionosphere_noalloc(self._h, x.data_ptr(), out.data_ptr(), x.numel(), float(fs),
                                                  float(carrier), float(tec), DIRECTIONS[direction],
                                                  self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_ionosphere_noalloc")
        return out

    def _out_for(self, x, n_out, out):
        torch = _torch()
        _check_samples(x, "x")
        n_out = x.numel() if n_out is None else int(n_out)
        if out is None:
            out = torch.empty(n_out, dtype=torch.complex64, device=x.device)
        _check_samples(out, "out")
        if out.numel() < n_out:
            raise ValueError("out is shorter than n_out")
        return n_out, out

    def correct_doppler_paper(self, x, alpha: float | None = None, n_window: int = 25, variant: str = "direct",
                              lut_size: int = 3000, blocks: int = 0, n_out: int | None = None, fs: float = 1.0,
                              out=None, stream=None, *, v_r: float | None = None):
        """The paper's sinc kernel (App. C): n_window inputs centred on the nearest, untapered, in
        the variant "direct" (Alg. 1), "tiled" (Alg. 3) or "lut" (Alg. 2, lut_size entries)."""
        alpha = _alpha_or_vr(alpha, v_r)
        if variant not in PAPER_VARIANTS:
            raise ValueError(f"variant must be one of {list(PAPER_VARIANTS)}")
        n_out, out = self._out_for(x, n_out, out)
        st = self._lib.correct_doppler_paper(self._h, x.data_ptr(), x.numel(), out.data_ptr(), n_out, float(fs),
                                             float(alpha), int(n_window), PAPER_VARIANTS[variant], int(lut_size),
                                             int(blocks), self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler_paper")
        return out

    def correct_doppler_linear(self, x, alpha: float | None = None, n_out: int | None = None, fs: float = 1.0,
                               out=None, stream=None, *, v_r: float | None = None):
        """Linear interpolation at t = alpha m (Sec. I, Table I)."""
        alpha = _alpha_or_vr(alpha, v_r)
        n_out, out = self._out_for(x, n_out, out)
        st = self._lib.correct_doppler_linear(self._h, x.data_ptr(), x.numel(), out.data_ptr(), n_out, float(fs),
                                              float(alpha), self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler_linear")
        return out

    def correct_doppler_tone(self, x, fs: float, alpha: float | None = None, f_ref: float = 0.0, out=None,
                             stream=None, *, v_r: float | None = None):
        """Frequency conversion: x[m] exp(2 pi i (alpha - 1) f_ref m / fs).  out may be x."""
        alpha = _alpha_or_vr(alpha, v_r)
        _, out = self._out_for(x, None, out)
        if out.numel() != x.numel():
            raise ValueError("out must have as many samples as x")
        st = self._lib.correct_doppler_tone(self._h, x.data_ptr(), out.data_ptr(), x.numel(), float(fs),
                                            float(alpha), float(f_ref), self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler_tone")
        return out

    def correct_doppler_fft_pq(self, x, fs: float, alpha: float | None = None, f_ref: float = 0.0,
                               tone: bool = False, n_out: int | None = None, out=None, stream=None, *,
                               v_r: float | None = None):
        """FFT P/Q resampling to pq_length(n, alpha) samples, then (tone=True) frequency conversion
        of the remaining dilation at the moved reference frequency (Sec. III-A)."""
        alpha = _alpha_or_vr(alpha, v_r)
        n_out, out = self._out_for(x, n_out, out)
        st = self._lib.correct_doppler_fft_pq(self._h, x.data_ptr(), x.numel(), out.data_ptr(), n_out, float(fs),
                                              float(alpha), float(f_ref), int(bool(tone)), self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler_fft_pq")
        return out

    def replica_spectrum(self, replica, n: int, out=None, stream=None):
        """DFT_n of the replica zero-padded to n (internal bin order), for compress_pulse."""
        torch = _torch()
        _check_samples(replica, "replica")
        n = int(n)
        if out is None:
            out = torch.empty(n, dtype=torch.complex64, device=replica.device)
        _check_samples(out, "out")
        if out.numel() < n:
            raise ValueError("out is shorter than n")
        st = self._lib.replica_spectrum(self._h, replica.data_ptr(), replica.numel(), n, out.data_ptr(),
                                        self._stream(stream))
        if st != RC_OK:
            self._raise(st, "replica_spectrum")
        return out

    def compress_pulse(self, x, spectrum, fs: float, carrier: float, tec: float, direction: str = "correct",
                       out=None, stream=None):
        """Pulse compression with the ionospheric correction in the same pass:
        y = IDFT(DFT(x) conj(R) exp(-/+ i 4 pi K2 / (c f_k))), R from replica_spectrum.  out may be x."""
        torch = _torch()
        _check_samples(x, "x")
        _check_samples(spectrum, "spectrum")
        if spectrum.numel() < x.numel():
            raise ValueError("the spectrum is shorter than x")
        if out is None:
            out = torch.empty_like(x)
        _check_samples(out, "out")
        if out.numel() != x.numel():
            raise ValueError("out must have as many samples as x")
        if direction not in DIRECTIONS:
            raise ValueError(f"direction must be one of {list(DIRECTIONS)}")
        st = self._lib.compress_pulse(self._h, x.data_ptr(), out.data_ptr(), x.numel(), spectrum.data_ptr(),
                                      float(fs), float(carrier), float(tec), DIRECTIONS[direction],
                                      self._stream(stream))
        if st != RC_OK:
            self._raise(st, "compress_pulse")
        return out

    def correct_pulse_batch(self, x_packed, y_packed, pulses, sinc: Sinc | None = None, stream=None):
        """Per-pulse Doppler then ionosphere over packed buffers; `pulses` is a sequence of
        dicts with keys off_in, n_in, off_out, n_out, fs, alpha (or v_r in m/s), tec, carrier and
        optional flags (default Doppler|iono) and direction ("correct"), or a table from pulse_table."""
        _check_samples(x_packed, "x_packed")
        _check_samples(y_packed, "y_packed")
        arr = pulse_array(pulses)
        ptr = arr if isinstance(arr, ctypes.Array) else arr.ctypes.data_as(ctypes.POINTER(RcPulse))
        k = (sinc or Sinc()).c()
        st = self._lib.correct_pulse_batch(self._h, x_packed.data_ptr(), x_packed.numel(), y_packed.data_ptr(),
                                           y_packed.numel(), ptr, len(arr), ctypes.byref(k),
                                           self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_pulse_batch")
        return y_packed

    def batch_plan(self, x_packed, y_packed, pulses, sinc: Sinc | None = None) -> "BatchPlan":
        """correct_pulse_batch(x_packed, y_packed, pulses, sinc) captured once in a HIP graph:
        BatchPlan.launch() replays it (see rc_batch_plan_create)."""
        return BatchPlan(self, x_packed, y_packed, pulses, sinc)

    def correct_doppler_bank(self, x, alphas=None, sinc: Sinc | None = None, n_out: int | None = None,
                             precision: str = "fp16x3", fs: float = 1.0, out=None, stream=None, *, v_r=None):
        """Row h of the (len(alphas), n_out) result is correct_doppler(x, alphas[h]).  Give the
        alphas, or the range rates v_r in m/s (Eq (1) by rc_alpha_from_vr), not both.  precision
        is the filter bank's contraction: "fp16x3", "bf16x3" or "fp32" (set_bank_engine picks the
        filter bank or per-hypothesis resampling)."""
        torch = _torch()
        _check_samples(x, "x")
        n_out = x.numel() if n_out is None else int(n_out)
        if (alphas is None) == (v_r is None):
            raise ValueError("give exactly one of alphas and v_r")
        a = _bank_alphas(alphas if alphas is not None else [_alpha_or_vr(None, v) for v in v_r])
        if out is None:
            out = torch.empty((len(a), n_out), dtype=torch.complex64, device=x.device)
        _check_samples(out, "out")
        if out.numel() < len(a) * n_out:
            raise ValueError("out is shorter than len(alphas) * n_out")
        if precision not in BANK_PRECISIONS:
            raise ValueError(f"precision must be one of {list(BANK_PRECISIONS)}")
        k = (sinc or Sinc()).c()
        st = self._lib.correct_doppler_bank(self._h, x.data_ptr(), x.numel(), out.data_ptr(), n_out, float(fs), a,
                                            len(a), ctypes.byref(k), BANK_PRECISIONS[precision],
                                            self._stream(stream))
        if st != RC_OK:
            self._raise(st, "correct_doppler_bank")
        return out


class BatchPlan:
    """A batch captured in a HIP graph (rc_batch_plan_*).  It keeps its buffers alive."""

    def __init__(self, ctx: "Context", x_packed, y_packed, pulses, sinc: Sinc | None = None):
        _check_samples(x_packed, "x_packed")
        _check_samples(y_packed, "y_packed")
        self._ctx, self._lib = ctx, ctx._lib
        self._x, self._y = x_packed, y_packed
        arr = pulse_array(pulses)
        ptr = arr if isinstance(arr, ctypes.Array) else arr.ctypes.data_as(ctypes.POINTER(RcPulse))
        self._k = (sinc or Sinc()).c()
        h = ctypes.c_void_p()
        st = self._lib.rc_batch_plan_create(ctx._h, x_packed.data_ptr(), x_packed.numel(), y_packed.data_ptr(),
                                            y_packed.numel(), ptr, len(arr), ctypes.byref(self._k), ctypes.byref(h))
        if st != RC_OK:
            ctx._raise(st, "rc_batch_plan_create")
        self._h = h
        self.count = len(arr)

    def launch(self, stream=None):
        st = self._lib.rc_batch_plan_launch(self._h, self._ctx._stream(stream))
        if st != RC_OK:
            self._ctx._raise(st, "rc_batch_plan_launch")
        return self._y

    def update(self, pulses, stream=None):
        """New pulses (same lengths, flags and engines) for the following launches."""
        arr = pulse_array(pulses)
        ptr = arr if isinstance(arr, ctypes.Array) else arr.ctypes.data_as(ctypes.POINTER(RcPulse))
        st = self._lib.rc_batch_plan_update(self._h, ptr, len(arr), self._ctx._stream(stream))
        if st != RC_OK:
            self._ctx._raise(st, "rc_batch_plan_update")

    def close(self):
        if self._h:
            self._lib.rc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A continuous-batching server (rc_server) on a Context: submit single-pulse requests on
    device buffers, wait for tickets, read latency statistics."""

    def __init__(self, ctx: "Context", sinc: Sinc | None = None, mem_budget_bytes: int = 8 << 30,
                 max_batch: int = 256):
        self._ctx = ctx  # keeps the context alive
        self._lib = ctx._lib
        k = (sinc or Sinc()).c()
        h = ctypes.c_void_p()
        st = self._lib.rc_server_create(ctx.handle, ctypes.byref(k), int(mem_budget_bytes), int(max_batch),
                                        ctypes.byref(h))
        if st != RC_OK:
            ctx._raise(st, "rc_server_create")
        self._h = h
        self._held = {}  # ticket -> (x, y): the buffers stay referenced until the ticket is released

    def submit(self, x, y, alpha: float = 1.0, tec: float = 0.0, carrier: float = 0.0, fs: float = 1.0,
               flags: int | None = None, direction: str = "correct", n_out: int | None = None,
               stream=None, charge_only: bool = False) -> int:
        """Queue one pulse: x (device complex64) -> y (device complex64, n_out samples).  The
        request reads x after the work already enqueued on `stream` (default: torch's current
        stream), so x may still be in flight there.  charge_only: return the bytes the request
        would hold against the budget instead of submitting it."""
        _check_samples(x, "x")
        _check_samples(y, "y")
        n_out = y.numel() if n_out is None else int(n_out)
        if n_out > y.numel():
            raise ValueError("y is shorter than n_out")
        fl = (DO_DOPPLER | DO_IONO) if flags is None else int(flags)
        req = RcRequest(x.data_ptr(), y.data_ptr(), x.numel(), n_out, float(fs), float(alpha), float(tec),
                        float(carrier), fl, DIRECTIONS[direction] if isinstance(direction, str) else int(direction),
                        self._ctx._stream(stream))
        t = ctypes.c_int64()
        if charge_only:
            return int(self._lib.rc_server_request_bytes(self._h, ctypes.byref(req)))
        st = self._lib.rc_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != RC_OK:
            self._ctx._raise(st, "rc_server_submit")
        self._held[t.value] = (x, y)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32()
        st = self._lib.rc_server_poll(self._h, int(ticket), ctypes.byref(done))
        if st != RC_OK:
            self._held.pop(int(ticket), None)
            self._ctx._raise(st, "rc_server_poll")
        if done.value:
            self._held.pop(int(ticket), None)
        return bool(done.value)

    def wait(self, ticket: int = 0):
        """Block until `ticket` (0: everything submitted so far) completes."""
        st = self._lib.rc_server_wait(self._h, int(ticket))
        if ticket == 0:
            self._held.clear()
        else:
            self._held.pop(int(ticket), None)
        if st != RC_OK:
            self._ctx._raise(st, "rc_server_wait")

    def stats(self) -> dict:
        s = RcServerStats()
        st = self._lib.rc_server_stats(self._h, ctypes.byref(s))
        if st != RC_OK:
            self._ctx._raise(st, "rc_server_stats")
        return {f: getattr(s, f) for f, _ in RcServerStats._fields_}

    def reset_stats(self):
        st = self._lib.rc_server_reset_stats(self._h)
        if st != RC_OK:
            self._ctx._raise(st, "rc_server_reset_stats")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rc_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bank_alphas(alphas) -> ctypes.Array:
    vals = [float(a) for a in alphas]
    return (ctypes.c_double * len(vals))(*vals)


def pulse_array(pulses):
    """The rc_pulse array for correct_pulse_batch: a sequence of pulse dicts is packed here (about
    3 us per pulse of Python work); a table from `pulse_table` or a ctypes RcPulse array is passed
    through without copying."""
    if isinstance(pulses, ctypes.Array) and pulses._type_ is RcPulse:
        return pulses
    np = _numpy()
    if isinstance(pulses, np.ndarray):
        if pulses.dtype != PULSE_DTYPE or pulses.ndim != 1 or not pulses.flags.c_contiguous:
            raise ValueError("a pulse table must be a contiguous 1-D array of PULSE_DTYPE (see pulse_table)")
        return pulses
    arr = (RcPulse * len(pulses))()
    for i, p in enumerate(pulses):
        d = p.get("direction", "correct")
        alpha = _alpha_or_vr(p.get("alpha"), p.get("v_r")) if ("alpha" in p or "v_r" in p) else 1.0
        arr[i] = RcPulse(int(p["off_in"]), int(p["n_in"]), int(p["off_out"]), int(p["n_out"]),
                         float(p["fs"]), alpha, float(p.get("tec", 0.0)),
                         float(p.get("carrier", 0.0)), int(p.get("flags", DO_DOPPLER | DO_IONO)),
                         DIRECTIONS[d] if isinstance(d, str) else int(d))
    return arr


def _numpy():
    import numpy
    return numpy


def _pulse_dtype():
    np = _numpy()
    dt = np.dtype([(name, {ctypes.c_int64: "<i8", ctypes.c_double: "<f8", ctypes.c_uint32: "<u4",
                           ctypes.c_int32: "<i4"}[ct]) for name, ct in RcPulse._fields_], align=True)
    if dt.itemsize != ctypes.sizeof(RcPulse) or any(
            dt.fields[name][1] != getattr(RcPulse, name).offset for name, _ in RcPulse._fields_):
        raise RuntimeError("numpy layout of rc_pulse differs from the C layout")
    return dt


PULSE_DTYPE = _pulse_dtype()


def pulse_table(off_in, n_in, off_out, n_out, fs, alpha=1.0, tec=0.0, carrier=0.0,
                flags=DO_DOPPLER | DO_IONO, direction="correct"):
    """Descriptor table (numpy array of PULSE_DTYPE, the rc_pulse layout) built column-wise: each
    argument is a scalar or a 1-D array over the pulses, broadcast to a common length."""
    np = _numpy()
    d = DIRECTIONS[direction] if isinstance(direction, str) else direction
    cols = [np.asarray(c) for c in (off_in, n_in, off_out, n_out, fs, alpha, tec, carrier, flags, d)]
    count = max([c.size for c in cols if c.ndim > 0] or [1])
    t = np.zeros(count, dtype=PULSE_DTYPE)
    for name, c in zip(PULSE_DTYPE.names, cols):
        t[name] = np.broadcast_to(c.reshape(-1) if c.ndim else c, (count,))
    return t


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    """Process-wide default context for a device."""
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = _contexts[device] = Context(device)
    return ctx
