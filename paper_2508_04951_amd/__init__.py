"""MI355X-native (gfx950) Doppler and ionospheric correction of sampled arbitrary waveforms
(Vickers, Mack & Osaretin, arXiv 2508.04951).

The compute lives in librc.so (hand-written HIP kernels behind the C ABI of include/rc.h);
this package is its Python binding.  torch supplies device memory and streams.
"""
from ._rc import (BANK_ENGINES, BANK_PRECISIONS, DIRECTIONS, DO_DOPPLER, DO_IONO, KERNELS, PAPER_VARIANTS,
                  SINC_ENGINES, SYMBOLS, WINDOWS, BatchPlan, Context, RcError, Server, Sinc, alpha_from_vr, context, k2_per_tec,
                  load_library, pq_length, pulse_array, PULSE_DTYPE, pulse_table)

__all__ = [
    "BatchPlan", "Context", "RcError", "Server", "Sinc", "BANK_ENGINES", "BANK_PRECISIONS", "PAPER_VARIANTS", "alpha_from_vr",
    "k2_per_tec", "context", "load_library", "pq_length", "pulse_array", "pulse_table", "PULSE_DTYPE", "KERNELS",
    "SINC_ENGINES", "DIRECTIONS", "WINDOWS", "DO_DOPPLER", "DO_IONO", "SYMBOLS",
]
