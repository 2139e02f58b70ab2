"""Autotuner: times the library's tunable launch shapes on this GPU and writes the fastest as
the JSON table that rc_load_tuning reads (and rc_create, through RC_TUNE_FILE).

    python -m paper_2508_04951_amd.tune [--out paper_2508_04951_amd/tuning.json] [--quick]

What it sweeps, each on a workload of the shape it serves, timed with HIP events over repeated
calls after a warm-up (the best of several rounds):
  * fft_levels    the strided-level split of the 2^20, 2^22 and 2^24-point transforms (every
                  split into one to three powers of two in [2, 256]), on ionosphere-only batches;
                  2^16 and below have a single split;
  * sinc_grid     workgroups per CU of the matrix-core resampler at H = 64 (the 1024 x 65536
                  batch) and H = 128 (8 x 2^24 long pulses), Doppler-only batches;
  * bluestein_chunk_bytes  the workspace cap of a Bluestein launch sequence, on a batch of
                  ionosphere-only pulses of lengths that are not powers of two.
The grid and chunk settings give bit-identical results and a split only reorders the float32
roundings of the transform (the tests check both); the table also records each candidate's time.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def splits(n_strided_log2: int):
    """Every ordered split of 2^n_strided_log2 into 1..3 factors, each a power of two in [2, 256]."""
    out = []
    for parts in (1, 2, 3):
        for c in itertools.product(range(1, 9), repeat=parts):
            if sum(c) == n_strided_log2:
                out.append([1 << v for v in c])
    return out


def best_time(torch, fn, reps: int, rounds: int = 3) -> float:
    """ms per call: the best of `rounds` timings of `reps` back-to-back calls."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(rounds):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / reps)
    return best


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--quick", action="store_true", help="fewer repetitions (a smoke run)")
    args = ap.parse_args()
    import torch

    import paper_2508_04951_amd as rc

    assert torch.cuda.is_available(), "the autotuner needs the GPU"
    reps = 3 if args.quick else 10
    table = {"device": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
             "fft_levels": {}, "sinc_grid": {}, "measured_ms": {}}
    ctx = rc.Context(0, tuning=None)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    # --- FFT level splits: ionosphere-only batches of 2^28 samples (2 GiB in, in place) -----------
    for log2n in (20, 22, 24):
        n = 1 << log2n
        pulses = (1 << 28) // n
        x = torch.randn(pulses * n, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        desc = rc.pulse_table(np.arange(pulses) * n, n, np.arange(pulses) * n, n, 10e6, tec=50 * 1e16,
                              carrier=450e6, flags=rc.DO_IONO)
        meas = {}
        for lv in splits(log2n - 12):
            ctx.set_fft_levels(n, lv)
            meas[json.dumps(lv)] = best_time(torch, lambda: ctx.correct_pulse_batch(x, y, desc), reps)
            log(f"[tune] 2^{log2n} levels {lv}: {meas[json.dumps(lv)]:.3f} ms")
        ctx.set_fft_levels(n, [])
        best = min(meas, key=meas.get)
        table["fft_levels"][str(n)] = json.loads(best)
        table["measured_ms"][f"fft_{n}_x{pulses}"] = meas
        del x, y
        torch.cuda.empty_cache()

    # --- matrix-core resampler grid: Doppler-only batches ------------------------------------
    for hw, n, pulses in ((64, 65536, 1024), (128, 1 << 24, 8)):
        x = torch.randn(pulses * n, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        rng = np.random.default_rng(1)
        alphas = 1.0 + 2.0 * rng.uniform(-8000, 8000, pulses) / 299792458.0
        desc = rc.pulse_table(np.arange(pulses) * n, n, np.arange(pulses) * n, n, 10e6, alpha=alphas,
                              flags=rc.DO_DOPPLER)
        k = rc.Sinc(hw, "kaiser", 8.0)
        meas = {}
        for w in (1, 2, 0):
            ctx.set_sinc_grid(hw, w)
            meas[str(w)] = best_time(torch, lambda: ctx.correct_pulse_batch(x, y, desc, k), reps)
            log(f"[tune] H={hw} grid {w} per CU: {meas[str(w)]:.3f} ms")
        ctx.set_sinc_grid(hw, 0)
        table["sinc_grid"][str(hw)] = int(min(meas, key=meas.get))
        table["measured_ms"][f"sinc_h{hw}_{pulses}x{n}"] = meas
        del x, y
        torch.cuda.empty_cache()

    # --- Bluestein chunk cap: 64 ionosphere-only pulses of lengths near 2^20 -----------------
    rng = np.random.default_rng(2)
    lens = rng.integers(600000, 1048575, 64)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
    x = torch.randn(int(lens.sum()), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    desc = rc.pulse_table(offs, lens, offs, lens, 10e6, tec=50 * 1e16, carrier=450e6, flags=rc.DO_IONO)
    meas = {}
    for mib in (64, 128, 256, 512, 1024):
        ctx.set_bluestein_chunk(mib << 20)
        meas[str(mib << 20)] = best_time(torch, lambda: ctx.correct_pulse_batch(x, y, desc), max(1, reps // 3))
        log(f"[tune] Bluestein chunk {mib} MiB: {meas[str(mib << 20)]:.3f} ms")
    table["bluestein_chunk_bytes"] = int(min(meas, key=meas.get))
    table["measured_ms"]["bluestein_chunk_64_pulses"] = meas
    table["written"] = time.strftime("%Y-%m-%d %H:%M:%S")
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({k: table[k] for k in ("fft_levels", "sinc_grid", "bluestein_chunk_bytes")}))


if __name__ == "__main__":
    main()
