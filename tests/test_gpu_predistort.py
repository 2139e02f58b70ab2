"""The GPU ionospheric operator against LFM predistortion, on the Fig. 2 setup (Sec. II-C):
413-431 MHz LFM of 100 us sampled at 2.048 GHz in a 2^19-sample record, 1e18 el/m^2.

The cubic-root predistortion (``oracle.predistort``) is built from Eq (4)-(12) alone, so these
tests check the HIP path's Eq (15)/(16) against an independent construction, on top of its
element-wise parity with the oracle.
"""
import numpy as np
import pytest

from oracle import predistort as pd

pytestmark = pytest.mark.gpu

F0, BW, T, FS, E = 413e6, 18e6, 100e-6, 2.048e9, 1e18
N = 1 << 19
N0 = N // 4
LOSS_MAX_DB = 0.01  # the Fig. 2 caption's bound


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2508_04951_amd as rc

    return rc.Context(0)


@pytest.fixture(scope="module")
def waves():
    k2 = pd.k2_from_tec(E)
    args = (N, N0, FS, F0, BW, T)
    return dict(lfm=pd.lfm(*args).astype(np.complex64), cubic=pd.cubic_waveform(*args, k2))


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def host(torch, t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def test_gpu_correction_is_the_cubic_predistortion(torch, ctx, orc, waves):
    y = host(torch, ctx.correct_ionosphere(dev(torch, waves["lfm"]), FS, 0.0, E, "correct"))
    loss_gpu = pd.snr_loss_db(waves["cubic"], y)
    loss_orc = pd.snr_loss_db(waves["cubic"], orc.ionosphere(waves["lfm"], FS, 0.0, E, "correct"))
    assert loss_gpu < LOSS_MAX_DB
    assert abs(loss_gpu - loss_orc) < 1e-5  # float32 transforms: ~1e-7 relative per sample


def test_gpu_bluestein_correction_is_the_cubic_predistortion(torch, ctx, orc):
    """The same check on a record of 500000 samples, which takes Bluestein's path."""
    n = 500000
    n0 = n // 4
    k2 = pd.k2_from_tec(E)
    lfm = pd.lfm(n, n0, FS, F0, BW, T).astype(np.complex64)
    cubic = pd.cubic_waveform(n, n0, FS, F0, BW, T, k2)
    y = host(torch, ctx.correct_ionosphere(dev(torch, lfm), FS, 0.0, E, "correct"))
    loss_gpu = pd.snr_loss_db(cubic, y)
    loss_orc = pd.snr_loss_db(cubic, orc.ionosphere(lfm, FS, 0.0, E, "correct", naive=False))
    assert loss_gpu < LOSS_MAX_DB
    assert abs(loss_gpu - loss_orc) < 1e-5


def test_gpu_distortion_of_the_predistortion_is_the_lfm(torch, ctx, waves):
    y = host(torch, ctx.correct_ionosphere(dev(torch, waves["cubic"]), FS, 0.0, E, "distort"))
    assert pd.snr_loss_db(waves["lfm"].astype(np.complex128), y) < LOSS_MAX_DB


def test_gpu_compression_restores_the_matched_filter_peak(torch, ctx, orc, waves):
    """The LFM goes out, the two-way ionosphere disperses it (Eq (15), oracle), and the GPU
    compresses it against the LFM replica with the correction in the same pass: the peak is the
    undispersed matched-filter peak at the pulse's position, within the Fig. 2 bound."""
    lfm = waves["lfm"]
    rx = orc.ionosphere(lfm, FS, 0.0, E, "distort")
    n_rep = int(np.ceil(T * FS))
    spec = ctx.replica_spectrum(dev(torch, lfm[N0:N0 + n_rep]), N)
    energy = float(np.sum(np.abs(lfm.astype(np.complex128)) ** 2))
    y = host(torch, ctx.compress_pulse(dev(torch, rx), spec, FS, 0.0, E, "correct"))
    assert int(np.argmax(np.abs(y))) == N0
    assert -20 * np.log10(np.abs(y).max() / energy) < LOSS_MAX_DB
    y0 = host(torch, ctx.compress_pulse(dev(torch, rx), spec, FS, 0.0, 0.0))
    assert -20 * np.log10(np.abs(y0).max() / energy) > 1.0  # uncorrected: the dispersion costs dB
