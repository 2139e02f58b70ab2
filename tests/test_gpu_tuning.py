"""GPU tests of the tuning settings (rc_set_fft_levels, rc_set_sinc_grid, rc_set_bluestein_chunk,
rc_load_tuning and RC_TUNE_FILE): the grid and chunk settings give bit-identical results, every
FFT split stays within the parity bar against the oracle, and bad settings are refused."""
import json
import os
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest

import waveforms as wf
from parity import check

pytestmark = pytest.mark.gpu

C = 299792458
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def alpha_exact(v):
    return float(Fraction(C + Fraction(v)) / Fraction(C - Fraction(v)))


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,levels", [(1 << 20, [16, 16]), (1 << 20, [2, 128]), (1 << 22, [4, 256]),
                                      (1 << 22, [16, 4, 16]), (1 << 24, [64, 64]), (1 << 24, [16, 16, 16])])
def test_fft_splits_match_the_oracle(torch, orc, n, levels):
    import paper_2508_04951_amd as rc

    ctx = rc.Context(0, tuning=None)
    ctx.set_fft_levels(n, levels)
    x = wf.bandlimited_noise(n, wf.rng_for(701, n))
    y = host(ctx.correct_ionosphere(torch.from_numpy(x).cuda(), 10e6, 450e6, 60 * wf.TECU, "correct"))
    check(y, orc.ionosphere(x, 10e6, 450e6, 60 * wf.TECU, "correct", naive=False), what=levels)


def test_sinc_grid_and_chunk_are_bit_identical(torch):
    import paper_2508_04951_amd as rc

    P, n = 96, 65536
    v, e = wf.batch_params(P)
    x = torch.from_numpy(np.concatenate([wf.batch_pulse(p) for p in range(P)])).cuda()
    desc = rc.pulse_table(np.arange(P) * n, n, np.arange(P) * n, n, 10e6, alpha=[alpha_exact(q) for q in v],
                          tec=e, carrier=450e6)
    k = rc.Sinc(64, "kaiser", 8.0)
    base = rc.Context(0, tuning=None)
    want = host(base.correct_pulse_batch(x, torch.empty_like(x), desc, k))
    for w in (1, 2):
        c = rc.Context(0, tuning=None)
        c.set_sinc_grid(64, w)
        assert np.array_equal(host(c.correct_pulse_batch(x, torch.empty_like(x), desc, k)), want), w
    lens = [70001, 300001, 99999, 4097, 1000003, 65537]
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]])
    xb = torch.from_numpy(np.concatenate([wf.bandlimited_noise(m, wf.rng_for(702, m)) for m in lens])).cuda()
    d2 = rc.pulse_table(offs, lens, offs, lens, 10e6, tec=40 * wf.TECU, carrier=450e6, flags=rc.DO_IONO)
    want = host(base.correct_pulse_batch(xb, torch.empty_like(xb), d2))
    c = rc.Context(0, tuning=None)
    c.set_bluestein_chunk(1 << 20)  # every pulse its own chunk
    assert np.array_equal(host(c.correct_pulse_batch(xb, torch.empty_like(xb), d2)), want)


def test_load_tuning_and_refusals(torch, tmp_path):
    import paper_2508_04951_amd as rc

    ctx = rc.Context(0, tuning=None)
    good = tmp_path / "t.json"
    good.write_text(json.dumps({"fft_levels": {"1048576": [16, 16]}, "sinc_grid": {"64": 1, "128": 2},
                                "bluestein_chunk_bytes": 1 << 27, "measured_ms": {"anything": [1, 2.5e-3]}}))
    ctx.load_tuning(str(good))
    for bad in ({"fft_levels": {"1048576": [16, 8]}}, {"fft_levels": {"1048576": [512, 2]}},
                {"sinc_grid": {"96": 1}}, {"fft_levels": [1, 2]}):
        p = tmp_path / "bad.json"
        p.write_text(json.dumps(bad))
        with pytest.raises(ValueError):
            ctx.load_tuning(str(p))
    p = tmp_path / "broken.json"
    p.write_text('{"fft_levels": {"1048576": [16, 16]')
    with pytest.raises(ValueError):
        ctx.load_tuning(str(p))
    with pytest.raises(ValueError):
        ctx.load_tuning(str(tmp_path / "missing.json"))
    with pytest.raises(ValueError):
        ctx.set_fft_levels(4096, [1])
    with pytest.raises(ValueError):
        ctx.set_sinc_grid(32, 1)


def test_the_shipped_table_loads(torch):
    import paper_2508_04951_amd as rc
    from paper_2508_04951_amd import _rc

    if not os.path.exists(_rc.TUNING_PATH):
        pytest.skip("no tuning table shipped")
    rc.Context(0, tuning=_rc.TUNING_PATH)


def test_rc_create_reads_rc_tune_file(torch, tmp_path):
    """In a fresh process: RC_TUNE_FILE pointing at a broken file makes rc_create fail."""
    p = tmp_path / "broken.json"
    p.write_text("{")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2508_04951_amd as rc\n"
            "try:\n    rc.Context(0)\nexcept rc.RcError as e:\n    print('refused', e.status)\n") % ROOT
    env = dict(os.environ, RC_TUNE_FILE=str(p))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "refused 1" in out.stdout, (out.stdout, out.stderr)
