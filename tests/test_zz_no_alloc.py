"""correct_ionosphere_noalloc, the entry point that allocates no device memory (its Bluestein
workspace is the library's static per-GPU array), against correct_ionosphere, the entry point
whose kernels it shares, and against the float64 oracle (Eq 15/16).

Outputs are compared bit for bit with correct_ionosphere (same kernels, same arithmetic) and
within the parity bar with the oracle, on consecutive calls whose second input is smaller than
the first, so that the static array still holds the first call's larger contents.
"""
import numpy as np
import pytest

import waveforms as wf
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2508_04951_amd as rc

    return rc.Context(0)


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


FS, FC = 10e6, 450e6


@pytest.mark.parametrize("lengths", [(300001, 70001), (1048575, 4097), (65536, 4096), (70001, 65536)])
def test_noalloc_equals_correct_ionosphere_on_two_calls(torch, ctx, orc, lengths):
    for call, n in enumerate(lengths):
        tec = (40 + 30 * call) * wf.TECU
        direction = ("correct", "distort")[call]
        x = wf.bandlimited_noise(n, wf.rng_for(301, n))
        xd = dev(torch, x)
        yd = torch.empty_like(xd)
        print(f"noalloc call {call}: n={n} {direction}", flush=True)
        ctx.correct_ionosphere_noalloc(xd, yd, FS, FC, tec, direction)
        y = host(yd)
        y_ref = host(ctx.correct_ionosphere(xd, FS, FC, tec, direction))
        assert np.array_equal(y, y_ref), (call, n)
        check(y, orc.ionosphere(x, FS, FC, tec, direction, naive=False), what=(call, n))


def test_noalloc_in_place_and_carrier_zero(torch, ctx, orc):
    n = 70001
    x = wf.bandlimited_noise(n, wf.rng_for(302, n))
    xd = dev(torch, x)
    ctx.correct_ionosphere_noalloc(xd, xd, FS, 0.0, 100 * wf.TECU, "correct")
    check(host(xd), orc.ionosphere(x, FS, 0.0, 100 * wf.TECU, "correct", naive=False))


def test_noalloc_uses_no_context_workspace(torch):
    """With the context's workspace capped at one byte, correct_ionosphere cannot stage a
    Bluestein length, while the static-workspace entry point still runs it."""
    import paper_2508_04951_amd as rc

    c = rc.Context(0)
    c.set_mem_budget(1)
    n = 12345
    x = wf.bandlimited_noise(n, wf.rng_for(303, n))
    xd = dev(torch, x)
    with pytest.raises(rc.RcError):
        c.correct_ionosphere(xd, FS, FC, 50 * wf.TECU, "correct")
    yd = torch.empty_like(xd)
    c.correct_ionosphere_noalloc(xd, yd, FS, FC, 50 * wf.TECU, "correct")
    c2 = rc.Context(0)
    assert np.array_equal(host(yd), host(c2.correct_ionosphere(xd, FS, FC, 50 * wf.TECU, "correct")))


def test_noalloc_rejects_lengths_beyond_the_static_workspace(torch, ctx):
    import paper_2508_04951_amd as rc

    for n in (1048577, 3000001):
        xd = torch.zeros(n, dtype=torch.complex64, device="cuda")
        with pytest.raises(rc.RcError):
            ctx.correct_ionosphere_noalloc(xd, xd, FS, FC, 50 * wf.TECU, "correct")
    # a power of two needs no workspace: the largest one runs
    n = 1 << 22
    x = wf.bandlimited_noise(n, wf.rng_for(304, 0))
    xd = dev(torch, x)
    yd = torch.empty_like(xd)
    ctx.correct_ionosphere_noalloc(xd, yd, FS, FC, 50 * wf.TECU, "correct")
    assert np.array_equal(host(yd), host(ctx.correct_ionosphere(xd, FS, FC, 50 * wf.TECU, "correct")))
