"""GPU tests of batch plans (rc_batch_plan_*: one correct_pulse_batch captured in a HIP graph and
replayed), through the C ABI.  Every replay is compared bit for bit with the eager
correct_pulse_batch call on the same arguments, with eager work and synchronisations between
replays; updates with new Doppler factors and TEC are compared the same way, and updates that
would need other launches are refused."""
from fractions import Fraction

import numpy as np
import pytest

import waveforms as wf

pytestmark = pytest.mark.gpu

C = 299792458


def alpha_exact(v):
    return float(Fraction(C + Fraction(v)) / Fraction(C - Fraction(v)))


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2508_04951_amd as rc

    return rc.Context(0)


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def mixed_batch(seed, vmax=8000.0):
    """Matrix-core, vector-tile and direct-sum Doppler pulses, power-of-two and Bluestein
    ionosphere lengths, a copy-only pulse, packed with gaps."""
    import paper_2508_04951_amd as rc

    rng = wf.rng_for(seed, 0)
    specs = [(65536, 3), (4096, 3), (8192, 1), (1000, 1), (65536, 2), (256, 3), (1 << 17, 3), (4096, 2),
             (3000, 0), (16, 3), (5000, 3), (70001, 2), (12, 3), (70001, 3)] + [(65536, 3)] * 40
    pulses, xs = [], []
    off_in = off_out = 5
    for i, (n, flags) in enumerate(specs):
        xs.append(wf.bandlimited_noise(n, wf.rng_for(seed, i + 1)))
        v = rng.uniform(-vmax, vmax) if i != 7 else 1.2e6  # one pulse on the direct sum
        pulses.append(dict(off_in=off_in, n_in=n, off_out=off_out, n_out=n, fs=10e6, alpha=alpha_exact(v),
                           tec=rng.uniform(5, 100) * wf.TECU, carrier=450e6,
                           flags=flags if flags else 0, direction="distort" if i % 4 == 3 else "correct"))
        off_in += n + 3
        off_out += n + 11
    pulses[8]["n_out"] = pulses[8]["n_in"]
    return pulses, xs, off_in, off_out


def packed(torch, pulses, xs, x_len):
    xp = np.zeros(x_len, np.complex64)
    for p, x in zip(pulses, xs):
        xp[p["off_in"]:p["off_in"] + p["n_in"]] = x
    return torch.from_numpy(xp).cuda()


def test_plan_replays_equal_the_eager_call(torch, ctx):
    import paper_2508_04951_amd as rc

    pulses, xs, x_len, y_len = mixed_batch(601)
    xd = packed(torch, pulses, xs, x_len)
    k = rc.Sinc(64)
    ref = torch.full((y_len,), complex("nan"), dtype=torch.complex64, device="cuda")
    ctx.correct_pulse_batch(xd, ref, pulses, k)
    want = host(ref)
    yd = torch.full((y_len,), complex("nan"), dtype=torch.complex64, device="cuda")
    plan = ctx.batch_plan(xd, yd, pulses, k)
    for rep in range(5):
        yd.fill_(float("nan"))  # eager work between the replays
        plan.launch()
        got = host(yd)
        assert np.array_equal(got, want, equal_nan=True), rep
        ctx.correct_pulse_batch(xd, ref, pulses, k)  # the eager path between replays too
    # replays on another stream, back to back, then checked
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            plan.launch()
    s.synchronize()
    assert np.array_equal(host(yd), want, equal_nan=True)
    plan.close()


def test_plan_update_new_alphas_and_tec(torch, ctx):
    import paper_2508_04951_amd as rc

    pulses, xs, x_len, y_len = mixed_batch(602, vmax=5000.0)
    xd = packed(torch, pulses, xs, x_len)
    k = rc.Sinc(64)
    yd = torch.zeros(y_len, dtype=torch.complex64, device="cuda")  # the gaps between pulses stay 0
    ref = torch.zeros_like(yd)
    plan = ctx.batch_plan(xd, yd, pulses, k)
    rng = wf.rng_for(602, 99)
    for rep in range(3):
        new = [dict(p) for p in pulses]
        for i, p in enumerate(new):
            if i != 7:  # keep the direct-sum pulse off the fast paths
                p["alpha"] = alpha_exact(rng.uniform(-5000, 5000))
            p["tec"] = rng.uniform(5, 100) * wf.TECU
            p["direction"] = "correct" if (i + rep) % 3 else "distort"
        plan.update(new)
        plan.launch()
        ctx.correct_pulse_batch(xd, ref, new, k)
        assert np.array_equal(host(yd), host(ref)), rep
    # an update that moves a pulse to another resampling engine needs another graph
    bad = [dict(p) for p in pulses]
    bad[0]["alpha"] = alpha_exact(2e5)
    with pytest.raises(rc.RcError) as ei:
        plan.update(bad)
    assert ei.value.status == 2
    bad = [dict(p) for p in pulses]
    bad[1]["n_out"] = 2048
    with pytest.raises(rc.RcError):
        plan.update(bad)
    with pytest.raises(ValueError):
        plan.update(pulses[:-1])
    # the refused updates left the plan as it was
    plan.launch()
    ctx.correct_pulse_batch(xd, ref, new, k)
    assert np.array_equal(host(yd), host(ref))
    plan.close()


def test_plan_on_the_batch_workload_shape(torch, ctx):
    """64 pulses of the batch workload (65536 samples, H = 64, v_r ~ U[-8, 8] km/s): the plan's
    replays equal the eager call bit for bit."""
    import paper_2508_04951_amd as rc

    P, n = 64, 65536
    v, e = wf.batch_params(P)
    xh = np.concatenate([wf.batch_pulse(p) for p in range(P)])
    xd = torch.from_numpy(xh).cuda()
    pulses = rc.pulse_table(np.arange(P) * n, n, np.arange(P) * n, n, 10e6,
                            alpha=[alpha_exact(q) for q in v], tec=e, carrier=450e6)
    k = rc.Sinc(64, "kaiser", 8.0)
    yd, ref = torch.empty_like(xd), torch.empty_like(xd)
    ctx.correct_pulse_batch(xd, ref, pulses, k)
    plan = ctx.batch_plan(xd, yd, pulses, k)
    for _ in range(3):
        plan.launch()
        assert np.array_equal(host(yd), host(ref))
    plan.close()


def test_plan_rejects_bad_arguments(torch, ctx):
    import paper_2508_04951_amd as rc

    x = torch.zeros(100, dtype=torch.complex64, device="cuda")
    y = torch.zeros(100, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        ctx.batch_plan(x, y, [])
    with pytest.raises(ValueError):
        ctx.batch_plan(x, y, [dict(off_in=0, n_in=200, off_out=0, n_out=200, fs=1.0, alpha=1.0)])
    with pytest.raises(ValueError):
        ctx.batch_plan(x, x, [dict(off_in=0, n_in=100, off_out=0, n_out=100, fs=1.0, alpha=1.0)])
