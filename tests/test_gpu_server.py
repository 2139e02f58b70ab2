"""GPU tests of the continuous-batching server (rc_server_*, through the C ABI): every request's
output equals, bit for bit, the same pulse run alone through correct_doppler and
correct_ionosphere, whatever it was batched with; admission by bytes; statistics."""
from fractions import Fraction

import numpy as np
import pytest

import waveforms as wf
from parity import check

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


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def alone(torch, ctx, x, r, k):
    """The single-pulse entry points on one request."""
    import paper_2508_04951_amd as rc

    y = x
    if r["flags"] & rc.DO_DOPPLER:
        y = ctx.correct_doppler(x, r["alpha"], k, n_out=r["n_out"])
    if r["flags"] & rc.DO_IONO:
        y = ctx.correct_ionosphere(y, 10e6, 450e6, r["tec"], r["direction"])
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_server_mixed_stream_equals_single_calls(torch, ctx, orc):
    import paper_2508_04951_amd as rc

    rng = wf.rng_for(301, 0)
    lens = [int(n) for n in wf.loguniform_lengths(30, rng, 8.0, 18.0)] + [4096, 65536, 1 << 17, 5000, 1]
    k = rc.Sinc(64, "kaiser", 8.0)
    srv = rc.Server(ctx, k, mem_budget_bytes=1 << 32, max_batch=7)
    reqs, tickets = [], []
    for i, n in enumerate(lens):
        flags = [rc.DO_DOPPLER | rc.DO_IONO, rc.DO_DOPPLER, rc.DO_IONO][i % 3]
        v = rng.uniform(-8000, 8000) if i % 5 else rng.uniform(9000, 20000)  # some off the matrix cores
        r = dict(n=n, n_out=n + (i % 4) * 7 if flags == rc.DO_DOPPLER else n, alpha=alpha_exact(v),
                 tec=rng.uniform(5, 100) * wf.TECU, flags=flags, direction="distort" if i % 7 == 3 else "correct")
        x = dev(torch, wf.bandlimited_noise(n, wf.rng_for(301, i + 1)) if n > 1 else np.array([1 - 1j], np.complex64))
        y = torch.full((r["n_out"],), complex("nan"), dtype=torch.complex64, device="cuda")
        tickets.append(srv.submit(x, y, alpha=r["alpha"], tec=r["tec"], carrier=450e6, fs=10e6, flags=flags,
                                  direction=r["direction"]))
        reqs.append((r, x, y))
    srv.wait(tickets[3])
    srv.wait()
    for i, (r, x, y) in enumerate(reqs):
        got = y.cpu().numpy()
        assert not np.isnan(got).any(), i
        assert np.array_equal(got, alone(torch, ctx, x, r, k)), i
    st = srv.stats()
    assert st["submitted"] == st["completed"] == len(lens)
    assert st["batches"] >= 1 and 1.0 <= st["mean_batch"] <= 7.0
    assert 0.0 < st["latency_ms_p50"] <= st["latency_ms_p99"] <= st["latency_ms_max"]
    assert st["samples_per_s"] > 0
    # every request against the oracle
    for i in range(len(reqs)):
        r, x, y = reqs[i]
        xh = x.cpu().numpy()
        ref = orc.correct_pulse(xh, 10e6, r["alpha"], r["tec"], 450e6, n_out=r["n_out"], half_width=64,
                                doppler_on=bool(r["flags"] & rc.DO_DOPPLER), iono_on=bool(r["flags"] & rc.DO_IONO),
                                direction=r["direction"])
        got = y.cpu().numpy()
        check(got, ref, what=i)
    srv.close()


def test_server_long_requests_against_the_oracle(torch, ctx, orc):
    """Requests up to the serving workload's longest length (2^22) and lengths that are not
    powers of two, submitted back to back so that they share batches: every request against the
    oracle (the full pulse, or, for the two longest Doppler-only requests, sampled outputs of the
    direct sum) and bit for bit against its single-pulse calls."""
    import paper_2508_04951_amd as rc

    rng = wf.rng_for(303, 0)
    lens = [1 << 22, (1 << 22) - 12345, 1 << 20, 3000001, 70001, 1 << 16, 4096, 262143]
    flag_set = [rc.DO_DOPPLER | rc.DO_IONO, rc.DO_DOPPLER, rc.DO_IONO, rc.DO_DOPPLER | rc.DO_IONO, rc.DO_IONO,
                rc.DO_DOPPLER | rc.DO_IONO, rc.DO_DOPPLER, rc.DO_DOPPLER | rc.DO_IONO]
    k = rc.Sinc(64, "kaiser", 8.0)
    srv = rc.Server(ctx, k, mem_budget_bytes=1 << 33, max_batch=16)
    reqs = []
    for i, (n, flags) in enumerate(zip(lens, flag_set)):
        r = dict(n=n, n_out=n, alpha=alpha_exact(rng.uniform(-8000, 8000)), tec=rng.uniform(5, 100) * wf.TECU,
                 flags=flags, direction="distort" if i == 4 else "correct")
        xh = wf.bandlimited_noise(n, wf.rng_for(303, i + 1))
        x = dev(torch, xh)
        y = torch.full((n,), complex("nan"), dtype=torch.complex64, device="cuda")
        torch.cuda.synchronize()
        srv.submit(x, y, alpha=r["alpha"], tec=r["tec"], carrier=450e6, fs=10e6, flags=flags,
                   direction=r["direction"])
        reqs.append((r, xh, x, y))
    srv.wait()
    for i, (r, xh, x, y) in enumerate(reqs):
        got = y.cpu().numpy()
        assert np.array_equal(got, alone(torch, ctx, x, r, k)), i
        if r["flags"] == rc.DO_DOPPLER and r["n"] > (1 << 18):
            idx = np.concatenate([np.arange(3000), np.arange(r["n"] - 3000, r["n"]),
                                  wf.rng_for(303, 100 + i).integers(0, r["n"], 6000)])
            check(got[idx], orc.doppler_at(xh, idx, r["alpha"], 64, "kaiser", 8.0), what=i)
        else:
            ref = orc.correct_pulse(xh, 10e6, r["alpha"], r["tec"], 450e6, n_out=r["n_out"], half_width=64,
                                    doppler_on=bool(r["flags"] & rc.DO_DOPPLER),
                                    iono_on=bool(r["flags"] & rc.DO_IONO), direction=r["direction"])
            check(got, ref, what=i)
    srv.close()


def test_server_admission_poll_and_errors(torch, ctx):
    import paper_2508_04951_amd as rc

    n = 1 << 24  # ~0.6 ms of device work per request: far longer than the next submit call
    x = dev(torch, wf.bandlimited_noise(n, wf.rng_for(302, 0)))
    ys = [torch.empty(n, dtype=torch.complex64, device="cuda") for _ in range(4)]
    # a budget of three requests: their samples (16 B each), descriptors and tile lists
    probe = rc.Server(ctx, rc.Sinc(64), mem_budget_bytes=1 << 40, max_batch=16)
    charge = max(probe.submit(x, ys[0], alpha=alpha_exact(1000.0 * i), tec=20 * wf.TECU, carrier=450e6, fs=10e6,
                              charge_only=True) for i in range(4))
    probe.close()
    assert 16 * n < charge < 16 * n + (1 << 20)
    srv = rc.Server(ctx, rc.Sinc(64), mem_budget_bytes=3 * charge + 1000, max_batch=16)
    t = [srv.submit(x, ys[i], alpha=alpha_exact(1000.0 * i), tec=20 * wf.TECU, carrier=450e6, fs=10e6)
         for i in range(3)]
    with pytest.raises(rc.RcError) as ei:  # the fourth does not fit while three are in flight
        srv.submit(x[:1024], ys[3][:1024], alpha=1.0)
    assert ei.value.status == 5  # RC_ERR_BUSY
    srv.wait(t[0])
    srv.wait(t[1])
    t3 = srv.submit(x, ys[3], alpha=alpha_exact(3000.0), tec=20 * wf.TECU, carrier=450e6, fs=10e6)
    while not srv.poll(t3):
        pass
    with pytest.raises(ValueError):
        srv.poll(t3)  # released
    with pytest.raises(rc.RcError) as ei:  # could never fit
        big = torch.empty(4 * n, dtype=torch.complex64, device="cuda")
        srv.submit(big, torch.empty_like(big), flags=rc.DO_DOPPLER, alpha=alpha_exact(500.0))
    assert ei.value.status == 2
    with pytest.raises(ValueError):
        srv.submit(x, ys[0], alpha=float("nan"))
    with pytest.raises(ValueError):
        srv.submit(x, x, alpha=1.1)  # Doppler in place
    st = srv.stats()
    assert st["rejected"] == 2 and st["completed"] == 4
    srv.wait()
    srv.reset_stats()
    assert srv.stats()["completed"] == 0
    srv.close()


def test_server_budget_bounds_the_context_workspace(torch):
    """With the context's workspace capped at the server's budget, a stream of Bluestein-length
    and matrix-core requests (each charged its own workspace) never needs more: every request
    completes and equals its single-pulse calls on an unbounded context."""
    import paper_2508_04951_amd as rc

    budget = 96 << 20
    c = rc.Context(0)
    c.set_mem_budget(budget)
    ref_ctx = rc.Context(0)
    k = rc.Sinc(64, "kaiser", 8.0)
    srv = rc.Server(c, k, mem_budget_bytes=budget, max_batch=8)
    rng = wf.rng_for(305, 0)
    lens = [300001, 70001, 1 << 20, 12345, 500000, 1 << 18, 262143, 99999, 700001, 4097] * 2
    done = []
    pending = []
    for i, n in enumerate(lens):
        r = dict(n=n, n_out=n, alpha=alpha_exact(rng.uniform(-8000, 8000)), tec=rng.uniform(5, 100) * wf.TECU,
                 flags=rc.DO_DOPPLER | rc.DO_IONO, direction="correct")
        x = dev(torch, wf.bandlimited_noise(n, wf.rng_for(305, i + 1)))
        y = torch.empty_like(x)
        while True:
            try:
                t = srv.submit(x, y, alpha=r["alpha"], tec=r["tec"], carrier=450e6, fs=10e6, flags=r["flags"])
                break
            except rc.RcError as e:
                assert e.status == 5, e  # only RC_ERR_BUSY: wait for the oldest and retry
                srv.wait(pending.pop(0)[0])
        pending.append((t, r, x, y))
        done.append((r, x, y))
    srv.wait()
    srv.close()
    for r, x, y in done:
        assert np.array_equal(y.cpu().numpy(), alone(torch, ref_ctx, x, r, k)), r["n"]


def test_server_reads_x_after_the_submitting_stream(torch, ctx):
    """x is produced on a side stream and submitted without a host synchronisation: the request
    waits for that stream's work, so it sees the finished x."""
    import paper_2508_04951_amd as rc

    n = 1 << 20
    xh = wf.bandlimited_noise(n, wf.rng_for(306, 0))
    src = dev(torch, xh)
    k = rc.Sinc(64, "kaiser", 8.0)
    srv = rc.Server(ctx, k, mem_budget_bytes=1 << 32, max_batch=4)
    side = torch.cuda.Stream()
    outs = []
    for i in range(4):
        x = torch.zeros(n, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(20):  # a queue of work ahead of the copy that fills x
                torch.mul(src, 1.0, out=y)
            x.copy_(src)
            t = srv.submit(x, y, alpha=alpha_exact(1500.0 * i), tec=30 * wf.TECU, carrier=450e6, fs=10e6)
        outs.append((t, i, x, y))
    srv.wait()
    srv.close()
    r = dict(n_out=n, flags=rc.DO_DOPPLER | rc.DO_IONO, direction="correct", tec=30 * wf.TECU)
    for t, i, x, y in outs:
        rr = dict(r, alpha=alpha_exact(1500.0 * i))
        assert np.array_equal(y.cpu().numpy(), alone(torch, ctx, src, rr, k)), i
