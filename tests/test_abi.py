"""CPU checks of the C ABI: the library loads, exports every function include/rc.h
declares, and its host-only entry points (no GPU work) behave as documented."""
import ctypes
import math
import os
import re
from fractions import Fraction

import pytest
import scipy.constants as sc

import paper_2508_04951_amd as rc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"sizeof"})


@pytest.fixture(scope="module")
def lib():
    return rc.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"correct_doppler", "correct_ionosphere", "correct_pulse_batch", "rc_create"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"librc.so does not export {n}"
    assert set(names) == set(rc.SYMBOLS)


def test_status_strings(lib):
    lib.rc_status_string.restype = ctypes.c_char_p
    assert lib.rc_status_string(0) == b"RC_OK"
    assert lib.rc_status_string(1) == b"RC_ERR_INVALID_ARG"
    assert lib.rc_status_string(4) == b"RC_ERR_DEVICE"
    assert lib.rc_status_string(99) == b"RC_ERR_UNKNOWN"


@pytest.mark.parametrize("v", [-8000.0, -1.0, 0.0, 7500.0, 8000.0, 3.0e7, -2.9e8])
def test_alpha_from_vr_is_correctly_rounded(v):
    c = 299792458
    exact = Fraction(c + Fraction(v)) / Fraction(c - Fraction(v))
    a = rc.alpha_from_vr(v)
    ulps = 1 if abs(v) < 0.25 * c else 2
    assert abs(Fraction(a) - exact) <= ulps * Fraction(math.ulp(float(exact)))


@pytest.mark.parametrize("v", [299792458.0, -3e8, float("inf"), float("nan")])
def test_alpha_from_vr_rejects_superluminal(v):
    assert math.isnan(rc.alpha_from_vr(v))


def test_k2_per_tec_matches_codata():
    ref = sc.e ** 2 / (8 * math.pi ** 2 * sc.m_e * sc.epsilon_0)
    assert rc.k2_per_tec() == pytest.approx(ref, rel=1e-14)


def test_null_context_is_rejected(lib):
    k = rc.Sinc().c()
    assert lib.correct_doppler(None, None, 1, None, 1, 1.0, 1.0, ctypes.byref(k), None) == 1
    assert lib.correct_ionosphere(None, None, None, 1, 1.0, 0.0, 0.0, 0, None) == 1
    assert lib.correct_pulse_batch(None, None, 1, None, 1, None, 0, ctypes.byref(k), None) == 1
    assert lib.rc_sync(None, None) == 1
    assert lib.rc_destroy(None) == 1
    assert lib.rc_create(0, None) == 1


def test_create_without_a_device_fails_cleanly(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.rc_create(0, ctypes.byref(h)) == 1 and not h.value


def test_struct_layouts_match_header():
    assert ctypes.sizeof(rc._rc.RcSinc) == 16
    assert ctypes.sizeof(rc._rc.RcPulse) == 72


def test_pulse_table_matches_the_dict_packing():
    import numpy as np

    P, n = 37, 4096
    rng = np.random.default_rng(5)
    alpha = 1.0 + rng.uniform(-5e-5, 5e-5, P)
    tec = rng.uniform(5e16, 1e18, P)
    flags = rng.integers(1, 4, P)
    dirs = ["correct" if p % 3 else "distort" for p in range(P)]
    d = [dict(off_in=p * n, n_in=n, off_out=p * (n + 7), n_out=n + 7, fs=10e6, alpha=float(alpha[p]),
              tec=float(tec[p]), carrier=450e6, flags=int(flags[p]), direction=dirs[p]) for p in range(P)]
    t = rc.pulse_table(np.arange(P) * n, n, np.arange(P) * (n + 7), n + 7, 10e6, alpha=alpha, tec=tec,
                       carrier=450e6, flags=flags, direction=np.array([rc.DIRECTIONS[x] for x in dirs]))
    assert t.dtype == rc.PULSE_DTYPE and t.dtype.itemsize == ctypes.sizeof(rc._rc.RcPulse)
    assert bytes(rc.pulse_array(d)) == t.tobytes()
    assert rc.pulse_array(t) is t  # passed through without a copy


def test_pulse_dicts_take_a_range_rate():
    """A pulse may give v_r (m/s) instead of alpha: the library's Eq (1) fills alpha; giving
    both, or |v_r| >= c, is an argument error."""
    base = dict(off_in=0, n_in=16, off_out=0, n_out=16, fs=10e6)
    arr = rc.pulse_array([dict(base, v_r=7500.0), dict(base, alpha=1.25), dict(base)])
    assert arr[0].alpha == rc.alpha_from_vr(7500.0)
    assert arr[1].alpha == 1.25 and arr[2].alpha == 1.0
    with pytest.raises(ValueError):
        rc.pulse_array([dict(base, v_r=10.0, alpha=1.0)])
    with pytest.raises(ValueError):
        rc.pulse_array([dict(base, v_r=3e8)])


def test_pulse_table_rejects_other_layouts():
    import numpy as np

    t = rc.pulse_table(np.arange(4) * 8, 8, np.arange(4) * 8, 8, 1.0)
    with pytest.raises(ValueError):
        rc.pulse_array(t[::2])  # not contiguous
    with pytest.raises(ValueError):
        rc.pulse_array(np.zeros(4, dtype=np.float64))


def test_empty_pulse_table():
    t = rc.pulse_table([], [], [], [], [])
    assert t.dtype == rc.PULSE_DTYPE and t.shape == (0,)
    assert len(rc.pulse_array(t)) == 0
