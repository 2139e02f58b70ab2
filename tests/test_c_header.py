"""include/rc.h as a C program sees it: the header compiles as C11, its struct layouts match the
ctypes mirrors the Python binding passes, and a C program linked against librc.so gets the same
host-side results as the binding (no GPU is touched)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2508_04951_amd as rc
from paper_2508_04951_amd import _rc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
PKG = os.path.dirname(os.path.abspath(_rc.__file__))

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def _program():
    sizes = {
        "rc_c64": 8,
        "rc_sinc": ctypes.sizeof(_rc.RcSinc),
        "rc_pulse": ctypes.sizeof(_rc.RcPulse),
        "rc_request": ctypes.sizeof(_rc.RcRequest),
        "rc_server_stats_t": ctypes.sizeof(_rc.RcServerStats),
    }
    asserts = "\n".join(f'_Static_assert(sizeof({t}) == {n}, "{t} layout");' for t, n in sizes.items())
    offsets = "\n".join(
        f'_Static_assert(offsetof(rc_pulse, {f}) == {getattr(_rc.RcPulse, f).offset}, "rc_pulse.{f}");'
        for f, _ in _rc.RcPulse._fields_)
    return f"""
#include <stddef.h>
#include <stdio.h>
#include "rc.h"
{asserts}
{offsets}
int main(void)
{{
    printf("%.17g %.17g %d\\n", rc_alpha_from_vr(7500.0), rc_k2_per_tec(), (int)RC_ERR_OUT_OF_MEMORY);
    printf("%s\\n", rc_status_string(RC_ERR_UNSUPPORTED));
    return 0;
}}
"""


def test_header_compiles_as_c_with_the_binding_layouts(tmp_path):
    src = tmp_path / "abi.c"
    src.write_text(_program())
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", INCLUDE, "-c", str(src),
                        "-o", str(tmp_path / "abi.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(not os.path.exists(os.path.join(PKG, "librc.so")), reason="librc.so not built")
def test_c_program_linked_against_the_library(tmp_path):
    src = tmp_path / "abi.c"
    src.write_text(_program())
    exe = tmp_path / "abi"
    r = subprocess.run(["gcc", "-std=c11", "-I", INCLUDE, str(src), "-o", str(exe), "-L", PKG, "-lrc",
                        f"-Wl,-rpath,{PKG}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    first, second = out.stdout.strip().splitlines()
    alpha, k2, oom = first.split()
    assert float(alpha) == rc.alpha_from_vr(7500.0)
    assert float(k2) == rc.k2_per_tec()
    assert int(oom) == 3
    assert second == _rc.load_library().rc_status_string(2).decode()
