"""The C ABI from a C program alone (tests/c_abi_example.c, built by the package build next to
this file): device buffers from hipMalloc, correct_ionosphere on a single-bin tone, the result
checked against its closed form inside the program."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi_example")


def test_c_program_corrects_a_tone():
    assert os.path.exists(EXE), "tests/c_abi_example is missing: run the package build"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert r.stdout.startswith("ok "), r.stdout
