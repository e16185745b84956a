"""The C ABI from a plain C program (tests/c_abi/plic_abi_check.c, built by
__graft_entry__.build()): device buffers from hipMalloc, the caller's own
stream, every solver's round trip and complement, the curvature of a plane
and of a lattice without interface, and the status codes of rejected calls.
It runs as a child process and exits 0 when every check passed."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "plic_abi_check")


def test_c_program():
    assert os.path.exists(EXE), "the C check is built by __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "C ABI OK" in r.stdout
