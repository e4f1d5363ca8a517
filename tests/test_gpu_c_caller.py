"""The library driven from a plain C program (tests/abi_caller.c): no Python,
no PyTorch in the process, host arrays in, host arrays out.  Its serial
iterate after 25 epochs must match the oracle's to 1e-12."""
import os
import subprocess
import sys

import numpy as np
import pytest

import datagen
import oracle
from conftest import ROOT, rel_err

pytestmark = pytest.mark.gpu

PKG = os.path.join(ROOT, "paper_1606_04809_amd")


def test_plain_c_caller_serial_matches_oracle(tmp_path):
    lib = os.path.join(PKG, "libasaga.so")
    if not os.path.exists(lib):
        pytest.fail("libasaga.so is not built")
    exe = tmp_path / "abi_caller"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "abi_caller.c"), "-o", str(exe), "-L", PKG, "-lasaga",
                           "-Wl,-rpath," + PKG])
    print("running the C caller", flush=True, file=sys.stderr)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.array([float(t) for t in r.stdout.split()])
    # the same 6 x 4 problem as the caller's arrays
    rowptr = np.array([0, 2, 3, 5, 7, 8, 10], dtype=np.int64)
    colidx = np.array([0, 2, 1, 0, 3, 1, 2, 3, 0, 1], dtype=np.int32)
    val = np.array([0.6, -0.8, 1.0, 0.28, 0.96, -0.6, 0.8, 1.0, 0.8, 0.6])
    b = np.array([1.0, -1.0, 1.0, 1.0, -1.0, -1.0])
    p = datagen.Problem("c-caller", 6, 4, rowptr, colidx, val, b, datagen.LOGISTIC, 0.1)
    sv = oracle.SparseSaga(p, seed=3)
    sv.epochs(25)
    assert rel_err(got[1:], sv.state.x) <= 1e-12, (got[1:], sv.state.x)
    assert abs(got[0] - sv.objective()) <= 1e-12 * abs(sv.objective())
