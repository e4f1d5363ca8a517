"""The C ABI without a GPU: the library loads, exports every function that
include/asaga.h declares, and rejects malformed problems on the host before
touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

A = pytest.importorskip("paper_1606_04809_amd")

HEADER = os.path.join(ROOT, "include", "asaga.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asaga_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    lib = ctypes.CDLL(A.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(A.EXPORTED) == names


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets as the C compiler lays out asaga.h
    src = tmp_path / "layout.c"
    checks = []
    for cname, py in (("asaga_problem", A.asaga_problem), ("asaga_opts", A.asaga_opts),
                      ("asaga_batch", A.asaga_batch), ("asaga_info", A.asaga_info),
                      ("asaga_instance", A.asaga_instance)):
        checks.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = {"lam": "lambda"}.get(fname, fname)
            checks.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"asaga.h\"\nint main(void){"
                   + "".join(checks) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in (("asaga_problem", A.asaga_problem), ("asaga_opts", A.asaga_opts),
                      ("asaga_batch", A.asaga_batch), ("asaga_info", A.asaga_info),
                      ("asaga_instance", A.asaga_instance)):
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def good():
    return dict(n=3, d=4, rowptr=np.array([0, 2, 3, 5]), colidx=np.array([0, 2, 1, 0, 3], np.int32),
                val=np.array([1.0, -0.5, 2.0, 0.3, 0.7]), b=np.array([1.0, -1.0, 1.0]), lam=0.1)


def expect(code, **changes):
    kw = good()
    opts = {k: changes.pop(k) for k in list(changes) if k in ("mode", "precision", "lanes_per_sample", "racy",
                                                              "waves", "step", "loss", "hot_columns",
                                                              "hot_tier_columns",
                                                              "flush_every", "threads_per_block",
                                                              "plain_launch", "method", "hot_reload_from")}
    kw.update(changes)
    with pytest.raises(A.AsagaError) as ei:
        A.Solver(**kw, **opts)
    assert ei.value.code == code, str(ei.value)
    assert A.asaga_last_error(None)


def test_malformed_csr_is_rejected_on_host():
    E = A.ASAGA_E_CSR
    expect(E, rowptr=np.array([1, 2, 3, 5]))                      # rowptr[0] != 0
    expect(E, rowptr=np.array([0, 3, 2, 5]))                      # decreasing
    expect(E, rowptr=np.array([0, 2, 2, 5]))                      # empty row
    expect(E, colidx=np.array([0, 2, 1, 0, 4], np.int32))        # column out of range
    expect(E, colidx=np.array([0, 2, 1, 0, -1], np.int32))       # negative column
    expect(E, colidx=np.array([2, 0, 1, 0, 3], np.int32))        # not increasing
    expect(E, colidx=np.array([0, 0, 1, 0, 3], np.int32))        # duplicate
    expect(E, val=np.array([1.0, np.nan, 2.0, 0.3, 0.7]))        # non-finite value
    expect(E, val=np.array([1.0, np.inf, 2.0, 0.3, 0.7]))
    expect(E, b=np.array([1.0, 0.0, 1.0]))                       # logistic label not +-1
    expect(E, b=np.array([1.0, np.nan, 1.0]), loss=A.ASAGA_LOSS_SQUARED)


def test_bad_arguments_are_rejected():
    E = A.ASAGA_E_ARG
    expect(E, lam=0.0)
    expect(E, lam=-1.0)
    expect(E, lam=float("inf"))
    expect(E, mode=7)
    expect(E, precision=3)
    expect(E, precision=-1)
    expect(E, lanes_per_sample=12)
    expect(E, racy=1)                                            # racy needs async mode
    expect(E, waves=-1)
    expect(E, step=float("nan"))
    expect(E, loss=5)
    expect(E, hot_columns=5121)
    expect(E, hot_columns=5121, precision=A.ASAGA_PREC_MIXED)
    expect(E, hot_columns=10241, precision=A.ASAGA_PREC_F32)      # the FP32 layout holds up to 10240
    expect(E, hot_tier_columns=10241, precision=A.ASAGA_PREC_F32)
    expect(E, hot_columns=-2)
    expect(E, flush_every=-1)
    expect(E, threads_per_block=100)
    expect(E, threads_per_block=2048)
    expect(E, threads_per_block=1088)
    expect(E, plain_launch=2)
    expect(E, method=2)
    expect(E, method=A.ASAGA_METHOD_SVRG, racy=1, mode=A.ASAGA_MODE_ASYNC)   # racy is a SAGA control
    expect(E, hot_reload_from=-2)
    expect(E, hot_reload_from=5121)
    expect(E, n=0, rowptr=np.array([0]), colidx=np.array([], np.int32), val=np.array([]), b=np.array([]))


def test_null_context_calls_fail_cleanly():
    lib = ctypes.CDLL(A.LIB_PATH)
    lib.asaga_epochs.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    assert lib.asaga_epochs(None, 1) == A.ASAGA_E_ARG
    lib.asaga_set_active.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.asaga_set_active(None, None) == A.ASAGA_E_ARG
    lib.asaga_set_stop.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.asaga_set_stop(None, None) == A.ASAGA_E_ARG
    lib.asaga_stop_report.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.asaga_stop_report(None, None, None) == A.ASAGA_E_ARG
    lib.asaga_widen.argtypes = [ctypes.c_void_p]
    assert lib.asaga_widen(None) == A.ASAGA_E_ARG
    lib.asaga_free.argtypes = [ctypes.c_void_p]
    lib.asaga_free(None)


def test_overlap_estimator_small_exact_case():
    # intervals [0,10], [5,15], [12,20] ticks at 1 tick per microsecond, every update logged:
    # at 5 one update is in flight ([0,10]); at 12 one ([5,15]); at 0 none
    log = np.array([[0 + 1, 10 + 1], [5 + 1, 15 + 1], [12 + 1, 20 + 1]])  # shifted: start 0 marks "not written"
    r = A.asaga_overlap_estimate(log, every=1, clock_hz=1e6, updates_per_s=1e5)
    assert r.logged == 3 and r.every == 1
    assert r.tau_max == 1.0 and r.tau_mean == pytest.approx(2.0 / 3.0)
    assert r.latency_mean_us == pytest.approx((10 + 10 + 8) / 3.0)
    assert r.little == pytest.approx(1e5 * r.latency_mean_us * 1e-6)


def test_overlap_estimator_recovers_workers_in_flight():
    # W workers run back-to-back updates of random length; one update in
    # `every` (in start order) is logged.  At any instant every other worker
    # has one update in flight, so the estimate is W - 1 on average.
    rng = np.random.default_rng(3)
    W, per, every = 64, 400, 8
    starts, ends = [], []
    for w in range(W):
        t = rng.uniform(0, 50)
        for _ in range(per):
            d = rng.uniform(20, 80)
            starts.append(t)
            ends.append(t + d)
            t += d
    order = np.argsort(starts)
    st = (np.asarray(starts)[order] * 1000).astype(np.int64) + 1
    en = (np.asarray(ends)[order] * 1000).astype(np.int64) + 1
    keep = (np.arange(len(st)) % every == 0) & (st > 100_000) & (en < st.max() - 100_000)  # steady state
    log = np.stack([st[keep], en[keep]], axis=1)
    r = A.asaga_overlap_estimate(log, every=every, clock_hz=1e9, updates_per_s=0.0)
    assert abs(r.tau_mean - (W - 1)) < 0.1 * W, r.tau_mean
    assert r.tau_p50 <= r.tau_p99 <= r.tau_max
    assert r.latency_mean_us == pytest.approx(50.0, rel=0.05)   # U(20, 80) units of 1000 ticks at 1 GHz


def test_overlap_estimator_rejects_bad_input():
    with pytest.raises(A.AsagaError):
        A.asaga_overlap_estimate(np.array([[10, 5]]), every=1, clock_hz=1.0)
    with pytest.raises(A.AsagaError):
        A.asaga_overlap_estimate(np.array([[1, 5]]), every=0, clock_hz=1.0)
    with pytest.raises(A.AsagaError):
        A.asaga_overlap_estimate(np.array([[1, 5]]), every=1, clock_hz=0.0)
    r = A.asaga_overlap_estimate(np.zeros((4, 2), dtype=np.int64), every=1, clock_hz=1.0)
    assert r.logged == 0


def test_opts_reserved_must_be_zero():
    # checked with the other options, before any device call
    kw = good()
    rowptr = np.ascontiguousarray(kw["rowptr"], dtype=np.int64)
    prob = A.asaga_problem(kw["n"], kw["d"], rowptr.ctypes.data, kw["colidx"].ctypes.data, kw["val"].ctypes.data,
                           kw["b"].ctypes.data, kw["lam"], A.ASAGA_VAL_F64, A.ASAGA_LOSS_LOGISTIC, A.ASAGA_MEM_HOST, 0)
    opts = A.asaga_opts()
    opts.reserved = 1
    with pytest.raises(A.AsagaError) as ei:
        A.asaga_init(prob, opts)
    assert ei.value.code == A.ASAGA_E_ARG


def test_batched_svrg_is_rejected():
    kw = good()
    with pytest.raises(A.AsagaError) as ei:
        A.Solver(**kw, mode=A.ASAGA_MODE_ASYNC, method=A.ASAGA_METHOD_SVRG,
                 batch=(np.zeros(3, np.int8), np.array([-1], np.int32), np.array([0.1])))
    assert ei.value.code == A.ASAGA_E_ARG


def test_header_compiles_as_plain_c(tmp_path):
    # the public header and a caller of it are plain C99 (no C++ or HIP types),
    # and such a caller links against the library with the system C toolchain
    pkg = os.path.join(ROOT, "paper_1606_04809_amd")
    obj, exe = tmp_path / "caller.o", tmp_path / "caller"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                           "-c", os.path.join(ROOT, "tests", "abi_caller.c"), "-o", str(obj)])
    subprocess.check_call(["gcc", str(obj), "-o", str(exe), "-L", pkg, "-lasaga", "-Wl,-rpath," + pkg])
    assert exe.exists()


def test_request_ceiling_rejects_bad_arguments():
    # checked before any device call
    for cols in (0, -5, 1 << 27):
        with pytest.raises(A.AsagaError) as e:
            A.asaga_request_ceiling(cols)
        assert e.value.code == A.ASAGA_E_ARG
    lib = A._lib
    assert lib.asaga_request_ceiling(100, None, None) == A.ASAGA_E_ARG
