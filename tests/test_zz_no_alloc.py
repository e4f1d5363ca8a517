"""The allocation-free objective (asaga_objective_noalloc) against the
context's objective (asaga_objective) on the same problem and point.

Two calls in a row on one GPU, the second with a smaller problem, both
through the C ABI: the static scratch array keeps the first call's
contents, so a stale term or partial sum left from the first call would
show in the second.  Tolerance: the two use the same row-dot, loss and
pairwise-sum kernels; they differ only in the order of the x^2 sum (the
context holds x in its relabelled column order) and in where the final
combination is rounded, so they agree to a few units of FP64 rounding
(1e-13 relative).
"""
import dataclasses
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_1606_04809_amd")
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def device_problem(p, bf16=False):
    """asaga_problem over torch CUDA tensors (kept alive by the return)."""
    dev = torch.device("cuda:0")
    vals = p.val_bf16 if bf16 else p.val
    keep = (torch.from_numpy(np.ascontiguousarray(p.rowptr, np.int64)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p.colidx, np.int32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(vals)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p.b, np.float64)).to(dev))
    vdt = A.ASAGA_VAL_BF16 if bf16 else A.ASAGA_VAL_F64
    prob = A.asaga_problem(p.n, p.d, *[t.data_ptr() for t in keep], float(p.lam), vdt, int(p.loss),
                           A.ASAGA_MEM_DEVICE, 0)
    return prob, keep


def with_bf16(p):
    """The instance with its values rounded to bfloat16 (the rounded matrix
    is the instance both sides evaluate)."""
    bits = datagen.bf16_round(p.val)
    return dataclasses.replace(p, val=datagen.bf16_widen(bits), val_bf16=bits)


def noalloc_objective(p, x, bf16=False):
    prob, keep = device_problem(p, bf16)
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()
    fd = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    A.asaga_objective_noalloc(prob, xd.data_ptr(), fd.data_ptr(), stream)
    torch.cuda.synchronize()
    return float(fd.cpu()[0])


def context_objective(p, x, bf16=False):
    with A.from_problem(p, bf16=bf16) as g:
        return g.objective(0, x)


@pytest.mark.parametrize("bf16", [False, True])
def test_noalloc_objective_matches_context_objective_twice(bf16):
    big = datagen.config2(n=60000, d=9000, seed=3)
    small = datagen.config1(n=700, d=150, k=12, seed=4)
    if bf16:
        small, big = with_bf16(small), with_bf16(big)
    rng = np.random.default_rng(11)
    for p in (big, small):
        x = rng.standard_normal(p.d) * 0.3
        got = noalloc_objective(p, x, bf16)
        want = context_objective(p, x, bf16)
        say(f"noalloc objective n={p.n} d={p.d} bf16={bf16}: {got!r} vs {want!r}")
        assert np.isfinite(got)
        assert abs(got - want) <= 1e-13 * abs(want), (p.n, got, want)


def test_noalloc_objective_squared_loss_and_zero_point():
    p = datagen.config3(n=5000)
    for x in (np.zeros(p.d), np.random.default_rng(2).standard_normal(p.d)):
        got = noalloc_objective(p, x)
        want = context_objective(p, x)
        assert abs(got - want) <= 1e-13 * abs(want), (got, want)
    # at x = 0 the squared-loss objective is mean(b^2) / 2
    assert noalloc_objective(p, np.zeros(p.d)) == pytest.approx(0.5 * np.mean(p.b ** 2), rel=1e-13)


def test_noalloc_objective_rejects_what_it_cannot_hold():
    p = datagen.config1(n=300, d=80, k=10)
    prob, keep = device_problem(p)
    xd = torch.zeros(p.d, dtype=torch.float64, device="cuda")
    fd = torch.zeros(1, dtype=torch.float64, device="cuda")
    for field, value in (("n", A.ASAGA_NOALLOC_MAX_ROWS + 1), ("n", 0), ("mem", A.ASAGA_MEM_HOST),
                         ("lam", 0.0), ("loss", 7), ("reserved", 1)):
        bad = A.asaga_problem.from_buffer_copy(prob)
        setattr(bad, field, value)
        with pytest.raises(A.AsagaError) as ei:
            A.asaga_objective_noalloc(bad, xd.data_ptr(), fd.data_ptr())
        assert ei.value.code == A.ASAGA_E_ARG, (field, value)
        if field == "n" and value > 0:
            assert "scratch" in str(ei.value)
    # a rejected call enqueued nothing: the output is untouched
    torch.cuda.synchronize()
    assert float(fd.cpu()[0]) == 0.0
