"""The allocation-free batched evaluation (sevo_evaluate_batch_noalloc)
against sevo_evaluate_batch, through the C ABI: the same bits on two calls in
a row (the second smaller, over the first's table contents), in every
precision, and its limits reported as errors with nothing written."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
from paper_2505_17430_amd import sevo as S  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def items_of(groups, salt, dtype):
    out = []
    for (f, d, k, n) in groups:
        X = W.uniform_points(W.group_seed(f, d, k, salt), d, n)
        xd = torch.from_numpy(X).cuda().to(dtype)
        out.append((S.problem(f, d), k, xd, torch.full((n,), float("nan"), dtype=dtype, device="cuda")))
    return out


def raw_call(ctx, fn, items, precision):
    arr = S.Context.prepare_batch(items)
    return getattr(ctx._L, fn)(ctx._h, arr, len(arr), precision, None)


@pytest.mark.parametrize("precision", [S.FP32, S.SPLIT_BF16, S.FP64])
def test_noalloc_matches_batch_on_two_calls(precision):
    ctx = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
    try:
        dtype = torch.float64 if precision == S.FP64 else torch.float32
        first = [(0, 10, 0, 5100), (2, 30, 1, 777), (3, 50, 2, 1300), (5, 100, 3, 2049), (1, 100, 4, 33),
                 (4, 64, 0, 129), (2, 96, 1, 300)]
        if precision == S.FP64:
            first.append((0, 200, 0, 257))
        second = [(5, 100, 3, 100), (0, 10, 5, 40)]
        for groups, salt in ((first, 1), (second, 2)):
            a = items_of(groups, salt, dtype)
            b = [(p, k, x, torch.full_like(e, float("nan"))) for (p, k, x, e) in a]
            for (p, k, _, _) in a:                       # instances made resident first
                ctx.instance(p, k)
            assert raw_call(ctx, "sevo_evaluate_batch", a, precision) == S.OK
            rc = raw_call(ctx, "sevo_evaluate_batch_noalloc", b, precision)
            assert rc == S.OK, ctx.last_error()
            torch.cuda.synchronize()
            for (p, k, x, ea), (_, _, _, eb) in zip(a, b):
                assert torch.equal(ea, eb), (p.func, p.dim, k)
                assert not torch.isnan(eb).any()
            say(f"  precision {precision}: {len(groups)} items, same bits")
    finally:
        ctx.close()


def test_noalloc_limits_are_errors():
    ctx = S.Context(0, W.BASE_SEED, W.INSTANCE_SEED)
    try:
        # an instance not made yet: nothing is generated (that would allocate)
        it = items_of([(2, 30, 77, 64)], 3, torch.float32)
        assert raw_call(ctx, "sevo_evaluate_batch_noalloc", it, S.FP32) == S.ESTATE
        assert "not resident" in ctx.last_error()
        # D > 120 in single precision needs the GEMM workspace
        big = items_of([(0, 200, 0, 64)], 4, torch.float32)
        ctx.instance(big[0][0], 0)
        assert raw_call(ctx, "sevo_evaluate_batch_noalloc", big, S.FP32) == S.EUNSUPPORTED
        # tables beyond the static array: 20,000 items of 64 B
        ctx.instance(S.problem(0, 10), 0)
        x = torch.zeros((10, 1), device="cuda")
        e = torch.full((1,), -5.0, device="cuda")
        many = [(S.problem(0, 10), 0, x, e)] * 20000
        assert raw_call(ctx, "sevo_evaluate_batch_noalloc", many, S.FP32) == S.EINVAL
        assert "static table" in ctx.last_error()
        torch.cuda.synchronize()
        assert float(e[0]) == -5.0 and torch.isnan(it[0][3]).all() and torch.isnan(big[0][3]).all()
    finally:
        ctx.close()
