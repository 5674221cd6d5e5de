"""The allocation-free field evaluation (crp_eval_field_noalloc) against
crp_eval_field: the same kernels on the same inputs, so bitwise equal, over
two calls in a row (the second smaller, so stale staging contents would
show), for the grid forms and layouts and the analytic field; the size limit
and the empty call."""
import ctypes as C

import numpy as np
import pytest

import crp_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1307_2643_amd import crp
    crp.load()
    return crp


def _positions(n, box, seed):
    rng = np.random.default_rng(seed)
    return (rng.random((n, 3)) * 5.0 - 2.0) * box


def _check_two_calls(ctx, mode, box, n1, n2, seed):
    for n, s in ((n1, seed), (n2, seed + 1)):
        pos = _positions(n, box, s)
        ref = ctx.eval_field(pos, mode)
        got = ctx.eval_field_noalloc(pos, mode)
        print(f"noalloc mode={mode} n={n}", flush=True)
        assert np.array_equal(got, ref), (mode, n)


def test_noalloc_matches_eval_field(P):
    w = I.W_SMALL
    grid = w.make_grid()
    box = 32 * w.spacing_m
    big = P.EVAL_NOALLOC_MAX
    for gdtype in (np.float64, np.float32):
        prm = P.params_for(w, P.FP64, queue_capacity=1 << 12, neutral_capacity=1 << 12)
        ctx = P.Context(prm)
        ctx.set_field_grid(grid.astype(gdtype), w.spacing_m)
        ctx.set_tables(w.make_tables())
        for mode in (P.FP64, P.MIX):
            _check_two_calls(ctx, mode, box, big, 1000, 10 + mode)
        if gdtype == np.float32:
            ctx.set_launch(layout=P.LAYOUT_CORNER)
            ctx.inject(w.make_injection(64))
            ctx.propagate()                    # builds the corner records
            _check_two_calls(ctx, P.MIX, box, 70_001, 65, 20)
        # the limit and the empty call
        with pytest.raises(P.CrpError):
            ctx.eval_field_noalloc(np.zeros((big + 1, 3)), P.FP64)
        assert ctx.eval_field_noalloc(np.zeros((0, 3)), P.FP64).shape == (0, 3)
        ctx.close()


def test_noalloc_analytic_field_and_raw_abi(P):
    w = I.W_GALBACK
    prm = P.params_for(w, P.FP64, queue_capacity=1 << 12, neutral_capacity=1 << 12)
    ctx = P.Context(prm)
    ctx.set_field_analytic(I.GALACTIC_FIELD)
    _check_two_calls(ctx, P.EVAL_ANALYTIC, 10 * I.KPC_M, 50_000, 7, 30)
    # straight through the C-ABI with caller-owned host buffers
    pos = _positions(333, 10 * I.KPC_M, 31)
    out = np.full_like(pos, np.nan)
    lib = P.load()
    st = lib.crp_eval_field_noalloc(ctx.h, pos.shape[0], pos.ctypes.data_as(C.c_void_p),
                                    out.ctypes.data_as(C.c_void_p), P.EVAL_ANALYTIC)
    assert st == 0
    assert np.array_equal(out, ctx.eval_field(pos, P.EVAL_ANALYTIC))
    # a bad mode is refused before anything runs
    assert lib.crp_eval_field_noalloc(ctx.h, 1, pos.ctypes.data_as(C.c_void_p),
                                      out.ctypes.data_as(C.c_void_p), 99) == -1
    ctx.close()
