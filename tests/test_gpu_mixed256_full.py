"""The 256^3 mixed-nuclei workload at its full size: 1e6 H/He/N/Fe candidates on
the E^-2 spectrum, 256^3 FP64 turbulent grid (50 kpc cells), full interaction
tables, a 1 Mpc observer at (50, 0, 0) Mpc and a 100 Mpc trajectory limit, all
propagated in one run with the FP64 method, in the launch the autotuner picks
with the benchmark's trial budget (the corner records of the FP64 grid when
they are faster).  The oracle follows the first 1e4
candidates (ids 0..9999: 2500 of each species) on its own; every record the
GPU wrote for them -- their secondaries and neutral records included -- must
match the oracle's: integer bookkeeping exactly, positions within 1e-9 of
max(L, |x|), energies within 1e-6 (bitwise in practice: both sides take the
same FP64 operations in the same order)."""
import os

import numpy as np
import pytest

import crp_inputs as I
from bench import TUNE_CYCLES_FP64
from parity_helpers import compare_neutral, compare_records, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

W = I.W_MIXED256
N_SUB = 10_000


@pytest.fixture(scope="module")
def P():
    from paper_1307_2643_amd import crp
    crp.load()
    return crp


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _select(rec, ids_below):
    keep = rec["id"] < ids_below
    return {k: v[keep] for k, v in rec.items()}


def test_full_run_subset_matches_oracle(P, O):
    import torch
    n = W.n_candidates
    grid = W.make_grid()
    tables = W.make_tables()
    inj = W.make_injection()
    say(f"{W.name}: {n} candidates on the GPU")
    prm = P.params_for(W, P.FP64, queue_capacity=2 * n, neutral_capacity=n)
    ctx = P.Context(prm)
    ctx.set_field_grid(torch.as_tensor(grid, device="cuda:0"), W.spacing_m)
    ctx.set_tables(tables)
    ctx.inject(inj)
    launch, _ = ctx.tune(max_cycles=TUNE_CYCLES_FP64, cache_path=None)
    say(f"tuned launch {launch}")
    assert ctx.propagate()
    cnt = ctx.counts()
    fin = ctx.read_finished()
    neu = ctx.read_neutral()
    ctx.close()
    say(f"gpu: {len(fin['id'])} finished, {len(neu['id'])} neutral, {cnt['steps']} steps")
    # whole-run invariants: every primary finished once, with its secondaries
    prim = fin["lineage"] == 0
    assert prim.sum() == n and len(np.unique(fin["id"][prim])) == n
    assert cnt["finished"] == len(fin["id"]) == n + cnt["charged_sec"]
    assert len(neu["id"]) == cnt["neutral_sec"] and cnt["queue_deferred"] == 0
    assert cnt["observed"] > 0 and cnt["charged_sec"] > 0
    say(f"oracle: first {N_SUB} candidates")
    fo, no, co, _ = O.propagate(O.config_for(W), O.GridRef(grid, W.spacing_m),
                                O.TablesRef(tables), inj.subset(slice(0, N_SUB)),
                                nthreads=len(os.sched_getaffinity(0)), neu_cap=1 << 20)
    fg = _select(fin, N_SUB)
    ng = _select(neu, N_SUB)
    assert len(fg["id"]) == co["finished"] and len(ng["id"]) == co["neutral_sec"]
    same = compare_records(fg, fo, f"{W.name} first {N_SUB}")
    compare_neutral(ng, no, f"{W.name} first {N_SUB} neutral", fo)
    say(f"bitwise identical: {same.sum()} of {len(same)}")
    assert same.mean() > 0.999
