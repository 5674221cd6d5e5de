"""GPU parity of the output modules and observables (through the C-ABI):
per-step trajectory points from the propagation kernel, and the observable
reduction kernel over finished records, against the oracle on the same seeded
inputs.

Bar: trajectory points bitwise (both sides record the same FP64 state after
the same cycle); observable counts, sky counts and `outside` exact; the
fixed-point deflection sums within one unit (2^-32 rad) per record, the only
freedom being the last bit of the two atan2 implementations; the weight sums
within (count + 8) * 2^-50 relative, the bound of a sum of positive terms in
any order plus the ulps of pow.
"""
import numpy as np
import pytest

import crp_inputs as I
from oracle import observables as OB
from parity_helpers import compare_counts, compare_records, make_ctx, say

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def small_grid():
    return I.W_SMALL.make_grid()


@pytest.fixture(scope="module")
def mixed_grid():
    return I.W_MIXED256.make_grid()


def compare_traj(tg, to, what):
    from paper_1307_2643_amd import crp
    tg = crp.sort_traj(tg)
    to = crp.sort_traj(to)
    assert len(tg["id"]) == len(to["id"]), f"{what}: {len(tg['id'])} vs {len(to['id'])} points"
    for k in to:
        bad = np.nonzero(np.any((tg[k] != to[k]).reshape(len(to["id"]), -1), axis=1))[0]
        assert bad.size == 0, f"{what}: field {k} differs at {bad[:5]}"
    say(f"{what}: {len(tg['id'])} trajectory points bitwise identical")


@pytest.mark.parametrize("precision,every,ids,layout",
                         [(0, 1, 1 << 30, 0), (1, 1, 1 << 30, 0), (0, 5, 700, 0), (1, 3, 50, 0),
                          (0, 1, 1 << 30, 1), (1, 2, 1 << 30, 1)],
                         ids=["fp64-every", "mix-every", "fp64-k5", "mix-k3", "fp64-every-corner",
                              "mix-k2-corner"])
def test_trajectory_points_parity(P, O, small_grid, precision, every, ids, layout):
    """Every k-th step of the selected ids (the 32^3 FP64 grid, read from the
    linear grid or from its 192-byte corner records) against the oracle."""
    w = I.W_SMALL
    inj = w.make_injection()
    cap = 1 << 21
    ctx = make_ctx(P, w, small_grid, w.make_tables(), precision, traj_every=every,
                   traj_ids=ids, traj_capacity=cap)
    ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=layout)
    say(f"trajectory parity precision={precision} every={every} ids<{ids} layout={layout}")
    ctx.inject(inj)
    assert ctx.propagate()
    cg = ctx.counts()
    tg = ctx.read_trajectory()
    fg = ctx.read_finished()
    ctx.close()
    cfg = O.config_for(w, precision=precision, traj_every=every, traj_ids=ids)
    fo, _, co, to = O.propagate_traj(cfg, O.GridRef(small_grid, w.spacing_m),
                                     O.TablesRef(w.make_tables()), inj, cap)
    compare_counts(cg, co, "trajectory run")
    assert compare_records(fg, fo, "trajectory run").all()
    assert cg["traj_points"] == len(to["id"]) and cg["traj_dropped"] == 0
    assert cg["traj_unread"] == len(to["id"])
    compare_traj(tg, to, f"p{precision} every {every}")


@pytest.mark.parametrize("layout", [0, 1], ids=["linear", "corner"])
def test_trajectory_with_secondaries_and_budget(P, O, mixed_grid, layout):
    """Mixed nuclei with secondaries and observer detections, run in slices of
    a cycle budget (parked candidates keep recording where they stopped)."""
    w = I.W_MIXED256
    inj = w.make_injection(800)
    cap = 1 << 22
    ctx = make_ctx(P, w, mixed_grid, w.make_tables(), P.FP64, traj_every=4,
                   traj_ids=1 << 30, traj_capacity=cap)
    ctx.set_launch(block=256 if layout else 128, blocks_per_cu=0, refill=4, layout=layout)
    say(f"trajectory with secondaries, budget 150 cycles per call, layout {layout}")
    ctx.inject(inj)
    calls = 1
    while not ctx.propagate(150):
        calls += 1
    assert calls > 1
    tg = ctx.read_trajectory()
    cg = ctx.counts()
    ctx.close()
    cfg = O.config_for(w, traj_every=4, traj_ids=1 << 30)
    fo, _, co, to = O.propagate_traj(cfg, O.GridRef(mixed_grid, w.spacing_m),
                                     O.TablesRef(w.make_tables()), inj, cap)
    assert np.any(to["lineage"] > 0)
    assert cg["traj_points"] == len(to["id"])
    compare_traj(tg, to, "secondaries + budget")


def test_trajectory_capacity_overflow(P, O, small_grid):
    w = I.W_SMALL
    inj = w.make_injection(200)
    cfg = O.config_for(w, traj_every=1, traj_ids=1 << 30)
    _, _, _, to = O.propagate_traj(cfg, O.GridRef(small_grid, w.spacing_m),
                                   O.TablesRef(w.make_tables()), inj, 1 << 22)
    total = len(to["id"])
    cap = total // 4
    ctx = make_ctx(P, w, small_grid, w.make_tables(), P.FP64, traj_every=1,
                   traj_ids=1 << 30, traj_capacity=cap)
    say(f"trajectory overflow cap={cap} of {total}")
    ctx.inject(inj)
    assert ctx.propagate()
    cg = ctx.counts()
    tg = ctx.read_trajectory()
    ctx.close()
    assert cg["traj_points"] == cap and cg["traj_dropped"] == total - cap
    assert len(tg["id"]) == cap
    # every kept point is one of the oracle's, with the same values
    ko = {(int(a), int(b), int(c)): i for i, (a, b, c) in
          enumerate(zip(to["id"], to["lineage"], to["n"]))}
    idx = np.array([ko[(int(a), int(b), int(c))] for a, b, c in
                    zip(tg["id"], tg["lineage"], tg["n"])])
    assert np.unique(idx).size == cap
    for k in to:
        assert np.array_equal(tg[k], to[k][idx]), k


def test_trajectory_read_in_pieces_and_snapshot(P, O, small_grid):
    w = I.W_SMALL
    inj = w.make_injection(100)
    ctx = make_ctx(P, w, small_grid, w.make_tables(), P.MIX, traj_every=2,
                   traj_ids=1 << 30, traj_capacity=1 << 20)
    ctx.inject(inj)
    say("trajectory snapshot / restore / piecewise read")
    assert ctx.propagate()
    blob = ctx.snapshot()
    n = ctx.counts()["traj_unread"]
    parts = [ctx.read_trajectory(n // 3), ctx.read_trajectory(n // 3), ctx.read_trajectory()]
    assert ctx.counts()["traj_unread"] == 0
    whole = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    ctx.restore(blob)
    again = ctx.read_trajectory()
    ctx.close()
    cfg = O.config_for(w, precision=O.MIX, traj_every=2, traj_ids=1 << 30)
    _, _, _, to = O.propagate_traj(cfg, O.GridRef(small_grid, w.spacing_m),
                                   O.TablesRef(w.make_tables()), inj, 1 << 20)
    compare_traj(whole, to, "piecewise read")
    compare_traj(again, to, "restored")


# ---------------------------------------------------------------------------
# Observables.
# ---------------------------------------------------------------------------
def compare_obs(og, oo, what):
    assert og["outside"] == oo["outside"], what
    assert np.array_equal(og["counts"], oo["counts"]), what
    assert np.array_equal(og["sky"], oo["sky"]), what
    c = oo["counts"].astype(np.int64)
    dd = np.abs(og["defl"].astype(np.int64) - oo["defl"].astype(np.int64))
    assert np.all(dd <= c), f"{what}: deflection sums differ by {dd.max()} units"
    tol = (c + 8) * 2.0 ** -50 * np.abs(oo["wsum"])
    assert np.all(np.abs(og["wsum"] - oo["wsum"]) <= tol), what
    say(f"{what}: {int(c.sum())} records in {np.count_nonzero(c)} bins, "
        f"deflection sums equal in {np.mean(dd == 0) * 100:.1f}% of bins")


def spec_mixed(sky_n=16, gamma=-1.5, sign=-1.0):
    return OB.spec(10.0 ** np.linspace(17.0, 21.0, 17), a_edges=(1, 2, 5, 15, 57),
                   status_mask=(1 << 1) | (1 << 2) | (1 << 3), sky_n=sky_n, sky_sign=sign,
                   e_ref=1e18, gamma=gamma)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mix"])
def test_observables_parity(P, O, mixed_grid, precision):
    w = I.W_MIXED256
    inj = w.make_injection(4000)
    ctx = make_ctx(P, w, mixed_grid, w.make_tables(), precision)
    sp = spec_mixed()
    ctx.set_observables(sp)
    say(f"observables precision={precision}")
    ctx.inject(inj)
    assert ctx.propagate()
    ms = ctx.observe()
    og = ctx.read_observables()
    fg = ctx.read_finished()
    ctx.close()
    fo, _, _, _ = O.propagate(O.config_for(w, precision=precision),
                              O.GridRef(mixed_grid, w.spacing_m), O.TablesRef(w.make_tables()),
                              inj)
    assert compare_records(fg, fo, "observables run").all()
    oo = OB.observe(sp, fo)
    assert oo["counts"].sum() > 1000 and oo["outside"] > 0
    compare_obs(og, oo, f"observables p{precision} ({ms:.3f} ms)")


def test_observables_accumulate_and_edge_cases(P, O, mixed_grid):
    """Two batches observed one after the other equal one pass over both;
    a spec with a single bin, no sky map and gamma 0 (weights exactly 1)."""
    w = I.W_MIXED256
    inj = w.make_injection(3000)
    a, b = inj.subset(slice(0, 1700)), inj.subset(slice(1700, 3000))
    for sp in (spec_mixed(sky_n=7, sign=1.0), OB.spec([1e16, 1e22], a_edges=(1, 60),
                                                       status_mask=0b11110, gamma=0.0)):
        ctx = make_ctx(P, w, mixed_grid, w.make_tables(), P.FP64)
        ctx.set_observables(sp)
        assert ctx.observe() == 0.0                    # nothing finished yet
        say(f"observables in two batches, sky_n={sp['sky_n']}")
        for part in (a, b):
            ctx.inject(part)
            assert ctx.propagate()
            ctx.observe()
            ctx.discard_finished()
        og = ctx.read_observables()
        ctx.close()
        fo, _, _, _ = O.propagate(O.config_for(w), O.GridRef(mixed_grid, w.spacing_m),
                                  O.TablesRef(w.make_tables()), inj)
        oo = OB.observe(sp, fo)
        compare_obs(og, oo, "two batches")
        if sp["gamma"] == 0.0:
            assert np.array_equal(og["wsum"], og["counts"].astype(np.float64))


def test_observables_reject_bad_specs(P, small_grid):
    w = I.W_SMALL
    ctx = make_ctx(P, w, small_grid, w.make_tables(), P.FP64)
    with pytest.raises(P.CrpError):
        ctx.observe()                                  # no spec yet
    for bad in (OB.spec([1e18, 1e18]), OB.spec([1e18, 1e19], a_edges=(5, 5)),
                OB.spec(np.logspace(16, 22, 300)), OB.spec([1e18, 1e19], sky_n=600),
                OB.spec([1e18, 1e19], sky_sign=0.5), OB.spec([1e18, 1e19], e_ref=0.0)):
        with pytest.raises(P.CrpError):
            ctx.set_observables(bad)
    ctx.close()
