"""GPU (HIP, through the C-ABI) versus the CPU oracle on the same seeded inputs.

Bar: integer bookkeeping exact (counts, channels, event numbers, statuses,
species); FP64 positions within 1e-9 * max(L, |x|) and energies within 1e-6
relative; the precision form is compared with the oracle's precision form
under the same bar, and its error against the FP64 oracle is reported.
"""
import numpy as np
import pytest

import crp_inputs as I
from parity_helpers import (CNT_KEYS, compare_counts, compare_neutral, compare_records, make_ctx,
                            run_gpu, say)

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


# ---------------------------------------------------------------------------
# Field gather: the stepper's interpolation is bitwise the oracle's.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gdtype,mode", [(np.float64, 0), (np.float32, 0), (np.float32, 1),
                                         (np.float64, 1)])
def test_eval_field_bitwise(P, O, small_grid, gdtype, mode):
    w = I.W_SMALL
    g = small_grid.astype(gdtype)
    ctx = make_ctx(P, w, g, w.make_tables(), P.FP64)
    rng = np.random.default_rng(1)
    box = 32 * w.spacing_m
    pos = (rng.random((100_000, 3)) * 7.0 - 3.0) * box       # several periods, both signs
    pos[:100] = np.round(pos[:100] / w.spacing_m) * w.spacing_m  # exact vertices
    say(f"eval_field dtype={np.dtype(gdtype).name} mode={mode}")
    got = ctx.eval_field(pos, mode)
    ref = O.eval_field(O.GridRef(g, w.spacing_m), pos, O.MIX if mode == 1 else O.FP64)
    assert np.array_equal(got, ref)
    if gdtype == np.float32:
        ctx.set_launch(layout=P.LAYOUT_CORNER)
        ctx.propagate()  # nothing pending: no-op
        say("eval_field corner layout")
        ctx.inject(w.make_injection(64))
        ctx.propagate()            # builds the corner records on first use
        got2 = ctx.eval_field(pos, mode)
        assert np.array_equal(got2, ref)
    ctx.close()


def test_eval_field_non_power_of_two_grid(P, O):
    rng = np.random.default_rng(2)
    g = rng.standard_normal((6, 5, 7, 3)) * 1e-13
    w = I.W_SMALL
    ctx = make_ctx(P, w, g, w.make_tables(), P.FP64)
    pos = (rng.random((20000, 3)) * 40 - 20) * w.spacing_m
    say("eval_field 6x5x7")
    got = ctx.eval_field(pos, 0)
    ref = O.eval_field(O.GridRef(g, w.spacing_m), pos, O.FP64)
    assert np.array_equal(got, ref)
    ctx.close()


def _far_positions(spacing):
    """Offsets on both sides of 2^31, 2^62 and 2^63 cells and far beyond, with
    fractional offsets near 2^31 and a few non-finite positions."""
    vals = [2.0 ** 31 - 1, 2.0 ** 31, 2.0 ** 31 + 0.5, 2.0 ** 52 + 2, 2.0 ** 62 - 2 ** 10,
            2.0 ** 62, 2.0 ** 63, 2.0 ** 64 + 2 ** 12, 3.0 * 2.0 ** 70, 1e300, 12345.25,
            2.0 ** 31 - 2 + 0.75]
    vals = vals + [-v for v in vals]
    p = np.array([[vals[k], vals[(k + 3) % len(vals)], vals[(k + 7) % len(vals)]]
                  for k in range(len(vals))]) * spacing
    bad = np.array([[np.nan, 0.0, 0.0], [np.inf, 1.0, 0.0], [0.0, -np.inf, 0.5]]) * spacing
    return p, bad


@pytest.mark.parametrize("shape", [(32, 32, 32), (6, 5, 7)], ids=["pow2", "odd"])
def test_eval_field_far_positions_exact_wrap(P, O, shape):
    """The periodic cell is floor(x / d) mod N for every finite offset, on the
    GPU as in the oracle: bitwise for FP64/FP32 grids, both interpolation
    forms, linear and corner layouts.  Non-finite positions give a non-finite
    field on both sides."""
    w = I.W_SMALL
    rng = np.random.default_rng(3)
    g64 = rng.standard_normal(shape + (3,)) * 1e-13
    pos, bad = _far_positions(1.0)              # spacing 1 m: positions are offsets in cells
    for gdtype in (np.float64, np.float32):
        g = g64.astype(gdtype)
        prm = P.params_for(w, P.FP64, queue_capacity=1 << 12, neutral_capacity=1 << 12)
        ctx = P.Context(prm)
        ctx.set_field_grid(g, 1.0)
        ctx.set_tables(w.make_tables())
        for mode in (0, 1):
            say(f"far positions shape={shape} dtype={np.dtype(gdtype).name} mode={mode}")
            ref = O.eval_field(O.GridRef(g, 1.0), pos, O.MIX if mode == 1 else O.FP64)
            assert np.array_equal(ctx.eval_field(pos, mode), ref)
            assert np.all(np.isnan(ctx.eval_field(bad, mode)).any(axis=1))
        if gdtype == np.float32:
            ctx.set_launch(layout=P.LAYOUT_CORNER)
            inj = w.make_injection(64)
            inj = I.Injection(inj.id, inj.A, inj.Z, inj.E, inj.pos * 0.0, inj.dir,
                              np.full(64, 10.0))
            ctx.inject(inj)
            ctx.propagate()                     # builds the corner records on first use
            for mode in (0, 1):
                say(f"far positions corner layout mode={mode}")
                ref = O.eval_field(O.GridRef(g, 1.0), pos, O.MIX if mode == 1 else O.FP64)
                assert np.array_equal(ctx.eval_field(pos, mode), ref)
        ctx.close()


@pytest.mark.parametrize("precision,gdtype", [(0, np.float64), (1, np.float64), (0, np.float32),
                                             (1, np.float32)])
def test_corner_records_odd_grid_match_oracle(P, O, precision, gdtype):
    """Corner records of a 6 x 5 x 7 grid (the records of the last cell
    planes take their far corners from vertex plane 0): 300 protons cross
    many periods of it; the records of the run from the corner records equal
    those of the run from the linear grid bit for bit and match the oracle's."""
    w = I.W_SMALL
    rng = np.random.default_rng(11)
    g = (rng.standard_normal((6, 5, 7, 3)) * 1e-13).astype(gdtype)
    tables = w.make_tables()
    inj = w.make_injection(300)
    runs = {}
    for layout, block in ((0, 128), (1, 256 if gdtype == np.float64 else 128)):
        say(f"odd grid corner records precision={precision} dtype={np.dtype(gdtype).name} "
            f"layout={layout}")
        ctx = make_ctx(P, w, g, tables, precision)
        ctx.set_launch(block=block, blocks_per_cu=0, refill=4, layout=layout)
        done, fg, ng, cg = run_gpu(ctx, inj)
        assert done
        runs[layout] = (fg, cg)
        ctx.close()
    _assert_identical(runs[0][0], runs[1][0])
    for k in CNT_KEYS:
        assert runs[0][1][k] == runs[1][1][k], k
    fo, no, co, _ = O.propagate(O.config_for(w, precision=precision), O.GridRef(g, w.spacing_m),
                                O.TablesRef(tables), inj)
    compare_counts(runs[1][1], co, "odd grid")
    same = compare_records(runs[1][0], fo, f"odd grid p{precision}")
    assert same.mean() > 0.99


# ---------------------------------------------------------------------------
# Whole path: small workload (1000 protons, 32^3 FP64 grid, loss table).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", [0, 1], ids=["linear", "corner"])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_workload_parity(P, O, small_grid, precision, layout):
    """FP64 method on the FP64 grid, precision form on the FP32 grid; each
    from the linear grid and from the corner records (192-byte FP64 records,
    128-byte FP32 records), which hold the same values."""
    w = I.W_SMALL
    grid = small_grid if precision == 0 else small_grid.astype(np.float32)
    tables = w.make_tables()
    inj = w.make_injection()
    say(f"small workload precision={precision} layout={layout}")
    ctx = make_ctx(P, w, grid, tables, precision)
    ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=layout)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done
    fo, no, co, _ = O.propagate(O.config_for(w, precision=precision),
                                O.GridRef(grid, w.spacing_m), O.TablesRef(tables), inj)
    compare_counts(cg, co, "small")
    same = compare_records(fg, fo, f"small p{precision}")
    assert same.mean() > 0.99
    ctx.close()


# ---------------------------------------------------------------------------
# Mixed nuclei with interactions, secondaries and the observer (256^3 grid).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,gdtype,launch", [
    (0, np.float64, dict(block=128, blocks_per_cu=0, refill=4, layout=0)),
    (0, np.float64, dict(block=128, blocks_per_cu=0, refill=4, layout=1)),
    (0, np.float64, dict(block=256, blocks_per_cu=1, refill=16, layout=1)),
    (1, np.float32, dict(block=128, blocks_per_cu=0, refill=4, layout=0)),
    (1, np.float64, dict(block=256, blocks_per_cu=0, refill=4, layout=1))],
    ids=["fp64-linear", "fp64-corner", "fp64-corner-b256", "mix-f32grid", "mix-f64grid-corner"])
def test_mixed_workload_subset_parity(P, O, mixed_grid, precision, gdtype, launch):
    """3000 candidates of the mixed workload; the FP64 grid's corner records
    (192 bytes per cell) in both precision forms and both block sizes."""
    w = I.W_MIXED256
    grid = mixed_grid.astype(gdtype)
    tables = w.make_tables()
    inj = w.make_injection(3000)
    say(f"mixed 256^3 subset precision={precision} grid={np.dtype(gdtype).name} {launch}")
    ctx = make_ctx(P, w, grid, tables, precision)
    ctx.set_launch(**launch)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done
    fo, no, co, _ = O.propagate(O.config_for(w, precision=precision),
                                O.GridRef(grid, w.spacing_m), O.TablesRef(tables), inj,
                                nthreads=0)
    compare_counts(cg, co, "mixed")
    assert co["charged_sec"] > 0 and co["neutral_sec"] > 0
    same = compare_records(fg, fo, f"mixed p{precision}")
    assert same.mean() > 0.99
    compare_neutral(ng, no, "mixed neutral", fo)
    ctx.close()


def test_observer_detections_match(P, O, mixed_grid):
    """Protons and nuclei aimed near the observer sphere: detection statuses exact."""
    w = I.W_MIXED256
    tables = w.make_tables()
    n = 2000
    rng = np.random.default_rng(5)
    inj = w.make_injection(n)
    tgt = np.array(w.observer) + rng.standard_normal((n, 3)) * 2 * I.MPC_M
    d = tgt / np.linalg.norm(tgt, axis=1)[:, None]
    inj.dir = d / np.linalg.norm(d, axis=1)[:, None]
    inj.E = np.full(n, 3e20)
    ctx = make_ctx(P, w, mixed_grid, tables, 0)
    say("observer detections")
    done, fg, ng, cg = run_gpu(ctx, inj)
    fo, no, co, _ = O.propagate(O.config_for(w), O.GridRef(mixed_grid, w.spacing_m),
                                O.TablesRef(tables), inj)
    assert co["observed"] > 100
    compare_counts(cg, co, "observer")
    compare_records(fg, fo, "observer")
    ctx.close()


# ---------------------------------------------------------------------------
# Invariance: launch shape, batch split, cycle budget, checkpoint/restore.
# ---------------------------------------------------------------------------
def _gpu_run(P, w, grid, tables, inj, precision=0, launch=None, batches=1, max_cycles=0,
             qcap=1 << 16):
    ctx = make_ctx(P, w, grid, tables, precision, qcap=qcap)
    if launch:
        ctx.set_launch(**launch)
    n = len(inj)
    cuts = np.linspace(0, n, batches + 1).astype(int)
    fins, neus = [], []
    for b in range(batches):
        ctx.inject(inj.subset(slice(cuts[b], cuts[b + 1])))
        while not ctx.propagate(max_cycles):
            pass
        fins.append(ctx.read_finished())
        neus.append(ctx.read_neutral())
    cnt = ctx.counts()
    ctx.close()
    fin = {k: np.concatenate([f[k] for f in fins]) for k in fins[0]}
    neu = {k: np.concatenate([f[k] for f in neus]) for k in neus[0]}
    return fin, neu, cnt


def _assert_identical(a, b):
    from paper_1307_2643_amd import crp
    a = crp.sort_finished(a)
    b = crp.sort_finished(b)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("launch", [dict(block=128, blocks_per_cu=1, refill=1),
                                    dict(block=256, blocks_per_cu=2, refill=64),
                                    dict(block=128, blocks_per_cu=8, refill=3, layout=1),
                                    dict(block=256, blocks_per_cu=0, refill=32, layout=1)])
def test_launch_shape_invariance(P, mixed_grid, launch):
    w = I.W_MIXED256
    grid = mixed_grid.astype(np.float32)
    tables = w.make_tables()
    inj = w.make_injection(3000)
    say(f"invariance launch={launch}")
    ref, rn, rc = _gpu_run(P, w, grid, tables, inj, precision=1)
    got, gn, gc = _gpu_run(P, w, grid, tables, inj, precision=1, launch=launch)
    _assert_identical(ref, got)
    for k in CNT_KEYS:
        assert rc[k] == gc[k]


def test_injection_order_longest_first(P, mixed_grid):
    """crp_inject queues a batch in decreasing lmax * Z / E (ties in the
    caller's order), from host arrays and from device arrays alike; the run's
    records and counters equal those of the caller's order bit for bit."""
    import torch
    w = I.W_MIXED256
    grid = mixed_grid.astype(np.float32)
    tables = w.make_tables()
    inj = I.inject_distances(3000, 77, dmax_m=40 * I.MPC_M)
    key = inj.lmax * inj.Z / inj.E
    order = np.argsort(-key, kind="stable")
    runs = {}
    for name, kw, on_dev in (("sorted", {}, False), ("sorted-device", {}, True),
                             ("as-given", dict(inject_order=P.ORDER_AS_GIVEN), False)):
        say(f"injection order: {name}")
        ctx = make_ctx(P, w, grid, tables, 1, **kw)
        if on_dev:
            d = [torch.as_tensor(a, device="cuda:0") for a in
                 (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
            ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=d[4], dir=d[5], lmax=d[6],
                       on_device=True)
        else:
            ctx.inject(inj)
        queued = ctx.peek_pending()["id"]
        expect = inj.id if name == "as-given" else inj.id[order]
        assert np.array_equal(queued, expect), name
        assert ctx.propagate()
        runs[name] = (ctx.read_finished(), ctx.counts())
        ctx.close()
    for name in ("sorted-device", "as-given"):
        _assert_identical(runs["sorted"][0], runs[name][0])
        for k in CNT_KEYS:
            assert runs["sorted"][1][k] == runs[name][1][k], (name, k)
    # ties keep the caller's order (a stable sort): five energies, one lmax
    tie = I.Injection(inj.id, inj.A, inj.Z, 1e19 * (1 + inj.id % 5).astype(np.float64), inj.pos,
                      inj.dir, np.full(len(inj.id), 30 * I.MPC_M))
    ctx = make_ctx(P, w, grid, tables, 1)
    ctx.inject(tie)
    key = tie.lmax * tie.Z / tie.E
    assert np.array_equal(ctx.peek_pending()["id"], tie.id[np.argsort(-key, kind="stable")])
    ctx.close()


def test_batch_split_and_budget_invariance(P, mixed_grid):
    w = I.W_MIXED256
    tables = w.make_tables()
    inj = w.make_injection(3000)
    say("batch split + budget")
    ref, _, rc = _gpu_run(P, w, mixed_grid, tables, inj)
    got, _, gc = _gpu_run(P, w, mixed_grid, tables, inj, batches=3, max_cycles=37)
    _assert_identical(ref, got)
    for k in CNT_KEYS:
        assert rc[k] == gc[k]


def test_budget_state_matches_oracle_cycle_cap(P, O, mixed_grid):
    w = I.W_MIXED256
    tables = w.make_tables()
    inj = w.make_injection(1500)
    say("cycle cap vs oracle")
    ctx = make_ctx(P, w, mixed_grid, tables, 0)
    ctx.inject(inj)
    done = ctx.propagate(25)
    assert not done
    pend = ctx.peek_pending()
    fin = ctx.read_finished()
    fo, _, co, _ = O.propagate(O.config_for(w, max_cycles=25), O.GridRef(mixed_grid, w.spacing_m),
                               O.TablesRef(tables), inj)
    allg = {k: np.concatenate([fin[k], pend[k]]) for k in fin}
    compare_records(allg, fo, "cycle cap 25")
    ctx.close()


def test_snapshot_restore_resume(P, mixed_grid):
    w = I.W_MIXED256
    tables = w.make_tables()
    inj = w.make_injection(2000)
    say("snapshot/restore")
    ref, _, rc = _gpu_run(P, w, mixed_grid, tables, inj)
    ctx = make_ctx(P, w, mixed_grid, tables, 0)
    ctx.inject(inj)
    assert not ctx.propagate(40)
    blob = ctx.snapshot()
    ctx.close()
    ctx2 = make_ctx(P, w, mixed_grid, tables, 0)
    ctx2.restore(blob)
    while not ctx2.propagate(0):
        pass
    got = ctx2.read_finished()
    _assert_identical(ref, got)
    c2 = ctx2.counts()
    for k in CNT_KEYS:
        assert c2[k] == rc[k]
    ctx2.close()


# ---------------------------------------------------------------------------
# Error paths and edge cases.
# ---------------------------------------------------------------------------
def test_inject_validation_all_or_nothing(P, small_grid):
    w = I.W_SMALL
    ctx = make_ctx(P, w, small_grid, w.make_tables(), 0)
    inj = w.make_injection(10)
    inj.Z = inj.Z.copy()
    inj.Z[7] = 3          # Z > A
    say("inject validation")
    with pytest.raises(P.CrpError) as ei:
        ctx.inject(inj)
    assert ei.value.status == -1 and "candidate 7" in str(ei.value)
    assert ctx.counts()["pending"] == 0
    inj2 = w.make_injection(10)
    inj2.dir = inj2.dir * 1.001
    with pytest.raises(P.CrpError):
        ctx.inject(inj2)
    ctx.inject(w.make_injection(10))
    assert ctx.counts()["pending"] == 10
    assert ctx.propagate()
    assert len(ctx.read_finished()["id"]) == 10
    ctx.close()


def test_empty_and_capacity(P, mixed_grid):
    w = I.W_MIXED256
    tables = w.make_tables()
    ctx = make_ctx(P, w, mixed_grid, tables, 0, qcap=256)
    say("empty / capacity")
    assert ctx.propagate()                  # nothing pending
    with pytest.raises(P.CrpError) as ei:
        ctx.inject(w.make_injection(300))
    assert ei.value.status == -5
    assert ctx.counts()["pending"] == 0     # all or nothing
    ctx.close()


def test_failed_allocation_leaves_later_calls_working(P, small_grid):
    """A device allocation that does not fit fails with CRP_ENOMEM and leaves
    nothing behind that a later call would report: a context asking for a
    2^40-slot queue is refused, and the next context runs a workload to
    completion with every primary finished."""
    w = I.W_SMALL
    say("allocation failure, then a normal run")
    prm = P.params_for(w, P.FP64, queue_capacity=1 << 40, neutral_capacity=1 << 12)
    with pytest.raises(P.CrpError) as ei:
        P.Context(prm)
    assert ei.value.status == -3
    ctx = make_ctx(P, w, small_grid, w.make_tables(), 0)
    inj = w.make_injection(200)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done and cg["finished"] == 200 and len(fg["id"]) == 200
    ctx.close()


def _spawning_injection(w, n):
    """Heavy nuclei above the channels' thresholds: many secondaries (nucleon
    loss) and neutral records (pion-like) per primary."""
    inj = w.make_injection(n)
    inj.A[:] = 56
    inj.Z[:] = 26
    inj.E[:] = np.where(np.arange(n) % 2 == 0, 5e20, 3e21)
    return inj


def _drain_run(P, ctx, inj, max_cycles=0):
    """Propagates to completion, reading the neutral records whenever the
    buffer is full; returns (finished, neutral, counters, number of waits)."""
    ctx.inject(inj)
    fins, neus, waits = [], [], 0
    while True:
        try:
            done = ctx.propagate(max_cycles)
        except P.CrpError as e:
            assert e.status == P.EOVERFLOW, e
            waits += 1
            done = False
        fins.append(ctx.read_finished())
        neus.append(ctx.read_neutral())
        if done:
            break
    fin = {k: np.concatenate([f[k] for f in fins]) for k in fins[0]}
    neu = {k: np.concatenate([n[k] for n in neus]) for k in neus[0]}
    return fin, neu, ctx.counts(), waits


@pytest.mark.parametrize("precision,layout", [(0, 0), (1, 0), (0, 1)],
                         ids=["fp64", "mix", "fp64-corner"])
def test_capacity_starved_run_equals_roomy_run(P, O, mixed_grid, precision, layout):
    """Nothing is lost when the queue or the neutral-record buffer is too
    small: spawning candidates wait (parked just before their interaction),
    the queue doubles and the run goes on; with a full neutral buffer the
    caller reads the records and propagates again.  The records equal those
    of a run with room to spare (linear layout), bit for bit, and the
    oracle's; the starved runs read the grid in the given layout (1: the FP64
    grid's corner records, whose wave-wide gathers skip the parked lanes)."""
    w = I.W_MIXED256
    tables = w.make_tables()
    grid = mixed_grid if precision == 0 else mixed_grid.astype(np.float32)
    inj = _spawning_injection(w, 256)
    say(f"roomy run precision={precision}")
    roomy = make_ctx(P, w, grid, tables, precision, qcap=1 << 16, ncap=1 << 16)
    fr, nr, cr, waits = _drain_run(P, roomy, inj)
    roomy.close()
    assert waits == 0 and cr["queue_deferred"] == 0 and cr["charged_sec"] > 256
    assert cr["neutral_sec"] > 64
    for qcap, ncap, budget in ((256, 1 << 16, 0), (256, 16, 0), (300, 40, 25)):
        say(f"starved run qcap={qcap} ncap={ncap} budget={budget}")
        ctx = make_ctx(P, w, grid, tables, precision, qcap=qcap, ncap=ncap)
        ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=layout)
        fs, ns, cs, waits = _drain_run(P, ctx, inj, budget)
        ctx.close()
        assert cs["queue_deferred"] > 0
        if ncap < cr["neutral_sec"]:
            assert waits > 0 and cs["neutral_deferred"] > 0
        _assert_identical(fr, fs)
        a, b = P.sort_neutral(nr), P.sort_neutral(ns)
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        for k in CNT_KEYS:
            assert cr[k] == cs[k], k
    fo, no, co, _ = O.propagate(O.config_for(w, precision=precision),
                                O.GridRef(grid, w.spacing_m), O.TablesRef(tables), inj,
                                nthreads=0, neu_cap=1 << 16)
    compare_counts(cr, co, "spawning")
    compare_records(fr, fo, f"spawning p{precision}")
    compare_neutral(nr, no, "spawning neutral", fo)


def test_single_candidate_and_ragged_batch(P, O, mixed_grid):
    """Batches of 1 and 65 candidates (one full wave plus one lane)."""
    w = I.W_MIXED256
    tables = w.make_tables()
    for n in (1, 65):
        inj = w.make_injection(n)
        ctx = make_ctx(P, w, mixed_grid, tables, 0)
        say(f"ragged n={n}")
        done, fg, ng, cg = run_gpu(ctx, inj)
        fo, no, co, _ = O.propagate(O.config_for(w), O.GridRef(mixed_grid, w.spacing_m),
                                    O.TablesRef(tables), inj)
        compare_counts(cg, co, f"n={n}")
        compare_records(fg, fo, f"n={n}")
        ctx.close()


# ---------------------------------------------------------------------------
# Degenerate cases of the method: energies below the floor and beyond both
# ends of the tables, the lightest and heaviest nuclei the boundary accepts,
# axis-aligned directions, starts on grid vertices and just below a vertex
# (the cell offset rounds to 1), trajectory limits far below the minimum step;
# then a field-free grid (straight lines) and a fixed step (hmin = hmax).
# ---------------------------------------------------------------------------
def _edge_injection(spacing):
    species = [(1, 1), (2, 1), (4, 2), (14, 7), (56, 26), (255, 1), (255, 100), (255, 255)]
    energies = [1e15, 1e16, 1.0000001e16, 1e18, 1e21, 1e23, 1e24, 1e26]
    n = 70                                                   # one wave and six lanes
    rng = np.random.default_rng(77)
    A = np.array([species[i % 8][0] for i in range(n)], np.int32)
    Z = np.array([species[i % 8][1] for i in range(n)], np.int32)
    E = np.array([energies[(i // 8 + i) % 8] for i in range(n)])
    d = rng.standard_normal((n, 3))
    d[:6] = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos = rng.uniform(-300.0, 300.0, (n, 3)) * spacing
    pos[:10] = np.round(pos[:10] / spacing) * spacing        # on vertices
    pos[10] = (0.0, -0.0, 0.0)
    pos[11] = (-1e-30, -1e-30, -1e-30)                       # offset rounds to 1
    lmax = np.full(n, 100 * I.MPC_M)
    lmax[12], lmax[13], lmax[14] = 1.0, 1e3, 1e-3 * spacing  # below the minimum step
    return I.Injection(np.arange(n, dtype=np.uint32), A, Z, E, pos, d, lmax)


@pytest.mark.parametrize("precision", [0, 1])
def test_degenerate_cases_match_oracle(P, O, mixed_grid, precision):
    w = I.W_MIXED256
    tables = w.make_tables()
    inj = _edge_injection(w.spacing_m)
    grid = mixed_grid if precision == 0 else mixed_grid.astype(np.float32)
    say(f"degenerate cases precision={precision}")
    ctx = make_ctx(P, w, grid, tables, precision, ncap=1 << 20)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done
    fo, no, co, _ = O.propagate(O.config_for(w, precision=precision),
                                O.GridRef(grid, w.spacing_m), O.TablesRef(tables), inj,
                                nthreads=0, neu_cap=1 << 20)
    compare_counts(cg, co, "degenerate")
    assert co["energy_floor"] > 0 and co["charged_sec"] > 0 and co["forced"] > 0
    same = compare_records(fg, fo, f"degenerate p{precision}")
    assert same.all()
    compare_neutral(ng, no, "degenerate neutral", fo)
    ctx.close()


def test_field_free_and_fixed_step_match_oracle(P, O, mixed_grid):
    w = I.W_MIXED256
    tables = w.make_tables()
    inj = _edge_injection(w.spacing_m)
    zero = np.zeros((8, 8, 8, 3))
    say("field-free grid")
    ctx = make_ctx(P, w, zero, tables, 0, ncap=1 << 20)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done
    fo, no, co, _ = O.propagate(O.config_for(w), O.GridRef(zero, w.spacing_m),
                                O.TablesRef(tables), inj, nthreads=0, neu_cap=1 << 20)
    compare_counts(cg, co, "field-free")
    assert compare_records(fg, fo, "field-free").all()
    # straight lines: the primaries end at x0 + L u0
    fg = P.sort_finished(fg)
    prim = fg["lineage"] == 0
    ids = fg["id"][prim]
    x0 = inj.pos[ids]
    dev = np.linalg.norm(fg["x"][prim] - (x0 + fg["L"][prim, None] * inj.dir[ids]), axis=1)
    assert np.all(dev <= 1e-9 * np.maximum(fg["L"][prim], 1.0) + 1e-9 * np.linalg.norm(x0, axis=1))
    assert np.array_equal(fg["u0"][prim], inj.dir[ids])
    ctx.close()
    h = 100 * I.KPC_M
    say("fixed step hmin = hmax")
    ctx = make_ctx(P, w, mixed_grid, tables, 0, ncap=1 << 20, hmin=h, hmax=h)
    done, fg, ng, cg = run_gpu(ctx, inj)
    assert done
    fo, no, co, _ = O.propagate(O.config_for(w, hmin=h, hmax=h),
                                O.GridRef(mixed_grid, w.spacing_m), O.TablesRef(tables), inj,
                                nthreads=0, neu_cap=1 << 20)
    compare_counts(cg, co, "fixed step")
    assert compare_records(fg, fo, "fixed step").all()
    compare_neutral(ng, no, "fixed step neutral", fo)
    ctx.close()


def test_read_back_in_chunks(P):
    """More finished records than one read-back chunk (2^25 rows): positions
    and directions interleaved chunk by chunk come back in the right rows.  A
    field-free grid and a trajectory limit below the minimum step make every
    candidate one straight step, x = x0 + L u0."""
    import torch
    w = I.W_SMALL
    n = (1 << 25) + 1000
    rng = np.random.default_rng(91)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos = rng.uniform(-1.0, 1.0, (n, 3)) * 3 * I.MPC_M
    dev = dict(id=torch.arange(n, dtype=torch.int32, device="cuda:0"),
               A=torch.ones(n, dtype=torch.int32, device="cuda:0"),
               Z=torch.ones(n, dtype=torch.int32, device="cuda:0"),
               E=torch.full((n,), 1e19, dtype=torch.float64, device="cuda:0"),
               pos=torch.as_tensor(pos, device="cuda:0"), dir=torch.as_tensor(d, device="cuda:0"),
               lmax=torch.full((n,), 1e-3 * w.hmin_m, dtype=torch.float64, device="cuda:0"))
    ctx = make_ctx(P, w, np.zeros((8, 8, 8, 3)), w.make_tables(), P.FP64, qcap=n, ncap=1 << 10)
    say(f"read-back in chunks: {n} candidates")
    ctx.inject(**dev, on_device=True)
    assert ctx.propagate()
    fin = ctx.read_finished()
    assert len(fin["id"]) == n
    order = np.argsort(fin["id"])
    ids = fin["id"][order].astype(np.int64)
    assert np.array_equal(ids, np.arange(n))
    x, u, u0, L = fin["x"][order], fin["u"][order], fin["u0"][order], fin["L"][order]
    assert np.array_equal(u0, d)
    assert np.all(np.abs(u - d) <= 4e-16)
    assert np.all(np.linalg.norm(x - (pos + L[:, None] * d), axis=1) <= 1e-12 * 3 * I.MPC_M)
    ctx.close()


def test_tuner_cache_round_trip(P, mixed_grid, tmp_path):
    """The autotuner appends its choice under a key of (device, grid shape,
    element type, precision, field mode) and takes the latest entry of that
    key from the cache without trials (and without pending work); other keys
    and malformed lines are ignored; the tuning leaves pending work as it was."""
    w = I.W_MIXED256
    tables = w.make_tables()
    cache = str(tmp_path / "tune.txt")
    open(cache, "w").write("garbage line\nanother : block=7 refill=x\n")
    inj = w.make_injection(3000)
    ctx = make_ctx(P, w, mixed_grid, tables, 0)
    ctx.inject(inj)
    say("tuner with an empty cache")
    best, rate = ctx.tune(max_cycles=0, cache_path=cache)
    assert rate > 0 and ctx.get_launch() == best
    assert ctx.counts()["pending"] == 3000           # the calibration work is still there
    lines = open(cache).read().splitlines()
    assert len(lines) == 3 and lines[-1].split(" : ")[1].startswith(f"block={best['block']}")
    ctx.close()
    # a new context of the same key: the cached shape, no trials, no pending work needed
    ctx = make_ctx(P, w, mixed_grid, tables, 0)
    ctx.set_launch(block=256, blocks_per_cu=2, refill=64)
    best2, rate2 = ctx.tune(max_cycles=0, cache_path=cache)
    assert best2 == best and rate2 == pytest.approx(rate, rel=1e-6)
    assert ctx.get_launch() == best
    ctx.close()
    # another key (the precision form): no entry, so trials -- which need work
    ctx = make_ctx(P, w, mixed_grid, tables, 1)
    with pytest.raises(P.CrpError) as ei:
        ctx.tune(max_cycles=0, cache_path=cache)
    assert ei.value.status == -4
    ctx.close()
