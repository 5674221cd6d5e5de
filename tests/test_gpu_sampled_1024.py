"""Full-size parity: the 1e7-candidate mixed-nuclei batch on the 1024^3 FP32
grid, propagated whole on the GPU in the launch the autotuner picks (the
configuration the benchmark times), checked against the oracle on a sample of
candidates that the oracle follows one by one, and against properties that
hold at any size.

Every candidate's history depends only on its own inputs and its counter-based
random stream (key: seed, id, lineage), so the oracle run on the sampled
candidates alone must reproduce every record the GPU wrote for them, including
their secondaries: bitwise here, as both sides take the same operation order.
"""
import os

import numpy as np
import pytest

import crp_inputs as I
from parity_helpers import compare_neutral, compare_records, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

W = I.W_MIXED1024
N_SAMPLE = 400


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
def big():
    """Device grid, host copy for the oracle, tables and the injection batch."""
    import torch
    say(f"generating {W.grid_n}^3 grid on the GPU")
    grid = W.make_grid(device="cuda:0")
    torch.cuda.synchronize()
    host = grid.cpu().numpy()
    tables = W.make_tables()
    inj = W.make_injection()
    d_inj = [torch.as_tensor(a, device="cuda:0") for a in
             (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
    state = {"grid": grid, "host": host, "tables": tables, "inj": inj, "d_inj": d_inj,
             "launch": None}
    yield state
    state.clear()
    torch.cuda.empty_cache()


def _context(P, big, precision):
    n = W.n_candidates
    prm = P.params_for(W, precision, device=0, queue_capacity=2 * n,
                       neutral_capacity=max(n, 1 << 20))
    ctx = P.Context(prm)
    ctx.set_field_grid(big["grid"], W.spacing_m)
    ctx.set_tables(big["tables"])
    return ctx


def _inject(ctx, d, count=None):
    s = slice(0, count)
    ctx.inject(id=d[0][s], A=d[1][s], Z=d[2][s], E=d[3][s], pos=d[4][s], dir=d[5][s],
               lmax=d[6][s], on_device=True)


def _sample_ids(n):
    rng = np.random.default_rng(4242)
    ids = rng.choice(n, N_SAMPLE - 8, replace=False)
    # the first and last candidates of the batch (its ragged end) as well
    return np.unique(np.concatenate([ids, np.arange(4), np.arange(n - 4, n)]))


def _digest(P, fin):
    """SHA-256 of every field of the records in (id, lineage) order."""
    import hashlib
    f = P.sort_finished(fin)
    h = hashlib.sha256()
    for k in sorted(f):
        h.update(np.ascontiguousarray(f[k]).tobytes())
    return h.hexdigest()


def _select(rec, ids):
    keep = np.isin(rec["id"], ids)
    return {k: v[keep] for k, v in rec.items()}


def _check_whole_batch(P, fin, neu, cnt, n):
    """Properties of the full output that hold at any size."""
    key = (fin["id"].astype(np.int64) << 32) | fin["lineage"].astype(np.int64)
    assert np.unique(key).size == key.size, "duplicate (id, lineage) records"
    prim = fin["lineage"] == 0
    assert prim.sum() == n and np.array_equal(np.sort(fin["id"][prim]), np.arange(n))
    assert cnt["finished"] == len(fin["id"])
    assert cnt["observed"] + cnt["max_traj"] + cnt["energy_floor"] == cnt["finished"]
    assert cnt["finished"] == n + cnt["charged_sec"]
    assert len(neu["id"]) == cnt["neutral_sec"]
    assert cnt["queue_deferred"] == 0 and cnt["neutral_deferred"] == 0
    assert np.all(fin["Z"] >= 1) and np.all(fin["Z"] <= fin["A"])
    assert np.all(np.isfinite(fin["x"])) and np.all(fin["E"] > 0)
    # the last step is shortened to end on the trajectory budget
    assert np.all(fin["L"] <= W.lmax_m)
    un = np.linalg.norm(fin["u"], axis=1)
    assert np.all(np.abs(un - 1.0) < 1e-6)


def test_autotuned_launch(P, big):
    """The benchmark's tuning step for this workload: the batch's first
    TUNE_N_HEADLINE candidates, every trial run to completion."""
    from bench import TUNE_N_HEADLINE
    ctx = _context(P, big, P.MIX)
    _inject(ctx, big["d_inj"], TUNE_N_HEADLINE)
    say(f"autotuning on {TUNE_N_HEADLINE} candidates")
    tuned, rate = ctx.tune(max_cycles=0, cache_path=None)
    ctx.close()
    big["launch"] = dict(tuned)
    say(f"tuned launch {big['launch']} ({rate:.3e} steps/s)")
    assert rate > 0


@pytest.mark.parametrize("precision", [1, 0], ids=["mix", "fp64"])
def test_full_batch_sampled_parity(P, O, big, precision):
    n = W.n_candidates
    ctx = _context(P, big, precision)
    if big["launch"]:
        ctx.set_launch(**big["launch"])
    launch = ctx.get_launch()
    say(f"full batch n={n} precision={precision} launch={launch}")
    _inject(ctx, big["d_inj"])
    assert ctx.propagate(0)
    cnt = ctx.counts()
    fin = ctx.read_finished()
    neu = ctx.read_neutral()
    ctx.close()
    say(f"gpu: {len(fin['id'])} finished, {len(neu['id'])} neutral, {cnt['steps']} steps")
    _check_whole_batch(P, fin, neu, cnt, n)
    big[f"digest{precision}"] = (_digest(P, fin), {k: cnt[k] for k in
                                                   ("steps", "attempts", "finished", "events")})

    ids = _sample_ids(n)
    sub = big["inj"].subset(ids)
    G = O.GridRef(big["host"], W.spacing_m)
    T = O.TablesRef(big["tables"])
    threads = len(os.sched_getaffinity(0))
    fo, no, co, _ = O.propagate(O.config_for(W, precision=precision), G, T, sub,
                                nthreads=threads)
    say(f"oracle: {len(fo['id'])} records for {len(ids)} sampled candidates")
    fg = _select(fin, ids)
    same = compare_records(fg, fo, f"1024^3 sample p{precision}")
    assert same.all()
    compare_neutral(_select(neu, ids), no, f"1024^3 sample neutral p{precision}", fo)


def test_full_batch_trajectory_and_observables(P, O, big):
    """The full batch with per-step output for the first 200 candidate ids and
    the observable reduction over all of its finished records: the points of
    those candidates (and of their secondaries) against the oracle run on them
    alone; the reduction against properties that hold at any size."""
    from oracle import observables as OB
    n = W.n_candidates
    ids = 200
    prm = P.params_for(W, P.MIX, device=0, queue_capacity=2 * n,
                       neutral_capacity=max(n, 1 << 20), traj_every=1, traj_ids=ids,
                       traj_capacity=1 << 24)
    ctx = P.Context(prm)
    ctx.set_field_grid(big["grid"], W.spacing_m)
    ctx.set_tables(big["tables"])
    if big["launch"]:
        ctx.set_launch(**big["launch"])
    say(f"full batch with trajectory output of ids < {ids}, launch={ctx.get_launch()}")
    _inject(ctx, big["d_inj"])
    assert ctx.propagate(0)
    sp = OB.spec(10.0 ** np.linspace(15.0, 22.0, 29), a_edges=(1, 2, 5, 15, 57),
                 status_mask=0b11110, sky_n=32, sky_sign=-1.0, e_ref=1e18, gamma=-1.5)
    ctx.set_observables(sp)
    ctx.observe()
    ob = ctx.read_observables()
    cnt = ctx.counts()
    tg = ctx.read_trajectory()
    ctx.close()
    assert cnt["traj_dropped"] == 0 and cnt["traj_points"] == len(tg["id"])
    # observables: every finished record lands in one bin or in `outside`
    assert int(ob["counts"].sum()) + ob["outside"] == cnt["finished"]
    assert np.array_equal(ob["sky"].sum(axis=2), ob["counts"])
    c = ob["counts"].astype(np.float64)
    nz = c > 0
    mean = ob["defl"][nz].astype(np.float64) / OB.DEFL_SCALE / c[nz]
    assert np.all(mean >= 0) and np.all(mean <= np.pi)
    assert np.all(ob["wsum"][nz] > 0) and np.all(ob["wsum"][~nz] == 0)
    # trajectory points of the first candidates, bitwise against the oracle
    sub = big["inj"].subset(np.arange(ids))
    G = O.GridRef(big["host"], W.spacing_m)
    T = O.TablesRef(big["tables"])
    cfg = O.config_for(W, precision=O.MIX, traj_every=1, traj_ids=ids)
    _, _, _, to = O.propagate_traj(cfg, G, T, sub, 1 << 24,
                                   nthreads=len(os.sched_getaffinity(0)))
    tg = P.sort_traj(tg)
    to = O.sort_traj(to)
    assert len(tg["id"]) == len(to["id"])
    for k in to:
        assert np.array_equal(tg[k], to[k]), k
    say(f"{len(to['id'])} trajectory points of {ids} candidates bitwise identical; "
        f"{int(ob['counts'].sum())} records observed in {int(nz.sum())} bins")


def test_full_batch_multiresolution_sampled_parity(P, O, big):
    """The bench's multi-resolution case: the 1e7 batch started at the centre
    of a 512^3 refine-4 patch inside the 1024^3 grid, corner records for both
    levels, against the oracle on 200 sampled candidates with all their
    secondaries."""
    import torch
    n = W.n_candidates
    nside, refine, off = 512, 4, 448
    say("generating the 512^3 patch on the GPU")
    patch = I.turbulent_grid(nside, W.spacing_m / refine, 2.0, 64.0, W.brms_T, 31, np.float32,
                             device="cuda:0")
    torch.cuda.synchronize()
    centre = (off + nside / refine / 2) * W.spacing_m
    inj = big["inj"]
    pos = np.full((n, 3), centre)
    d = big["d_inj"]
    ctx = _context(P, big, P.MIX)
    ctx.set_field_patches([dict(data=patch, offset=(off, off, off), refine=refine)])
    ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=P.LAYOUT_CORNER)
    dpos = torch.as_tensor(pos, device="cuda:0")
    say("full batch from the patch centre")
    ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=dpos, dir=d[5], lmax=d[6], on_device=True)
    assert ctx.propagate(0)
    fin = ctx.read_finished()
    cnt = ctx.counts()
    ctx.close()
    host_patch = patch.cpu().numpy()
    del patch, dpos
    torch.cuda.empty_cache()
    assert cnt["finished"] == len(fin["id"]) == n + cnt["charged_sec"]
    ids = np.random.default_rng(4343).choice(n, 200, replace=False)
    sub = I.Injection(inj.id[ids], inj.A[ids], inj.Z[ids], inj.E[ids], pos[ids], inj.dir[ids],
                      inj.lmax[ids])
    G = O.GridRef(big["host"], W.spacing_m,
                  patches=[dict(data=host_patch, offset=(off, off, off), refine=refine)])
    fo, _, _, _ = O.propagate(O.config_for(W, precision=O.MIX), G, O.TablesRef(big["tables"]),
                              sub, nthreads=len(os.sched_getaffinity(0)))
    same = compare_records(_select(fin, ids), fo, "multi-resolution 1024^3 sample")
    assert same.all()


def test_batch_split_invariance_full_size(P, big):
    """The same 1e7 candidates injected and propagated as 10 batches of 1e6 in
    one context give bitwise the same records as the single 1e7 launch (each
    candidate's history depends only on its own inputs and random stream)."""
    if "digest1" not in big:
        pytest.skip("needs the full-batch precision-form run of this module")
    n = W.n_candidates
    ctx = _context(P, big, P.MIX)
    if big["launch"]:
        ctx.set_launch(**big["launch"])
    d = big["d_inj"]
    parts = []
    for b in range(10):
        s = slice(b * n // 10, (b + 1) * n // 10)
        say(f"batch {b}: candidates {s.start}..{s.stop}")
        ctx.inject(id=d[0][s], A=d[1][s], Z=d[2][s], E=d[3][s], pos=d[4][s], dir=d[5][s],
                   lmax=d[6][s], on_device=True)
        assert ctx.propagate(0)
        parts.append(ctx.read_finished())
    cnt = ctx.counts()
    ctx.close()
    fin = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    digest, ref_cnt = big["digest1"]
    for k, v in ref_cnt.items():
        assert cnt[k] == v, k
    assert _digest(P, fin) == digest


def test_neural_field_full_size(P, big):
    """The learned form at full size: the network trained on 1e8 points of the
    1024^3 grid by the library's own kernels, its RMS field error against the
    grid on held-out points, and the deflection-angle distribution of 2e5
    distance-workload candidates propagated with it against the grid run (the
    grid path is the reference).  The network replaces a 12.9 GB field with
    132,870 bytes of bf16 weights."""
    wd = I.W_DIST1024
    m = 200_000
    prm = P.params_for(wd, P.MIX, device=0, field_mode=P.FIELD_NEURAL, queue_capacity=2 * m,
                       neutral_capacity=1 << 20)
    ctx = P.Context(prm)
    ctx.set_field_grid(big["grid"], wd.spacing_m)
    ctx.set_tables(big["tables"])
    ctx.nf_init(I.nf_frequencies(seed=505), I.nf_init_flat(509), wd.brms_T)
    say("training the network on 1e8 points")
    losses = ctx.nf_train(1526, 65536, 1e-3, 1e-5, 506)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.1 * losses[0]
    pos = I.uniform_points(200_000, wd.grid_n * wd.spacing_m, 507)
    Bn = ctx.eval_field(pos, P.EVAL_NEURAL)
    Bg = ctx.eval_field(pos, P.MIX)
    rms = float(np.sqrt(((Bn - Bg) ** 2).sum(1).mean()) / wd.brms_T)
    inj = I.inject_distances(m, 508)
    ctx.inject(inj)
    say("propagating 2e5 candidates with the network")
    assert ctx.propagate(0)
    fn = ctx.read_finished()
    ctx.close()
    gprm = P.params_for(wd, P.MIX, device=0, queue_capacity=2 * m, neutral_capacity=1 << 20)
    cg = P.Context(gprm)
    cg.set_field_grid(big["grid"], wd.spacing_m)
    cg.set_tables(big["tables"])
    cg.inject(inj)
    assert cg.propagate(0)
    fg = cg.read_finished()
    cg.close()

    def hist(f):
        th = np.degrees(np.arccos(np.clip((f["u"] * f["u0"]).sum(1), -1, 1)))
        return np.histogram(th, bins=36, range=(0, 180))[0] / len(th)

    dist = float(0.5 * np.abs(hist(fn) - hist(fg)).sum())
    say(f"network: RMS field error {rms:.3f} of B_rms, deflection histogram distance {dist:.4f}")
    # measured 0.27: 64 Fourier features do not represent the band to 1%; a regression guard
    assert rms < 0.35
    assert dist <= 0.02
    assert len(fn["id"]) >= m and len(fg["id"]) >= m


def test_neural_field_narrow_band_under_one_percent(P, big):
    """The learned form at its stated error: on a 1024^3 FP32 field of the band
    2..3 cycles per box (seed 3, 1 nG RMS, 10 kpc cells), whose 48 modes the 64
    Fourier features can hold, the network trained on 3e9 points (45,780 steps
    of 65,536, lr 3e-3 -> 1e-5) by the library's own kernels is within 1% RMS
    of the grid's field on held-out points, and 2e5 distance-workload
    candidates propagated with it have a deflection-angle histogram within 2%
    (total variation, 36 bins) of the grid run's."""
    import torch
    wd = I.W_DIST1024
    m = 200_000
    grid = I.turbulent_grid(wd.grid_n, wd.spacing_m, 2.0, 3.0, wd.brms_T, 3, np.float32,
                            torch.device("cuda:0"))
    prm = P.params_for(wd, P.MIX, device=0, field_mode=P.FIELD_NEURAL, queue_capacity=2 * m,
                       neutral_capacity=1 << 20)
    ctx = P.Context(prm)
    ctx.set_field_grid(grid, wd.spacing_m)
    ctx.set_tables(big["tables"])
    ctx.nf_init(I.nf_frequencies(nmin=2.0, nmax=3.0, seed=505), I.nf_init_flat(509), wd.brms_T)
    say("training the network on 3e9 points of the 2..3 band")
    losses = ctx.nf_train(45780, 65536, 3e-3, 1e-5, 506)
    assert np.all(np.isfinite(losses))
    pos = I.uniform_points(200_000, wd.grid_n * wd.spacing_m, 507)
    Bn = ctx.eval_field(pos, P.EVAL_NEURAL)
    Bg = ctx.eval_field(pos, P.MIX)
    rms = float(np.sqrt(((Bn - Bg) ** 2).sum(1).mean()) / wd.brms_T)
    say(f"narrow band: RMS field error {rms:.4f} of B_rms")
    assert rms <= 0.01
    inj = I.inject_distances(m, 508)
    ctx.inject(inj)
    assert ctx.propagate(0)
    fn = ctx.read_finished()
    ctx.close()
    gprm = P.params_for(wd, P.MIX, device=0, queue_capacity=2 * m, neutral_capacity=1 << 20)
    cg = P.Context(gprm)
    cg.set_field_grid(grid, wd.spacing_m)
    cg.set_tables(big["tables"])
    cg.inject(inj)
    assert cg.propagate(0)
    fg = cg.read_finished()
    cg.close()
    del grid
    torch.cuda.empty_cache()

    def hist(f):
        th = np.degrees(np.arccos(np.clip((f["u"] * f["u0"]).sum(1), -1, 1)))
        return np.histogram(th, bins=36, range=(0, 180))[0] / len(th)

    dist = float(0.5 * np.abs(hist(fn) - hist(fg)).sum())
    say(f"narrow band: deflection histogram distance {dist:.4f}")
    assert dist <= 0.02
    assert len(fn["id"]) >= m and len(fg["id"]) >= m
