"""GPU parity of the galactic lenses (section 4: PARSEC-style transformation
matrices per energy range), through the C-ABI: construction from the records
of a backtracking run on the GPU against the oracle's construction from the
same records read back (bitwise: integer counts and one FP64 division per
entry), and the application to border maps against the oracle's sparse
product (FP64, the order of the sums differs: within (row length + 2) ulp of
the sum of |terms|).  The backtracking itself is compared with the oracle's
in tests/test_gpu_galactic.py; the GPU run is deterministic (the same records
for the same events in every launch), which the lens tests rely on."""
import numpy as np
import pytest

import crp_inputs as I
from oracle import lens as LN
from parity_helpers import say

pytestmark = pytest.mark.gpu

W = I.W_GALBACK


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


def backtrack_gpu(P, inj, model=None, precision=0):
    prm = P.params_for(W, precision, queue_capacity=1 << 16, neutral_capacity=1 << 10)
    ctx = P.Context(prm)
    ctx.set_field_analytic(model or I.GALACTIC_FIELD)
    ctx.set_tables(W.make_tables())
    ctx.inject(inj)
    assert ctx.propagate()
    return ctx


@pytest.fixture(scope="module")
def events(P):
    """6000 seeded events and the GPU's backtracked records of them."""
    inj = W.make_injection(6000)
    ctx = backtrack_gpu(P, inj)
    fg = ctx.read_finished()
    ctx.close()
    return inj, fg


def compare_lens(Lg, Lo, what):
    assert np.array_equal(Lg["rowptr"], Lo["rowptr"]), what
    assert np.array_equal(Lg["col"], Lo["col"]), what
    assert np.array_equal(Lg["count"].astype(np.int64), Lo["count"]), what
    assert np.array_equal(Lg["val"], Lo["val"]), what
    say(f"{what}: {len(Lo['col'])} entries bitwise identical")


def check_apply(P, ctx, Lo, seed, n_maps=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, (n_maps, Lo["n_r"], Lo["npix"]))
    y, ms = ctx.lens_apply(x)
    ref = LN.apply(Lo, x)
    # bound of a sum in any order: (terms + 2) ulp of sum |terms| (x >= 0, val > 0)
    nrow = np.diff(Lo["rowptr"]).reshape(Lo["n_r"], Lo["npix"])
    tol = (nrow + 2) * 2.0 ** -52 * ref
    assert np.all(np.abs(y - ref) <= tol + 1e-300)
    import torch
    xd = torch.as_tensor(x, device="cuda:0")
    yd, _ = ctx.lens_apply(xd)
    assert np.array_equal(yd.cpu().numpy(), y)
    return ms


@pytest.mark.parametrize("sky_n", [2, 8, 24], ids=["long-rows", "mid", "short-rows"])
def test_lens_build_and_apply_parity(P, O, events, sky_n):
    inj, fg = events
    sp = LN.spec(10.0 ** np.linspace(16.5, 20.0, 6), sky_n=sky_n)
    ctx = backtrack_gpu(P, inj)
    say(f"lens sky_n={sky_n}")
    nnz, ms = ctx.lens_build(sp)
    Lg = ctx.lens_read()
    assert ctx.counts()["finished_unread"] == len(fg["id"])     # records stay unread
    Lo = LN.build(sp, fg)
    assert nnz == len(Lo["col"])
    compare_lens(Lg, Lo, f"lens sky_n={sky_n}")
    check_apply(P, ctx, Lo, sky_n)
    ctx.close()


def test_field_free_identity_and_edge_cases(P, O):
    inj = W.make_injection(1000)
    zero = {k: (0.0 if k.startswith("b_") else v) for k, v in I.GALACTIC_FIELD.items()}
    prm = P.params_for(W, P.FP64, queue_capacity=1 << 14, neutral_capacity=1 << 10,
                       renormalize=0)
    ctx = P.Context(prm)
    with pytest.raises(P.CrpError):
        ctx.lens_read()                                        # nothing built yet
    ctx.set_field_analytic(zero)
    ctx.set_tables(W.make_tables())
    ctx.inject(inj)
    assert ctx.propagate()
    sp = LN.spec([1e16, 1e21], sky_n=5)
    say("lens identity")
    nnz, _ = ctx.lens_build(sp)
    L = ctx.lens_read()
    rows = np.repeat(np.arange(len(L["rowptr"]) - 1), np.diff(L["rowptr"]))
    assert np.all(L["col"] == rows % L["npix"]) and np.all(L["val"] == 1.0)
    # a range no record falls in: an empty lens, maps to zero
    nnz, _ = ctx.lens_build(LN.spec([1e25, 1e26], sky_n=3))
    assert nnz == 0
    y, _ = ctx.lens_apply(np.ones((2, 1, 54)))
    assert np.all(y == 0.0)
    for bad in (LN.spec([1e18, 1e18], sky_n=2), LN.spec([1e18, 1e19], sky_n=0),
                LN.spec([1e18, 1e19], sky_n=600)):
        with pytest.raises(P.CrpError):
            ctx.lens_build(bad)
    ctx.close()


def test_full_size_lens_properties(P, O):
    """The bench's lens set: 1e7 backtracked events (the full galactic batch),
    7 rigidity bins x 6144 pixels.  Checked by properties that hold at any
    size, and the first 2000 events' lens against the oracle's construction
    from the same records."""
    import torch
    n = 10_000_000
    inj = W.make_injection(n)
    prm = P.params_for(W, P.FP64, queue_capacity=2 * n, neutral_capacity=1 << 10)
    ctx = P.Context(prm)
    ctx.set_field_analytic(I.GALACTIC_FIELD)
    ctx.set_tables(W.make_tables())
    dev = [torch.as_tensor(a, device="cuda:0") for a in
           (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
    say("full-size lens: backtracking 1e7 events")
    ctx.inject(id=dev[0], A=dev[1], Z=dev[2], E=dev[3], pos=dev[4], dir=dev[5], lmax=dev[6],
               on_device=True)
    assert ctx.propagate()
    cnt = ctx.counts()
    edges = 10.0 ** np.linspace(16.5, 20.0, 8)
    sp = LN.spec(edges, sky_n=32)
    nnz, ms = ctx.lens_build(sp)
    L = ctx.lens_read()
    say(f"lens: {nnz} entries in {ms:.2f} ms")
    R = inj.E / inj.Z
    in_range = (R >= edges[0]) & (R < edges[-1])
    # every boundary event in range is counted once (events that reach the length
    # limit instead are not in the lens)
    assert int(L["count"].sum()) <= int(in_range.sum())
    assert int(L["count"].sum()) >= int(in_range.sum()) - cnt["max_traj"]
    rowlen = np.diff(L["rowptr"])
    rows = np.repeat(np.arange(len(rowlen)), rowlen)
    assert np.all(np.diff(L["col"])[np.diff(rows) == 0] > 0)          # sorted columns
    sums = np.bincount(rows, weights=L["val"], minlength=len(rowlen))
    assert np.all(np.abs(sums[rowlen > 0] - 1.0) <= 4e-16 * rowlen[rowlen > 0])
    y, _ = ctx.lens_apply(np.ones((1, 7, L["npix"])))
    assert np.allclose(y.ravel()[rowlen > 0], 1.0, rtol=1e-13) and np.all(y.ravel()[rowlen == 0] == 0)
    ctx.close()
    # the first 2000 events alone: the same lens as the oracle's from its own run
    sub = inj.subset(np.arange(2000))
    c2 = backtrack_gpu(P, sub)
    c2.lens_build(sp)
    Lg = c2.lens_read()
    fg = c2.read_finished()
    c2.close()
    compare_lens(Lg, LN.build(sp, fg), "first 2000 events")


def test_rebuilds_in_one_context(P, O, events):
    """Builds of growing, empty and shrinking lens sets in one context (the
    construction scratch and matrix buffers are reused) each equal the
    oracle's."""
    inj, fg = events
    ctx = backtrack_gpu(P, inj)
    edges = 10.0 ** np.linspace(16.5, 20.0, 6)
    for sky_n, e in ((2, edges), (24, edges), (3, [1e25, 1e26]), (8, edges), (24, edges[:3])):
        sp = LN.spec(e, sky_n=sky_n)
        say(f"rebuild sky_n={sky_n} bins={len(e) - 1}")
        nnz, _ = ctx.lens_build(sp)
        Lo = LN.build(sp, fg)
        assert nnz == len(Lo["col"])
        compare_lens(ctx.lens_read(), Lo, f"rebuild sky_n={sky_n}")
        if nnz:
            check_apply(P, ctx, Lo, sky_n + 100, n_maps=5)
    ctx.close()


def test_grouped_application_matches_four_map_passes(P, O, events):
    """More than four maps go through the pixel-interleaved path (groups of
    16 maps, the last one partial); every map's result has the bits of the
    same map applied in a pass of at most four, and the oracle's bound."""
    inj, fg = events
    ctx = backtrack_gpu(P, inj)
    sp = LN.spec(10.0 ** np.linspace(16.5, 20.0, 6), sky_n=8)
    ctx.lens_build(sp)
    Lo = LN.build(sp, fg)
    rng = np.random.default_rng(44)
    x = rng.uniform(0.0, 1.0, (21, Lo["n_r"], Lo["npix"]))
    say("grouped lens application, 21 maps")
    y, _ = ctx.lens_apply(x)
    parts = np.concatenate([ctx.lens_apply(x[k:k + 4])[0] for k in range(0, 21, 4)])
    assert np.array_equal(y, parts)
    ref = LN.apply(Lo, x)
    nrow = np.diff(Lo["rowptr"]).reshape(Lo["n_r"], Lo["npix"])
    assert np.all(np.abs(y - ref) <= (nrow + 2) * 2.0 ** -52 * ref + 1e-300)
    ctx.close()
