"""GPU parity of the multi-resolution grid (section 4: multi-resolution grids
for fast access to precomputed fields): refinement patches with level
selection over the periodic base grid, through the C-ABI, against the oracle
on the same seeded inputs.  Bitwise: both sides locate, select and
interpolate with the same operations in the same order."""
import numpy as np
import pytest

import crp_inputs as I
from parity_helpers import compare_counts, compare_records, make_ctx, say

pytestmark = pytest.mark.gpu

W = I.W_SMALL


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
def fields():
    """Base grid (32^3, 100 kpc) and three patches cut from finer turbulent
    fields: refine 2 and 4 nested, and one refine-2 patch at the box edge."""
    base = W.make_grid()
    fine2 = I.turbulent_grid(64, W.spacing_m / 2, 2.0, 32.0, W.brms_T, 11)
    fine4 = I.turbulent_grid(64, W.spacing_m / 4, 2.0, 32.0, 2 * W.brms_T, 12)
    patches = [dict(data=fine2[:33, 5:30, 10:51].copy(), offset=(4, 4, 4), refine=2),
               dict(data=fine4[3:20, 0:17, 7:24].copy(), offset=(8, 6, 10), refine=4),
               dict(data=fine2[0:9, 0:64, 0:11].copy(), offset=(28, 0, 27), refine=2)]
    return base, patches


def _grid_pair(O, base, patches, dtype):
    b = base.astype(dtype)
    ps = [dict(q, data=q["data"].astype(dtype)) for q in patches]
    return b, ps, O.GridRef(b, W.spacing_m, patches=ps)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_nested_eval_bitwise(P, O, fields, dtype):
    base, patches = fields
    b, ps, G = _grid_pair(O, base, patches, dtype)
    ctx = make_ctx(P, W, b, W.make_tables(), P.FP64)
    ctx.set_field_patches(ps)
    rng = np.random.default_rng(21)
    box = 32 * W.spacing_m
    pos = rng.uniform(-2.0, 3.0, (200_000, 3)) * box
    # points on patch faces and base vertices
    pos[:64] = np.round(pos[:64] / W.spacing_m) * W.spacing_m
    pos[64:128] = (np.array([4.0, 4.0, 4.0]) + rng.integers(0, 20, (64, 3)) / 2.0) * W.spacing_m
    for mode, omode in ((0, O.FP64), (1, O.MIX)):
        say(f"nested eval dtype={np.dtype(dtype).name} mode={mode}")
        got = ctx.eval_field(pos, mode)
        ref = O.eval_field(G, pos, omode)
        assert np.array_equal(got, ref)
    # removing the patches gives back the plain grid
    ctx.set_field_patches([])
    assert np.array_equal(ctx.eval_field(pos[:1000], 0),
                          O.eval_field(O.GridRef(b, W.spacing_m), pos[:1000], O.FP64))
    ctx.close()


@pytest.mark.parametrize("precision,dtype", [(0, np.float64), (1, np.float64), (1, np.float32),
                                             (0, np.float32)],
                         ids=["fp64-f64", "mix-f64", "mix-f32", "fp64-f32"])
def test_nested_propagation_parity(P, O, fields, precision, dtype):
    base, patches = fields
    b, ps, G = _grid_pair(O, base, patches, dtype)
    inj = W.make_injection()
    ctx = make_ctx(P, W, b, W.make_tables(), precision)
    ctx.set_field_patches(ps)
    say(f"nested propagation precision={precision} dtype={np.dtype(dtype).name}")
    ctx.inject(inj)
    assert ctx.propagate()
    fg, cg = ctx.read_finished(), ctx.counts()
    ctx.close()
    fo, _, co, _ = O.propagate(O.config_for(W, precision=precision), G,
                               O.TablesRef(W.make_tables()), inj)
    compare_counts(cg, co, "nested")
    assert compare_records(fg, fo, f"nested p{precision}").all()
    # the patches changed the result
    fp, _, cp, _ = O.propagate(O.config_for(W, precision=precision), O.GridRef(b, W.spacing_m),
                               O.TablesRef(W.make_tables()), inj)
    assert cp["steps"] != co["steps"]


@pytest.mark.parametrize("precision", [1, 0], ids=["mix", "fp64"])
def test_nested_corner_records_parity(P, O, fields, precision):
    """FP32 grid and patches from corner records, gathered by the whole wave."""
    base, patches = fields
    b, ps, G = _grid_pair(O, base, patches, np.float32)
    inj = W.make_injection()
    ctx = make_ctx(P, W, b, W.make_tables(), precision)
    ctx.set_field_patches(ps)
    ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=P.LAYOUT_CORNER)
    say(f"nested corner records precision={precision}")
    ctx.inject(inj)
    assert ctx.propagate()
    fg, cg = ctx.read_finished(), ctx.counts()
    ctx.close()
    fo, _, co, _ = O.propagate(O.config_for(W, precision=precision), G,
                               O.TablesRef(W.make_tables()), inj)
    compare_counts(cg, co, "nested corner")
    assert compare_records(fg, fo, f"nested corner p{precision}").all()


def test_nested_launch_shapes_device_patches_and_errors(P, O, fields):
    """Patch data in device memory, several launch shapes (corner records and
    linear gathers), and the argument checks."""
    import torch
    base, patches = fields
    b, ps, G = _grid_pair(O, base, patches, np.float32)
    inj = W.make_injection(400)
    dev = [dict(q, data=torch.as_tensor(q["data"], device="cuda:0")) for q in ps]
    results = []
    for launch in (dict(block=128, blocks_per_cu=0, refill=4, layout=1),
                   dict(block=256, blocks_per_cu=2, refill=32, layout=0)):
        ctx = make_ctx(P, W, b, W.make_tables(), P.MIX)
        ctx.set_field_patches(dev)
        ctx.set_launch(**launch)
        say(f"nested launch {launch}")
        ctx.inject(inj)
        assert ctx.propagate()
        results.append(P.sort_finished(ctx.read_finished()))
        ctx.close()
    fo, _, _, _ = O.propagate(O.config_for(W, precision=O.MIX), G, O.TablesRef(W.make_tables()),
                              inj)
    for r in results:
        assert compare_records(r, fo, "nested launch").all()
    ctx = make_ctx(P, W, b, W.make_tables(), P.MIX)
    bad = [dict(ps[0], refine=3), dict(ps[0], offset=(-1, 0, 0)),
           dict(ps[0], offset=(20, 4, 4))]                   # sticks out of the period
    for q in bad:
        with pytest.raises(P.CrpError):
            ctx.set_field_patches([q])
    with pytest.raises(P.CrpError):
        ctx.set_field_patches(ps + ps[:2])                   # more than 4
    ctx.set_field_patches(ps)
    ctx.set_field_grid(b, W.spacing_m)                       # a new base grid drops them
    pos = np.random.default_rng(2).uniform(0, 32, (1000, 3)) * W.spacing_m
    assert np.array_equal(ctx.eval_field(pos, 0),
                          O.eval_field(O.GridRef(b, W.spacing_m), pos, O.FP64))
    ctx.close()


def test_nested_trajectory_points(P, O, fields):
    """Per-step output on the multi-resolution grid from corner records."""
    base, patches = fields
    b, ps, G = _grid_pair(O, base, patches, np.float32)
    inj = W.make_injection(300)
    ctx = make_ctx(P, W, b, W.make_tables(), P.MIX, traj_every=2, traj_ids=1 << 30,
                   traj_capacity=1 << 20)
    ctx.set_field_patches(ps)
    ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=P.LAYOUT_CORNER)
    say("nested trajectory points")
    ctx.inject(inj)
    assert ctx.propagate()
    tg = P.sort_traj(ctx.read_trajectory())
    ctx.close()
    cfg = O.config_for(W, precision=O.MIX, traj_every=2, traj_ids=1 << 30)
    _, _, _, to = O.propagate_traj(cfg, G, O.TablesRef(W.make_tables()), inj, 1 << 20)
    to = O.sort_traj(to)
    assert len(tg["id"]) == len(to["id"])
    for k in to:
        assert np.array_equal(tg[k], to[k]), k
