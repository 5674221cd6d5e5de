"""GPU parity of the galactic-propagation path (section 4): the analytic field,
backtracking (charge -Z, reversed direction) and the spherical boundary,
against the oracle on the same seeded events.

The oracle evaluates the analytic field term by term (five divisions); the
kernel forms the toroidal factor over the common denominator of its disk and
halo parts and uses one reciprocal of D (two divisions).  Both are rational
(no libm), so they differ by a few roundings: the field is compared within a
bound derived from those roundings.  Propagation: integer bookkeeping exact,
energies within 1e-6, and the states after 100 cycles within 1e-9 of
max(L, |x|) for every event; over the whole path (up to 100 kpc, thousands of
gyrations of a low-rigidity nucleus in the disk field, where the motion is
chaotic and an ulp of field difference grows) nearly all final positions meet
that bar and the few that do not are counted."""
import numpy as np
import pytest

import crp_inputs as I
from parity_helpers import (CNT_KEYS, compare_counts, compare_records,
                            compare_records_chaotic, say)

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


def make(P, precision, **kw):
    prm = P.params_for(W, precision, queue_capacity=1 << 16, neutral_capacity=1 << 16, **kw)
    ctx = P.Context(prm)
    ctx.set_field_analytic(I.GALACTIC_FIELD)
    ctx.set_tables(W.make_tables())
    return ctx


def analytic_rounding_scale(m, pos):
    """Per component, the sum of the magnitudes of the terms that the two
    evaluation orders round differently: |y| (|g_disk| + |g_halo|) + |x| |q| for
    B_x (x and y swapped for B_y) and |b_x / D| + |b_x r^2 / (r_x^2 D^2)| for B_z.
    Either order rounds each of these terms at most a few times (divisions,
    the reciprocal and its square, the products with x and y, the sums), so
    the two results differ by at most ~8 units of 2^-53 of this scale; the
    test allows 16."""
    d = pos - np.asarray(m["center"])
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    r2 = x * x + y * y
    gd = np.abs(m["b_disk"] / (m["r_disk"] * (1 + r2 / m["r_disk"] ** 2)
                               * (1 + z * z / m["h_disk"] ** 2)))
    gh = np.abs(m["b_halo"] * (z / m["h_halo"])
                / (m["r_halo"] * (1 + r2 / m["r_halo"] ** 2) * (1 + z * z / m["h_halo"] ** 2) ** 2))
    D = 1 + r2 / m["r_x"] ** 2 + z * z / m["h_x"] ** 2
    q = np.abs(m["b_x"] * z / m["h_x"] ** 2 / D ** 2)
    sx = np.abs(y) * (gd + gh) + np.abs(x) * q
    sy = np.abs(x) * (gd + gh) + np.abs(y) * q
    sz = np.abs(m["b_x"] / D) + np.abs(m["b_x"] * r2 / m["r_x"] ** 2 / D ** 2)
    return np.stack([sx, sy, sz], axis=1)


def test_analytic_field_within_rounding_bound(P, O):
    ctx = make(P, P.FP64)
    rng = np.random.default_rng(11)
    pos = rng.uniform(-25, 25, (50_000, 3)) * I.KPC_M
    pos[:3] = 0.0                                          # the centre itself
    pos[3:1000, 2] *= 1e-3                                 # near the disk plane
    say("analytic field")
    got = ctx.eval_field(pos, P.EVAL_ANALYTIC)
    ref = O.eval_field(O.AnalyticRef(I.GALACTIC_FIELD), pos, O.FP64)
    bound = 16 * 2.0 ** -53 * analytic_rounding_scale(I.GALACTIC_FIELD, pos)
    err = np.abs(got - ref)
    say(f"analytic field: max |dB| / bound {np.max(err / np.maximum(bound, 1e-300)):.3f}, "
        f"bitwise equal {np.mean(np.all(got == ref, axis=1)):.3f}")
    assert np.all(err <= bound)
    ctx.close()


def _after_cycles(P, O, inj, precision, cycles, **kw):
    """GPU and oracle states after `cycles` cycles, all at the full bar."""
    ctx = make(P, precision, **kw)
    ctx.inject(inj)
    assert not ctx.propagate(cycles)
    allg = ctx.read_finished()
    pend = ctx.peek_pending()
    ctx.close()
    allg = {k: np.concatenate([allg[k], pend[k]]) for k in allg}
    fo, _, _, _ = O.propagate(O.config_for(W, precision=precision, max_cycles=cycles, **kw),
                              O.AnalyticRef(I.GALACTIC_FIELD), O.TablesRef(W.make_tables()), inj,
                              nthreads=0)
    compare_records(allg, fo, f"after {cycles} cycles p{precision}")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mix"])
def test_backtracking_parity(P, O, precision):
    inj = W.make_injection(3000)
    ctx = make(P, precision)
    say(f"galactic backtracking precision={precision}")
    ctx.inject(inj)
    assert ctx.propagate()
    fg, cg = ctx.read_finished(), ctx.counts()
    ctx.close()
    fo, _, co, _ = O.propagate(O.config_for(W, precision=precision),
                               O.AnalyticRef(I.GALACTIC_FIELD), O.TablesRef(W.make_tables()),
                               inj, nthreads=0)
    compare_counts(cg, co, "galactic")
    assert cg["boundary"] == co["boundary"] and co["boundary"] > 2000
    assert co["max_traj"] > 0                    # some low-rigidity nuclei stay confined
    compare_records_chaotic(fg, fo, f"galactic p{precision}", min_frac=0.99)
    _after_cycles(P, O, inj, precision, 100)


def test_forward_tracking_and_launch_shapes(P, O):
    """Charge +Z from the observer outwards, in two launch shapes."""
    inj = W.make_injection(1000)
    results = []
    for launch in (dict(block=128, blocks_per_cu=0, refill=4),
                   dict(block=256, blocks_per_cu=1, refill=64)):
        ctx = make(P, P.FP64, charge_sign=1)
        ctx.set_launch(**launch)
        say(f"forward tracking launch={launch}")
        ctx.inject(inj)
        assert ctx.propagate()
        results.append((P.sort_finished(ctx.read_finished()), ctx.counts()))
        ctx.close()
    fo, _, co, _ = O.propagate(O.config_for(W, charge_sign=1), O.AnalyticRef(I.GALACTIC_FIELD),
                               O.TablesRef(W.make_tables()), inj)
    for fg, cg in results:
        compare_counts(cg, co, "forward")
        compare_records_chaotic(fg, fo, "forward", min_frac=0.99)
    _after_cycles(P, O, inj, P.FP64, 100, charge_sign=1)
    for k in results[0][0]:
        assert np.array_equal(results[0][0][k], results[1][0][k])
    for k in CNT_KEYS:
        assert results[0][1][k] == results[1][1][k]


def test_backtracking_trajectory_points(P, O):
    """Per-step output of backtracked paths through the analytic field: the
    points of the first 40 events, every third step and the last; integer
    fields exact, energies within 1e-6, positions and lengths within 1e-9 of
    max(L, |x|) for every point of the first 100 steps and nearly all later
    ones (the chaotic paths excepted)."""
    inj = W.make_injection(500)
    ctx = make(P, P.FP64, traj_every=3, traj_ids=40, traj_capacity=1 << 20)
    say("galactic trajectory points")
    ctx.inject(inj)
    assert ctx.propagate()
    tg = P.sort_traj(ctx.read_trajectory())
    cg = ctx.counts()
    ctx.close()
    cfg = O.config_for(W, traj_every=3, traj_ids=40)
    _, _, _, to = O.propagate_traj(cfg, O.AnalyticRef(I.GALACTIC_FIELD),
                                   O.TablesRef(W.make_tables()), inj, 1 << 20)
    to = O.sort_traj(to)
    assert cg["traj_points"] == len(to["id"]) > 1000
    for k in ("id", "lineage", "n", "A"):
        assert np.array_equal(tg[k], to[k]), k
    scale = np.maximum(np.maximum(to["L"], np.linalg.norm(to["x"], axis=1)), 1.0)
    ok = (np.linalg.norm(tg["x"] - to["x"], axis=1) <= 1e-9 * scale) & \
        (np.abs(tg["L"] - to["L"]) <= 1e-9 * scale)
    say(f"trajectory points within 1e-9: {ok.sum()} of {len(ok)}")
    # every point of the first 100 accepted steps meets the bar; over the whole
    # (possibly chaotic) path nearly every point does
    assert np.all(ok[tg["n"] <= 100])
    assert ok.mean() >= 0.95
    assert np.all(np.abs(tg["E"] / to["E"] - 1) <= 1e-6)
    # every path ends on or beyond the 20 kpc sphere or at its length limit
    last = np.r_[np.nonzero(np.diff(tg["id"].astype(np.int64)))[0], len(tg["id"]) - 1]
    r = np.linalg.norm(tg["x"][last], axis=1)
    assert np.all((r >= W.boundary_radius_m) | (tg["L"][last] >= W.lmax_m * (1 - 1e-12)))
