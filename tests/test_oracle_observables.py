"""Pins of the oracle's output modules and observables: per-step trajectory
output (section 3: output modules may record a candidate after every step)
and the reductions of the section 5 application (spectrum, mean deflection
against energy, sky maps).

Nothing here compares the oracle with a retyped copy of itself: trajectory
points are checked against the finished records and geometry (chord <= arc,
straight lines), the deflection against exact angles and the gyration angle
L / R of a uniform field, the cube map against the closed-form solid angle of
its pixels, and the reductions against brute-force loops that use other
formulas (acos of the dot product, linear scans).
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

import crp_inputs as I
from oracle import observables as OB

C = I.C_LIGHT


def uniform_grid(B, n=4):
    g = np.zeros((n, n, n, 3))
    g[...] = np.asarray(B, np.float64)
    return g


# ---------------------------------------------------------------------------
# Per-step trajectory output.
# ---------------------------------------------------------------------------
def _small_run(O, every, ids, cap=1 << 20, n=60, **kw):
    w = I.W_SMALL
    g = O.GridRef(w.make_grid(), w.spacing_m)
    t = O.TablesRef(w.make_tables())
    inj = w.make_injection(n)
    cfg = O.config_for(w, traj_every=every, traj_ids=ids, **kw)
    return O.propagate_traj(cfg, g, t, inj, cap, nthreads=4), (g, t, inj, w)


def test_every_step_output_ends_in_the_finished_record(oracle_lib):
    O = oracle_lib
    (fin, _, cnt, tr), _ = _small_run(O, 1, 1 << 30)
    fin = O.sort_finished(fin)
    tr = O.sort_traj(tr)
    assert cnt["traj_dropped"] == 0
    # one point per accepted step, numbered 1..nsteps
    assert len(tr["id"]) == int(fin["nsteps"].sum()) == cnt["steps"]
    starts = np.concatenate([[0], np.cumsum(fin["nsteps"])[:-1]]).astype(np.int64)
    for k in range(len(fin["id"])):
        s, e = starts[k], starts[k] + int(fin["nsteps"][k])
        assert np.all(tr["id"][s:e] == fin["id"][k])
        assert np.array_equal(tr["n"][s:e], np.arange(1, fin["nsteps"][k] + 1, dtype=np.uint32))
        # the last point is the finished state, bit for bit
        assert np.array_equal(tr["x"][e - 1], fin["x"][k])
        assert tr["E"][e - 1] == fin["E"][k] and tr["L"][e - 1] == fin["L"][k]
        # length grows; the chord between points does not exceed the arc
        # length by more than the per-step error the controller allows (tol)
        dL = np.diff(tr["L"][s:e])
        assert np.all(dL > 0)
        chord = np.linalg.norm(np.diff(tr["x"][s:e], axis=0), axis=1)
        assert np.all(chord <= dL * (1 + I.W_SMALL.tol))


def test_every_kth_step_is_a_subset_and_ids_limit(oracle_lib):
    O = oracle_lib
    (fin1, _, _, t1), _ = _small_run(O, 1, 1 << 30)
    (fin7, _, c7, t7), _ = _small_run(O, 7, 25)
    # recording does not change the propagation
    a, b = O.sort_finished(fin1), O.sort_finished(fin7)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    t1 = O.sort_traj(t1)
    t7 = O.sort_traj(t7)
    last = {int(i): int(n) for i, n in zip(a["id"], a["nsteps"])}
    keep = (t1["id"] < 25) & ((t1["n"] % 7 == 0) |
                              (t1["n"] == np.array([last[int(i)] for i in t1["id"]])))
    for k in t1:
        assert np.array_equal(t1[k][keep], t7[k]), k
    assert c7["traj_dropped"] == 0 and np.all(t7["id"] < 25)


def test_capacity_overflow_is_counted(oracle_lib):
    O = oracle_lib
    (_, _, call, tall), _ = _small_run(O, 1, 1 << 30, n=20)
    cap = len(tall["id"]) // 3
    (_, _, c, t), _ = _small_run(O, 1, 1 << 30, cap=cap, n=20)
    assert len(t["id"]) == cap and c["traj_dropped"] == len(tall["id"]) - cap


def test_straight_line_trajectory_points(oracle_lib):
    """No field: every recorded point lies on the injection ray at distance L."""
    O = oracle_lib
    g = O.GridRef(uniform_grid((0.0, 0.0, 0.0)), I.MPC_M)
    t = O.TablesRef(I.tables_constant())
    inj = I.inject_protons_fixed(16, 1e19, 5 * I.MPC_M, seed=3)
    cfg = O.make_config(hmin=10 * I.KPC_M, hmax=300 * I.KPC_M, traj_every=1, traj_ids=1 << 30)
    _, _, _, tr = O.propagate_traj(cfg, g, t, inj, 1 << 16)
    d = inj.dir[tr["id"]]
    assert np.max(np.linalg.norm(tr["x"] - tr["L"][:, None] * d, axis=1)) < 1e-9 * I.MPC_M


# ---------------------------------------------------------------------------
# Deflection angle.
# ---------------------------------------------------------------------------
def test_deflection_exact_angles():
    u0 = np.array([[1.0, 0, 0], [1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0]])
    u = np.array([[1.0, 0, 0], [0, 5.0, 0], [0, -1.0, 0], [0, 1.0, 0]])
    ang = OB.deflection(u0, u)
    assert ang[0] == 0.0
    assert ang[1] == pytest.approx(math.pi / 2, abs=4e-16)
    assert ang[2] == pytest.approx(math.pi, abs=4e-16)
    assert ang[3] == pytest.approx(math.pi / 2, abs=4e-16)
    # fixed point of a right angle: floor(pi / 2 * 2^32) from a 40-digit pi
    getcontext().prec = 60
    pi = Decimal("3.1415926535897932384626433832795028841971")
    assert int(OB.deflection_fixed(u0[1:2], u[1:2])[0]) == int(pi / 2 * Decimal(2 ** 32))
    assert int(OB.deflection_fixed(u0[:1], u[:1])[0]) == 0


def test_deflection_recovers_planar_angles():
    th = np.linspace(1e-9, math.pi - 1e-9, 4001)
    u0 = np.tile([0.6, 0.8, 0.0], (len(th), 1))
    perp = np.array([-0.8, 0.6, 0.0])
    u = 3.0 * (np.cos(th)[:, None] * u0 + np.sin(th)[:, None] * perp)
    assert np.max(np.abs(OB.deflection(u0, u) - th)) < 2e-15


def test_mean_deflection_of_uniform_field_gyration(oracle_lib):
    """Protons moving across a uniform field turn by L / R, R = E / (c B)."""
    O = oracle_lib
    B0 = 1e-12
    g = O.GridRef(uniform_grid((0.0, 0.0, B0)), I.MPC_M)
    t = O.TablesRef(I.tables_constant())
    n = 400
    rng = np.random.default_rng(9)
    E = 10.0 ** rng.uniform(19.0, 21.0, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    d = np.stack([np.cos(phi), np.sin(phi), np.zeros(n)], axis=1)
    L = 2.0 * I.MPC_M
    inj = I.Injection(np.arange(n, dtype=np.uint32), np.ones(n, np.int32), np.ones(n, np.int32),
                      E, np.zeros((n, 3)), d, np.full(n, L))
    cfg = O.make_config(tol=1e-8, hmin=1 * I.KPC_M, hmax=100 * I.KPC_M, e_floor=0.0)
    fin, _, _, _ = O.propagate(cfg, g, t, inj)
    fin = O.sort_finished(fin)
    edges = 10.0 ** np.linspace(19.0, 21.0, 5)
    sp = OB.spec(edges, status_mask=1 << O.MAX_TRAJ, gamma=0.0)
    obs = OB.observe(sp, fin)
    expect = L * C * B0 / fin["E"]                      # L / R per candidate
    e = np.searchsorted(edges, fin["E"], side="right") - 1
    want = np.array([expect[e == k].mean() for k in range(4)])
    got = OB.mean_deflection(obs)[0]
    assert np.allclose(got, want, rtol=1e-5)
    assert int(obs["counts"].sum()) == n and obs["outside"] == 0


# ---------------------------------------------------------------------------
# Cube-map sky pixels.
# ---------------------------------------------------------------------------
def _pixel_loop(v, n):
    """Brute force: explicit comparisons and a scan over the pixel edges."""
    out = []
    for x in v:
        m = 0
        for a in (1, 2):
            if abs(x[a]) > abs(x[m]):
                m = a
        if x[m] == 0:
            out.append(-1)
            continue
        face = 2 * m + (1 if x[m] < 0 else 0)
        p, q = [a for a in range(3) if a != m]
        coords = []
        for c in (x[p] / abs(x[m]), x[q] / abs(x[m])):
            k = 0
            while k < n - 1 and (c + 1.0) * 0.5 * n >= k + 1:
                k += 1
            coords.append(k)
        out.append((face * n + coords[0]) * n + coords[1])
    return np.array(out)


def test_cube_pixel_matches_brute_force_and_face_centres():
    rng = np.random.default_rng(5)
    v = rng.standard_normal((3000, 3))
    v[:20] = rng.integers(-2, 3, (20, 3))            # ties and zeros
    for n in (1, 3, 8):
        assert np.array_equal(OB.cube_pixel(v, n), _pixel_loop(v, n))
    c = OB.cube_pixel(np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1],
                                [0, 0, -1.0]]), 4)
    assert np.array_equal(c, [(f * 4 + 2) * 4 + 2 for f in range(6)])


def test_cube_pixel_solid_angles():
    """Isotropic directions fill each pixel in proportion to its solid angle,
    atan(st / sqrt(1 + s^2 + t^2)) differenced over its corners."""
    n = 4
    N = 2_000_000
    v = I.isotropic(np.random.default_rng(17), N)
    cnt = np.bincount(OB.cube_pixel(v, n), minlength=6 * n * n)
    edges = np.linspace(-1.0, 1.0, n + 1)
    F = lambda s, t: np.arctan(s * t / np.sqrt(1 + s * s + t * t))
    om = np.array([[F(edges[i + 1], edges[j + 1]) - F(edges[i], edges[j + 1]) -
                    F(edges[i + 1], edges[j]) + F(edges[i], edges[j]) for j in range(n)]
                   for i in range(n)]).ravel()
    assert abs(6 * om.sum() - 4 * math.pi) < 1e-12
    exp = N * np.tile(om, 6) / (4 * math.pi)
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert stats.chi2.sf(chi2, 6 * n * n - 1) > 1e-3


# ---------------------------------------------------------------------------
# The reductions.
# ---------------------------------------------------------------------------
def _records(n, seed):
    rng = np.random.default_rng(seed)
    return dict(status=rng.integers(0, 5, n).astype(np.int32),
                A=rng.choice([1, 4, 14, 56, 70], n).astype(np.int32),
                E=10.0 ** rng.uniform(17.5, 21.5, n),
                E0=10.0 ** rng.uniform(18.0, 21.0, n),
                u=rng.standard_normal((n, 3)) * rng.uniform(0.5, 2.0, (n, 1)),
                u0=I.isotropic(rng, n))


def test_observe_matches_brute_force_loops():
    fin = _records(3000, 21)
    edges = 10.0 ** np.linspace(18.0, 21.0, 7)
    sp = OB.spec(edges, a_edges=(1, 2, 15, 57), status_mask=(1 << 1) | (1 << 2), sky_n=3,
                 sky_sign=-1.0, e_ref=1e18, gamma=-1.5)
    obs = OB.observe(sp, fin)
    ng, ne = 3, 6
    counts = np.zeros((ng, ne), np.int64)
    wsum = np.zeros((ng, ne))
    ang = np.zeros((ng, ne))
    sky = np.zeros((ng, ne, 54), np.int64)
    outside = 0
    pix = _pixel_loop(-fin["u"], 3)
    for k in range(len(fin["E"])):
        if fin["status"][k] not in (1, 2):
            continue
        e = [i for i in range(ne) if edges[i] <= fin["E"][k] < edges[i + 1]]
        g = [i for i in range(ng) if sp["a_edges"][i] <= fin["A"][k] < sp["a_edges"][i + 1]]
        if not e or not g:
            outside += 1
            continue
        e, g = e[0], g[0]
        counts[g, e] += 1
        wsum[g, e] += math.pow(fin["E0"][k] / 1e18, -1.5)
        a = fin["u"][k] / math.sqrt(sum(fin["u"][k] ** 2))
        ang[g, e] += math.acos(max(-1.0, min(1.0, float(np.dot(a, fin["u0"][k])))))
        sky[g, e, pix[k]] += 1
    assert obs["outside"] == outside
    assert np.array_equal(obs["counts"], counts)
    assert np.array_equal(obs["sky"], sky)
    assert np.allclose(obs["wsum"], wsum, rtol=1e-13, atol=0)
    # acos of a rounded dot product is good to ~1e-8 rad near 0 and pi
    assert np.allclose(obs["defl"].astype(np.float64) / OB.DEFL_SCALE, ang, rtol=0,
                       atol=1e-7 * max(1, counts.max()))


def test_weights_of_exact_powers():
    """E0 = e_ref 4^k with gamma = -1.5 has weight 8^-k exactly."""
    n = 40
    k = np.arange(n) % 5
    fin = dict(status=np.ones(n, np.int32), A=np.ones(n, np.int32),
               E=np.full(n, 1e19), E0=1e18 * 4.0 ** k,
               u=np.tile([0, 0, 1.0], (n, 1)), u0=np.tile([0, 0, 1.0], (n, 1)))
    obs = OB.observe(OB.spec([1e18, 1e20], gamma=-1.5), fin)
    assert obs["wsum"][0, 0] == sum(8.0 ** -int(j) for j in k)
    assert obs["counts"][0, 0] == n and obs["defl"][0, 0] == 0
    assert np.array_equal(OB.observe(OB.spec([1e18, 1e20]), fin)["wsum"], [[float(n)]])
