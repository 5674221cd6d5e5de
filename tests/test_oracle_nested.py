"""Pins of the oracle's multi-resolution grid (section 4: multi-resolution
grids for fast access to precomputed fields): refinement patches with level
selection on top of the periodic base grid.

The checks use fields whose values are known without the oracle: a linear
field (which trilinear interpolation reproduces exactly on every level, so a
wrong patch origin, refinement or stride shows up as a wrong value), constant
patches whose containing region is worked out with plain interval tests,
periodic images on a grid with exactly representable coordinates, and a
propagation through a field-free patch inside a uniform field, which must be
a straight line there.
"""
import numpy as np
import pytest

import crp_inputs as I

M = np.array([[0.3, -1.1, 0.7], [2.0, 0.1, -0.4], [-0.6, 0.9, 1.3]]) * 1e-13
b = np.array([0.5, -0.2, 0.8]) * 1e-13


def linear(x):
    return x @ M.T + b


def vertices(n, origin, h):
    i = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), axis=-1)
    return origin + i * h


def test_linear_field_on_every_level(oracle_lib):
    O = oracle_lib
    n, h = 16, 2.0
    base = linear(vertices((n, n, n), 0.0, h))
    specs = [((3, 4, 2), 2, (13, 11, 15)), ((6, 6, 5), 4, (17, 9, 13)),
             ((8, 7, 6), 8, (9, 9, 9))]
    patches = []
    for off, ref, dims in specs:
        org = np.array(off) * h
        patches.append(dict(data=linear(vertices(dims, org, h / ref)), offset=off, refine=ref))
    g = O.GridRef(base, h, patches=patches)
    rng = np.random.default_rng(3)
    # inside one period, away from the periodic wrap of the last base cell
    pts = rng.uniform(0.0, (n - 1) * h, (20000, 3))
    for mode, tol in ((O.FP64, 1e-13), (O.MIX, 2e-6)):
        B = O.eval_field(g, pts, mode)
        ref = linear(pts)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(B - ref)) < tol * scale, mode


def _expected_level(pts, specs, n, h):
    """Last patch whose half-open box [off h, (off + (dims - 1)/ref) h) holds the
    point (taken modulo the period n h), else -1."""
    w = np.mod(pts, n * h)
    lev = np.full(len(pts), -1)
    for k, (off, ref, dims) in enumerate(specs):
        lo = np.array(off, float) * h
        hi = lo + (np.array(dims) - 1) / ref * h
        inside = np.all((w >= lo) & (w < hi), axis=1)
        lev[inside] = k
    return lev


def test_level_selection_constant_patches(oracle_lib):
    O = oracle_lib
    n, h = 12, 1.0
    specs = [((2, 2, 2), 2, (9, 9, 9)), ((3, 3, 3), 4, (5, 5, 5)), ((5, 1, 4), 2, (7, 11, 5))]
    patches = [dict(data=np.full(d + (3,), float(k + 1)) * np.array([1.0, 0, 0]), offset=o,
                    refine=r) for k, (o, r, d) in enumerate(specs)]
    g = O.GridRef(np.zeros((n, n, n, 3)), h, patches=patches)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-2 * n * h, 3 * n * h, (30000, 3))
    # exact faces: the lower face of a patch belongs to it, the upper does not
    faces = np.array([[2.0, 3.0, 3.0], [6.0, 3.0, 3.0], [5.9, 3.0, 3.0], [3.0, 3.0, 3.0],
                      [4.0, 3.5, 3.5], [3.999, 3.5, 3.5], [5.0, 1.0, 4.0], [8.0, 6.0, 6.0]])
    pts = np.concatenate([faces, faces + n * h, faces - 2 * n * h, pts])
    B = O.eval_field(g, pts, O.FP64)
    lev = _expected_level(pts, specs, n, h)
    # weights of a constant field sum to 1 up to rounding
    assert np.max(np.abs(B[:, 0] - (lev + 1))) < 1e-14 * 4
    assert np.all(B[:, 1:] == 0.0)
    assert len(np.unique(lev)) == 4


def test_periodic_images_are_bitwise_equal(oracle_lib):
    O = oracle_lib
    n, h = 8, 1.0
    rng = np.random.default_rng(8)
    base = rng.standard_normal((n, n, n, 3))
    patches = [dict(data=rng.standard_normal((7, 9, 5, 3)), offset=(1, 2, 3), refine=2)]
    g = O.GridRef(base, h, patches=patches)
    # dyadic coordinates: every shift by a period is exact
    pts = np.round(rng.uniform(0, n, (5000, 3)) * 1024) / 1024
    ref = O.eval_field(g, pts, O.FP64)
    for k in (-3, 1, 2):
        for ax in range(3):
            q = pts.copy()
            q[:, ax] += k * n * h
            assert np.array_equal(O.eval_field(g, q, O.FP64), ref)


def test_field_free_patch_is_crossed_in_a_straight_line(oracle_lib):
    """Uniform base field; a patch with zero field.  Trajectory segments well
    inside the patch are straight, segments outside curve with R = E/(c B)."""
    O = oracle_lib
    n, h = 8, 1.0 * I.MPC_M
    B0 = 1e-12
    base = np.zeros((n, n, n, 3))
    base[..., 2] = B0
    patches = [dict(data=np.zeros((17, 17, 17, 3)), offset=(2, 2, 2), refine=4)]  # [2, 6) Mpc
    g = O.GridRef(base, h, patches=patches)
    t = O.TablesRef(I.tables_constant())
    m = 6
    E = np.full(m, 2e20)                                  # R = 0.65 Mpc in B0
    ang = np.linspace(0.2, 1.2, m)
    d = np.stack([np.cos(ang), np.sin(ang), np.zeros(m)], axis=1)
    start = np.tile([4.0 * I.MPC_M, 4.0 * I.MPC_M, 4.0 * I.MPC_M], (m, 1))
    inj = I.Injection(np.arange(m, dtype=np.uint32), np.ones(m, np.int32), np.ones(m, np.int32),
                      E, start, d, np.full(m, 6 * I.MPC_M))
    hmax = 0.05 * I.MPC_M
    cfg = O.make_config(tol=1e-8, hmin=1e-3 * I.MPC_M, hmax=hmax, e_floor=0.0, traj_every=1,
                        traj_ids=m)
    _, _, _, tr = O.propagate_traj(cfg, g, t, inj, 1 << 20)
    tr = O.sort_traj(tr)
    lo, hi = 2 * I.MPC_M + 2 * hmax, 6 * I.MPC_M - 2 * hmax
    for k in range(m):
        x = tr["x"][tr["id"] == k]
        deep = np.all((x > lo) & (x < hi), axis=1)
        seg = np.diff(x, axis=0)[deep[:-1] & deep[1:]]
        assert len(seg) > 10
        u = seg / np.linalg.norm(seg, axis=1)[:, None]
        assert np.max(np.linalg.norm(u - d[k], axis=1)) < 1e-9
        # outside the patch (beyond one step of it) the path bends
        far = np.any((x < 2 * I.MPC_M - 2 * hmax) | (x > 6 * I.MPC_M + 2 * hmax), axis=1)
        seg2 = np.diff(x, axis=0)[far[:-1] & far[1:]]
        assert len(seg2) > 2
        u2 = seg2 / np.linalg.norm(seg2, axis=1)[:, None]
        assert np.max(np.linalg.norm(np.diff(u2, axis=0), axis=1)) > 1e-3
