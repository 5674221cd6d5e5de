"""Pins of the oracle's precision form at its rounding points.

The precision form is defined by where it rounds: the field's trilinear
weights and sums in FP32 after the cell offset is found in FP64; the
Cash-Karp stage increments G_i = (h u_i, (h kappa)(u_i x B(x_i))) with h and
h kappa formed in FP64 and rounded once to FP32; FP32 stage sums, 5th-order
increment, direction and error norm; FP64 positions that receive each FP32
offset.  The functions below take those steps one numpy float32 (or float64)
scalar operation at a time, in the order the definition gives them, and the
oracle's C implementation must agree with them bit for bit.  A variant that
keeps the sums in FP64 and rounds once at the end (a plausible slip) is shown
to differ from both, so these pins distinguish where the rounding happens, not
only the mathematics.
"""
import math

import numpy as np
import pytest

import crp_inputs as I

f32 = np.float32
f64 = np.float64
C_LIGHT = 299792458.0

# Cash-Karp tableau (Cash & Karp 1990), each rational rounded once to FP64.
CK_A = [[], [1 / 5], [3 / 40, 9 / 40], [3 / 10, -9 / 10, 6 / 5],
        [-11 / 54, 5 / 2, -70 / 27, 35 / 27],
        [1631 / 55296, 175 / 512, 575 / 13824, 44275 / 110592, 253 / 4096]]
CK_B = [37 / 378, 0.0, 250 / 621, 125 / 594, 0.0, 512 / 1771]
CK_E = [-277 / 64512, 0.0, 6925 / 370944, -6925 / 202752, -277 / 14336, 277 / 7084]


def cell_axis(p, n, spacing):
    """FP64 cell lookup on one axis of a periodic vertex grid (origin 0)."""
    inv = f64(1.0) / f64(spacing)
    f = f64(p) * inv
    fl = math.floor(f)
    i0 = int(fl) % n
    return i0, (i0 + 1) % n, f64(f - fl)


def field_mix_np(g, spacing, p, accumulate_fp64=False):
    """FP32 trilinear interpolation: t rounded to FP32, weights (wx wy) wz and
    corner sums in FP32 in the order c = dx + 2 dy + 4 dz."""
    n = g.shape[:3]
    ax = [cell_axis(p[a], n[a], spacing) for a in range(3)]
    w = []
    for a in range(3):
        tf = f32(ax[a][2])
        w.append((f32(1.0) - tf, tf))
    B = [None, None, None]
    for c in range(8):
        d = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
        wt = (w[0][d[0]] * w[1][d[1]]) * w[2][d[2]]
        idx = tuple(ax[a][d[a]] for a in range(3))
        for q in range(3):
            v = f32(g[idx + (q,)])
            term = f64(wt) * f64(v) if accumulate_fp64 else wt * v
            B[q] = term if c == 0 else B[q] + term
    return [f32(b) for b in B]


def cross32(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def ck_attempt_mix_np(g, spacing, x, u, kappa, h, accumulate_fp64=False):
    """One precision-form Cash-Karp attempt; returns (x5, u5, err)."""
    A = [[f32(a) for a in row] for row in CK_A]
    Bw = [f32(b) for b in CK_B]
    Ew = [f32(e) for e in CK_E]
    hf = f32(h)
    hk = f32(f64(h) * f64(kappa))
    x = [f64(v) for v in x]
    u32 = [f32(v) for v in u]

    def incr(xp, up):
        B = field_mix_np(g, spacing, xp)
        c = cross32(up, B)
        return [hf * up[0], hf * up[1], hf * up[2], hk * c[0], hk * c[1], hk * c[2]]

    def wsum(coef, terms):
        acc = None
        for cf, t in zip(coef, terms):
            term = f64(cf) * f64(t) if accumulate_fp64 else cf * t
            acc = term if acc is None else acc + term
        return f32(acc)

    G = [incr(x, u32)]
    for i in range(1, 6):
        s = [wsum(A[i], [G[j][q] for j in range(i)]) for q in range(6)]
        xs = [x[q] + f64(s[q]) for q in range(3)]
        us = [u32[q] + s[3 + q] for q in range(3)]
        G.append(incr(xs, us))
    bi, ei = (0, 2, 3, 5), (0, 2, 3, 4, 5)
    s5 = [wsum([Bw[j] for j in bi], [G[j][q] for j in bi]) for q in range(6)]
    x5 = [x[q] + f64(s5[q]) for q in range(3)]
    u5 = [f64(u32[q] + s5[3 + q]) for q in range(3)]
    e = [wsum([Ew[j] for j in ei], [G[j][3 + q] for j in ei]) for q in range(3)]
    err = f64(np.sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]))
    return np.array(x5), np.array(u5), err


@pytest.fixture(scope="module")
def grid32():
    w = I.W_SMALL
    return w.make_grid().astype(np.float32), w.spacing_m


def test_mix_field_rounding_points_bitwise(oracle_lib, grid32):
    O = oracle_lib
    g, sp = grid32
    rng = np.random.default_rng(21)
    p = (rng.random((400, 3)) * 3.0 - 1.0) * 32 * sp
    got = O.eval_field(O.GridRef(g, sp), p, O.MIX)
    ref = np.array([field_mix_np(g, sp, q) for q in p], np.float64)
    assert np.array_equal(got, ref)
    # rounding once after FP64 sums gives other bits on a good share of points
    once = np.array([field_mix_np(g, sp, q, accumulate_fp64=True) for q in p], np.float64)
    assert np.mean(np.any(once != got, axis=1)) > 0.2


def test_mix_attempt_rounding_points_bitwise(oracle_lib, grid32):
    O = oracle_lib
    g, sp = grid32
    G = O.GridRef(g, sp)
    rng = np.random.default_rng(22)
    differ = 0
    cases = 60
    for k in range(cases):
        x = rng.random(3) * 32 * sp
        u = I.isotropic(rng, 1)[0]
        E = 10 ** rng.uniform(18, 21)
        Z = int(rng.choice([1, 2, 7, 26]))
        kappa = Z * C_LIGHT / E
        h = 10 ** rng.uniform(-2, 0) * I.MPC_M
        x5, u5, err = O.ck_attempt(G, x, u, kappa, h, O.MIX)
        rx, ru, re = ck_attempt_mix_np(g, sp, x, u, kappa, h)
        assert np.array_equal(x5, rx), k
        assert np.array_equal(u5, ru), k
        assert err == re, k
        ox, ou, oe = ck_attempt_mix_np(g, sp, x, u, kappa, h, accumulate_fp64=True)
        differ += int(not (np.array_equal(ox, x5) and np.array_equal(ou, u5) and oe == err))
    assert differ > cases // 2
