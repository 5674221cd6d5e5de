"""Observables of finished candidates -- TEST INFRASTRUCTURE.

The application of the paper's section 5 (Fig. 3) reduces the detected
candidates to three observables: the energy spectrum, the mean deflection
(the angle between the initial and the observed direction) against energy,
and sky maps of arrival directions.  This module defines them in plain numpy,
as the reference for the GPU reduction of the same records.  Only tests/ and
bench.py's CPU-baseline leg may use it.

Definitions (the paper fixes the observables, not their binning; these are
this implementation's choices):

* a record takes part if bit `status` of `status_mask` is set;
* energy bin e: e_edges[e] <= E < e_edges[e + 1]; mass group g:
  a_edges[g] <= A < a_edges[g + 1]; a record outside either range (or with a
  zero sky direction) is counted in `outside` only;
* deflection: for unit vectors a = u/|u| and b = u0/|u0| the angle
  2 atan2(|a - b|, |a + b|) (accurate at every angle, unlike acos of the dot
  product); summed per bin in fixed point, floor(angle * 2^32), so that sums
  do not depend on the order of the records;
* weight: (E0 / e_ref)^gamma, the source-spectrum reweighting of the paper's
  application (injection E^-1 shown as E^-2.5: gamma = -1.5), summed per bin;
* sky map: the direction v = sky_sign * u on a cube map of 6 faces with
  sky_n x sky_n pixels each.  Face 2m + (v_m < 0) for the axis m of largest
  |v_m| (the lowest such axis on ties); on it the other two components, in
  axis order, give s = v_p / |v_m| and t = v_q / |v_m| in [-1, 1], and the
  pixel (i, j) = (floor(((s + 1) / 2) n), floor(((t + 1) / 2) n)) clamped to
  n - 1; index ((face * n) + i) * n + j.
"""
from __future__ import annotations

import numpy as np

DEFL_SCALE = 2.0 ** 32        # fixed-point unit of the deflection sums: 2^-32 rad


def spec(e_edges, a_edges=(1, 57), status_mask=1 << 1, sky_n=0, sky_sign=-1.0, e_ref=1e18,
         gamma=0.0):
    """An observable specification (status bit 1 = observed)."""
    return dict(e_edges=np.asarray(e_edges, np.float64), a_edges=np.asarray(a_edges, np.int32),
                status_mask=int(status_mask), sky_n=int(sky_n), sky_sign=float(sky_sign),
                e_ref=float(e_ref), gamma=float(gamma))


def unit(v):
    v = np.asarray(v, np.float64)
    n = np.sqrt((v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2])
    return v / n[:, None]


def deflection(u0, u):
    """Angle between u0 and u, radians (half-angle form)."""
    a = unit(u)
    b = unit(u0)
    d = a - b
    s = a + b
    nd = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    ns = np.sqrt((s[:, 0] * s[:, 0] + s[:, 1] * s[:, 1]) + s[:, 2] * s[:, 2])
    return 2.0 * np.arctan2(nd, ns)


def deflection_fixed(u0, u):
    return np.floor(deflection(u0, u) * DEFL_SCALE).astype(np.uint64)


def cube_pixel(v, n):
    """Cube-map pixel of directions v (rows); -1 for a zero vector."""
    v = np.asarray(v, np.float64)
    av = np.abs(v)
    m = np.argmax(av, axis=1)                      # first maximum on ties
    rows = np.arange(len(v))
    vm = v[rows, m]
    big = av[rows, m]
    other = np.array([[1, 2], [0, 2], [0, 1]])[m]
    s = v[rows, other[:, 0]] / np.where(big > 0, big, 1.0)
    t = v[rows, other[:, 1]] / np.where(big > 0, big, 1.0)
    i = np.minimum(np.floor(((s + 1.0) * 0.5) * n), n - 1).astype(np.int64)
    j = np.minimum(np.floor(((t + 1.0) * 0.5) * n), n - 1).astype(np.int64)
    face = 2 * m + (vm < 0)
    pix = (face * n + i) * n + j
    return np.where(big > 0, pix, -1)


def observe(sp, fin):
    """Reduce finished records (dict of arrays: status, A, E, E0, u, u0) to
    (counts[g][e] u64, wsum[g][e] f64, defl[g][e] u64 fixed point,
    sky[g][e][6 n^2] u64, outside)."""
    ee, ae = sp["e_edges"], sp["a_edges"]
    ne, ng, n = len(ee) - 1, len(ae) - 1, sp["sky_n"]
    counts = np.zeros((ng, ne), np.uint64)
    wsum = np.zeros((ng, ne), np.float64)
    defl = np.zeros((ng, ne), np.uint64)
    sky = np.zeros((ng, ne, 6 * n * n), np.uint64)
    status = np.asarray(fin["status"]).astype(np.int64)
    sel = ((sp["status_mask"] >> status) & 1) == 1
    E = fin["E"][sel]
    A = fin["A"][sel].astype(np.int64)
    u = fin["u"][sel]
    e = np.searchsorted(ee, E, side="right") - 1            # ee[e] <= E < ee[e+1]
    g = np.searchsorted(ae, A, side="right") - 1
    ok = (e >= 0) & (e < ne) & (g >= 0) & (g < ng) & ~np.isnan(E)
    pix = None
    if n > 0:
        pix = cube_pixel(sp["sky_sign"] * u, n)
        ok &= pix >= 0
    outside = int(np.count_nonzero(~ok))
    e, g = e[ok], g[ok]
    w = np.power(fin["E0"][sel][ok] / sp["e_ref"], sp["gamma"])
    dfx = deflection_fixed(fin["u0"][sel][ok], u[ok])
    np.add.at(counts, (g, e), np.uint64(1))
    np.add.at(wsum, (g, e), w)
    np.add.at(defl, (g, e), dfx)
    if n > 0:
        np.add.at(sky, (g, e, pix[ok]), np.uint64(1))
    return dict(counts=counts, wsum=wsum, defl=defl, sky=sky, outside=outside)


def mean_deflection(obs):
    """Mean deflection per bin, radians (NaN where empty)."""
    c = obs["counts"].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return obs["defl"].astype(np.float64) / DEFL_SCALE / c
