"""Galactic lenses from backtracked events -- TEST INFRASTRUCTURE.

Section 4 describes the lensing technique of PARSEC: for each energy (here:
rigidity) range, a transformation matrix maps the directions of cosmic rays at
the border of the Galaxy to the directions observed at Earth.  This module
builds such matrices from the finished records of a backtracking run (the
antiparticle launched at Earth along the reversed arrival direction and
stopped at the galactic boundary, section 4) and applies them to maps of the
flux at the border, in plain numpy / scipy, as the reference for the GPU lens
kernels.  Only tests/ and bench.py's CPU-baseline leg may use it.

Definitions (this implementation's choices where the paper gives none):

* a record takes part if bit `status` of `status_mask` is set (normally the
  boundary status only) and its rigidity E0 / Z falls in a bin
  r_edges[r] <= E0 / Z < r_edges[r + 1];
* Earth pixel i: the cube-map pixel of the launch direction u0 (the arrival
  direction on the sky); border pixel j: the cube-map pixel of the final
  direction u (the direction the cosmic ray came from, seen at the border);
  the cube map of `observables.cube_pixel` with sky_n x sky_n pixels per face,
  Np = 6 sky_n^2;
* lens r: L_r[i, j] = c_r(i, j) / sum_j' c_r(i, j'), with c_r the number of
  records in bin r with pixels (i, j); rows without records are zero;
* the lenses are stored as one CSR matrix of n_r * Np rows (row r Np + i) and
  Np columns, entries of a row in increasing column order, values FP64;
* applying it to border maps x[m][r][j] gives y[m][r][i] = sum_j L_r[i, j]
  x[m][r][j], the flux observed at Earth.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse

from . import observables as OB


def spec(r_edges, sky_n, status_mask=1 << 4):
    return dict(r_edges=np.asarray(r_edges, np.float64), sky_n=int(sky_n),
                status_mask=int(status_mask))


def keys(sp, fin):
    """Per record: (bin r, Earth pixel i, border pixel j), or -1 where it takes
    no part."""
    n = sp["sky_n"]
    status = np.asarray(fin["status"]).astype(np.int64)
    sel = ((sp["status_mask"] >> status) & 1) == 1
    R = fin["E0"] / fin["Z"].astype(np.float64)
    r = np.searchsorted(sp["r_edges"], R, side="right") - 1
    nr = len(sp["r_edges"]) - 1
    i = OB.cube_pixel(fin["u0"], n)
    j = OB.cube_pixel(fin["u"], n)
    ok = sel & (r >= 0) & (r < nr) & (i >= 0) & (j >= 0) & ~np.isnan(R)
    return np.where(ok, r, -1), np.where(ok, i, -1), np.where(ok, j, -1)


def build(sp, fin):
    """CSR lens (rowptr int64 [n_r Np + 1], col int32, val float64, count int64
    per entry)."""
    n = sp["sky_n"]
    npix = 6 * n * n
    nr = len(sp["r_edges"]) - 1
    r, i, j = keys(sp, fin)
    ok = r >= 0
    key = (r[ok] * npix + i[ok]) * npix + j[ok]
    uk, cnt = np.unique(key, return_counts=True)       # sorted: by row, then column
    rows = uk // npix
    cols = (uk % npix).astype(np.int32)
    nrows = nr * npix
    rowcount = np.bincount(rows, weights=cnt, minlength=nrows).astype(np.int64)
    rowptr = np.zeros(nrows + 1, np.int64)
    rowptr[1:] = np.cumsum(np.bincount(rows, minlength=nrows))
    val = cnt.astype(np.float64) / rowcount[rows].astype(np.float64)
    return dict(rowptr=rowptr, col=cols, val=val, count=cnt.astype(np.int64), npix=npix,
                n_r=nr)


def apply(L, x):
    """x: [n_maps][n_r][Np] border maps -> y: [n_maps][n_r][Np] Earth maps."""
    A = sparse.csr_matrix((L["val"], L["col"], L["rowptr"]),
                          shape=(L["n_r"] * L["npix"], L["npix"]))
    x = np.asarray(x, np.float64)
    m = x.shape[0]
    y = np.zeros_like(x)
    npix = L["npix"]
    for r in range(L["n_r"]):
        Ar = A[r * npix:(r + 1) * npix]
        y[:, r, :] = (Ar @ x[:, r, :].T).T
    return y.reshape(m, L["n_r"], npix)
