"""Pins of the oracle's galactic lenses (section 4: PARSEC-style transformation
matrices per energy range, mapping directions at the border of the Galaxy to
directions observed at Earth), built from backtracked events.

Checks that do not restate the oracle: a field-free Galaxy gives the identity
lens exactly; construction against brute-force counting with explicit loops;
application against a dense numpy product; rows that sum to one; and lenses
that spread further from the diagonal at lower rigidity in the galactic field.
"""
import numpy as np
import pytest

import crp_inputs as I
from oracle import lens as LN
from oracle import observables as OB

KPC = I.KPC_M


def _backtrack(O, model, n, E=None, Z=None, seed=707, renormalize=1):
    w = I.W_GALBACK
    inj = I.inject_galactic(n, seed)
    if E is not None:
        inj.E = np.full(n, E)
    if Z is not None:
        inj.Z = np.full(n, Z, np.int32)
        inj.A = np.full(n, max(1, 2 * Z - (Z == 1)), np.int32)
    cfg = O.config_for(w, renormalize=renormalize)
    fin, _, cnt, _ = O.propagate(cfg, O.AnalyticRef(model), O.TablesRef(w.make_tables()), inj,
                                 nthreads=4)
    return fin, cnt


def test_field_free_lens_is_the_identity(oracle_lib):
    O = oracle_lib
    zero = {k: (0.0 if k.startswith("b_") else v) for k, v in I.GALACTIC_FIELD.items()}
    fin, cnt = _backtrack(O, zero, 3000, renormalize=0)
    assert cnt["boundary"] == 3000
    assert np.array_equal(fin["u"], fin["u0"])          # straight lines, no renormalisation
    sp = LN.spec([1e16, 1e18, 1e19, 1e21], sky_n=4)
    L = LN.build(sp, fin)
    rows = np.repeat(np.arange(len(L["rowptr"]) - 1), np.diff(L["rowptr"]))
    assert np.all(L["col"] == rows % L["npix"])
    assert np.all(L["val"] == 1.0)
    assert int(L["count"].sum()) == 3000


def _records(n, seed):
    rng = np.random.default_rng(seed)
    return dict(status=rng.choice([2, 4, 4, 4], n).astype(np.int32),
                Z=rng.choice([1, 2, 7, 26], n).astype(np.int32),
                E0=10.0 ** rng.uniform(17.5, 20.5, n),
                u0=rng.standard_normal((n, 3)), u=rng.standard_normal((n, 3)))


def test_build_matches_brute_force_counting():
    from test_oracle_observables import _pixel_loop
    fin = _records(4000, 3)
    edges = np.array([1e17, 1e18, 3e18, 1e19, 1e20])
    sp = LN.spec(edges, sky_n=2)
    L = LN.build(sp, fin)
    npix = 24
    pi, pj = _pixel_loop(fin["u0"], 2), _pixel_loop(fin["u"], 2)
    counts = {}
    for k in range(len(fin["E0"])):
        if fin["status"][k] != 4:
            continue
        R = fin["E0"][k] / fin["Z"][k]
        rb = [b for b in range(len(edges) - 1) if edges[b] <= R < edges[b + 1]]
        if not rb:
            continue
        key = (rb[0] * npix + pi[k], pj[k])
        counts[key] = counts.get(key, 0) + 1
    dense = np.zeros((4 * npix, npix))
    for (row, col), c in counts.items():
        dense[row, col] = c
    tot = dense.sum(axis=1)
    nz = tot > 0
    dense[nz] /= tot[nz, None]
    got = np.zeros_like(dense)
    for row in range(4 * npix):
        s, e = L["rowptr"][row], L["rowptr"][row + 1]
        assert np.all(np.diff(L["col"][s:e]) > 0)      # increasing columns
        got[row, L["col"][s:e]] = L["val"][s:e]
    assert np.array_equal(got, dense)
    assert int(L["count"].sum()) == sum(counts.values())


def test_apply_matches_dense_product_and_rows_sum_to_one():
    fin = _records(20000, 5)
    sp = LN.spec([1e17, 1e18, 1e19, 1e21], sky_n=3)
    L = LN.build(sp, fin)
    npix, nr = L["npix"], L["n_r"]
    dense = np.zeros((nr * npix, npix))
    rows = np.repeat(np.arange(nr * npix), np.diff(L["rowptr"]))
    dense[rows, L["col"]] = L["val"]
    sums = dense.sum(axis=1)
    filled = np.diff(L["rowptr"]) > 0
    assert np.all(np.abs(sums[filled] - 1.0) < 1e-14) and np.all(sums[~filled] == 0)
    x = np.random.default_rng(6).uniform(0.0, 2.0, (5, nr, npix))
    y = LN.apply(L, x)
    for r in range(nr):
        ref = x[:, r, :] @ dense[r * npix:(r + 1) * npix].T
        assert np.allclose(y[:, r, :], ref, rtol=1e-14, atol=1e-15)
    # an isotropic border flux is seen isotropic from every filled direction
    y1 = LN.apply(L, np.ones((1, nr, npix)))
    assert np.allclose(y1[0].ravel()[filled], 1.0, rtol=1e-14)


def test_lens_spreads_more_at_lower_rigidity(oracle_lib):
    """Protons backtracked through the galactic field: the mean angle between
    the Earth and border pixel centres grows as the rigidity falls."""
    O = oracle_lib
    n = 4
    c = np.array([[[(2 * a + 1) / n - 1, (2 * b + 1) / n - 1] for b in range(n)]
                  for a in range(n)]).reshape(-1, 2)
    centres = []
    for face in range(6):
        m, sign = face // 2, (-1.0 if face % 2 else 1.0)
        p, q = [a for a in range(3) if a != m]
        v = np.zeros((n * n, 3))
        v[:, m] = sign
        v[:, p], v[:, q] = c[:, 0], c[:, 1]
        centres.append(v / np.linalg.norm(v, axis=1)[:, None])
    centres = np.concatenate(centres)
    spreads = []
    for E in (3e18, 1e19, 1e20):
        fin, cnt = _backtrack(O, I.GALACTIC_FIELD, 1500, E=E, Z=1, seed=11)
        L = LN.build(LN.spec([1e18, 1e21], sky_n=n), fin)
        rows = np.repeat(np.arange(len(L["rowptr"]) - 1), np.diff(L["rowptr"]))
        cosang = np.clip((centres[rows] * centres[L["col"]]).sum(1), -1, 1)
        spreads.append(float(np.sum(L["count"] * np.arccos(cosang)) / L["count"].sum()))
    assert spreads[0] > spreads[1] > spreads[2]
