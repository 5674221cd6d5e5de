"""The seeded synthetic inputs follow their stated recipes (they stand in for
the paper's workloads; both the oracle and the GPU path read them): equal
H/He/N/Fe fractions, an E^-2 spectrum on its range, isotropic directions,
source distances uniform on 1-1000 Mpc with the trajectory limit equal to the
distance, and the same arrays for the same seed."""
import numpy as np
from scipy import stats

import crp_inputs as I


def test_mixed_batch_recipe():
    inj = I.W_MIXED1024.make_injection(200_000)
    again = I.W_MIXED1024.make_injection(200_000)
    for k in ("id", "A", "Z", "E", "pos", "dir", "lmax"):
        assert np.array_equal(getattr(inj, k), getattr(again, k))       # seeded
    species = sorted(set(zip(inj.A.tolist(), inj.Z.tolist())))
    assert species == [(1, 1), (4, 2), (14, 7), (56, 26)]
    counts = np.bincount(np.searchsorted([1, 4, 14, 56], inj.A))
    assert counts.min() == counts.max() == 50_000                        # id mod 4
    assert inj.E.min() >= 1e18 and inj.E.max() <= 1e21
    # E^-2 on [e1, e2]: 1/E is uniform on [1/e2, 1/e1]
    v = (1.0 / inj.E - 1e-21) / (1e-18 - 1e-21)
    assert stats.kstest(v, "uniform").pvalue > 1e-3
    assert np.allclose(np.linalg.norm(inj.dir, axis=1), 1.0, atol=1e-15)
    assert np.all(np.abs(inj.dir.mean(axis=0)) < 0.01)                   # isotropic
    assert stats.kstest((inj.dir[:, 2] + 1.0) / 2.0, "uniform").pvalue > 1e-3
    assert np.all(inj.pos == 0.0) and np.all(inj.lmax == 100 * I.MPC_M)


def test_distance_batches_recipe():
    a = I.inject_distances(100_000, 404)
    b = I.inject_distances(100_000, 405, id0=100_000)
    assert not np.array_equal(a.E, b.E)                                  # seeds differ
    assert np.array_equal(b.id, np.arange(100_000, 200_000, dtype=np.uint32))
    d = np.linalg.norm(a.pos, axis=1)
    assert np.allclose(d, a.lmax, rtol=1e-12)                            # L_max = distance
    u = (a.lmax - I.MPC_M) / (999 * I.MPC_M)
    assert u.min() >= 0.0 and u.max() <= 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_nf_frequencies_narrow_band_takes_every_mode():
    """A band with fewer modes than features contributes all of them; the rest
    comes from the next shell; wide bands draw distinct in-band modes."""
    band = I.turbulence_modes(0, 2.0, 3.0, exclude_nyquist=False)
    F = I.nf_frequencies(nmin=2.0, nmax=3.0)
    assert F.shape == (64, 3) and len(np.unique(F, axis=0)) == 64
    mag = np.sqrt((F.astype(float) ** 2).sum(1))
    assert {tuple(m) for m in band} <= {tuple(m) for m in F}
    assert np.all((mag >= 2.0) & (mag <= 4.0))
    assert np.sum(mag > 3.0) == 64 - len(band)
    G = I.nf_frequencies(nmin=2.0, nmax=16.0)
    gm = np.sqrt((G.astype(float) ** 2).sum(1))
    assert len(np.unique(G, axis=0)) == 64 and np.all((gm >= 2.0) & (gm <= 16.0))
