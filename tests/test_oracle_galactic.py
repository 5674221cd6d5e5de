"""Pins of the oracle's galactic-propagation pieces (section 4): the analytic
field, the charge sign used for backtracking and the spherical boundary.

The field checks do not retype its formula: they differentiate numerically
(divergence, curl of the vector potential the X-field is defined from) or use
symmetries and special points of the model's definition.
"""
import numpy as np
import pytest

import crp_inputs as I

KPC = I.KPC_M


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def model(**over):
    m = dict(I.GALACTIC_FIELD)
    m.update(over)
    return m


def field(O, m, pts):
    return O.eval_field(O.AnalyticRef(m), np.asarray(pts, np.float64), O.FP64)


def random_points(n, seed, rmax=15.0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-rmax, rmax, (n, 3)) * KPC
    p[:, 2] *= 0.3
    return p


def test_divergence_free(O):
    pts = random_points(200, 1)
    h = 1e-4 * KPC
    div = np.zeros(len(pts))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        div += (field(O, model(), pts + e)[:, a] - field(O, model(), pts - e)[:, a]) / (2 * h)
    bmag = np.linalg.norm(field(O, model(), pts), axis=1)
    # |div B| * (1 kpc) against |B|: zero up to the finite-difference error
    assert np.max(np.abs(div) * KPC / np.maximum(bmag, 1e-16)) < 1e-5


def test_x_field_is_curl_of_its_vector_potential(O):
    """Only the X-field: B = curl(A_phi e_phi) with A_phi = b_x r / (2 D)."""
    m = model(b_disk=0.0, b_halo=0.0)
    bx, rx, hx = m["b_x"], m["r_x"], m["h_x"]

    def A(p):
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        D = 1.0 + (x * x + y * y) / rx ** 2 + z * z / hx ** 2
        a = bx / (2.0 * D)                       # A = a (-y, x, 0)
        return np.stack([-a * y, a * x, np.zeros_like(x)], axis=1)

    pts = random_points(100, 2)
    h = 1e-4 * KPC

    def d(comp, axis):
        e = np.zeros(3)
        e[axis] = h
        return (A(pts + e)[:, comp] - A(pts - e)[:, comp]) / (2 * h)

    curl = np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)], axis=1)
    B = field(O, m, pts)
    assert np.max(np.abs(curl - B)) < 1e-6 * np.max(np.abs(B))


def test_toroidal_parts_are_azimuthal_with_their_z_parity(O):
    pts = random_points(100, 3)
    flip = pts * np.array([1.0, 1.0, -1.0])
    for part, parity in ((dict(b_halo=0.0, b_x=0.0), 1.0), (dict(b_disk=0.0, b_x=0.0), -1.0)):
        m = model(**part)
        B = field(O, m, pts)
        radial = (B[:, 0] * pts[:, 0] + B[:, 1] * pts[:, 1]) / np.hypot(pts[:, 0], pts[:, 1])
        assert np.max(np.abs(radial)) < 1e-12 * np.max(np.abs(B))
        assert np.all(B[:, 2] == 0.0)
        assert np.allclose(field(O, m, flip), parity * B, rtol=1e-14, atol=0)


def test_disk_peak_value(O):
    """B_phi = b_disk (r/r_d) / ((1 + r^2/r_d^2)(1 + z^2/h_d^2)) peaks at r = r_d, z = 0
    with b_disk / 2, pointing along e_phi."""
    m = model(b_halo=0.0, b_x=0.0)
    rd = m["r_disk"]
    B = field(O, m, [[rd, 0.0, 0.0], [0.0, rd, 0.0]])
    assert B[0, 1] == pytest.approx(m["b_disk"] / 2, rel=1e-15) and B[0, 0] == 0.0
    assert B[1, 0] == pytest.approx(-m["b_disk"] / 2, rel=1e-15)
    # and the profile falls off on both sides
    r = np.array([0.5, 0.9, 1.1, 2.0]) * rd
    Bp = field(O, m, np.stack([r, 0 * r, 0 * r], axis=1))[:, 1]
    assert np.all(Bp < m["b_disk"] / 2)


def _run(O, w, m, inj, **cfg):
    f, _, c, _ = O.propagate(O.config_for(w, **cfg), O.AnalyticRef(m),
                             O.TablesRef(w.make_tables()), inj, nthreads=4)
    return O.sort_finished(f), c


def test_charge_sign_equals_reversed_field_bitwise(O):
    """Charge -Z in the field is the same motion as charge +Z in the field -B:
    (-kappa)(u x B) and kappa(u x (-B)) are the same floating-point numbers."""
    w = I.W_GALBACK
    inj = w.make_injection(64)
    neg = {k: (-v if k.startswith("b_") else v) for k, v in I.GALACTIC_FIELD.items()}
    fa, ca = _run(O, w, I.GALACTIC_FIELD, inj, charge_sign=-1)
    fb, cb = _run(O, w, neg, inj, charge_sign=1)
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert ca["steps"] == cb["steps"]


def test_backtracking_retraces_a_forward_trajectory(O):
    """Forward with charge +Z over 12 kpc, then back from the end point with the
    reversed direction and charge -Z over the same length: the start is
    recovered to within the integration tolerance."""
    w = I.W_GALBACK
    n = 40
    inj = w.make_injection(n)
    inj.E = np.full(n, 3e19)
    inj.A = np.ones(n, np.int32)
    inj.Z = np.ones(n, np.int32)
    L = 12.0 * KPC
    inj.lmax = np.full(n, L)
    fwd, _ = _run(O, w, I.GALACTIC_FIELD, inj, charge_sign=1, bnd_r=0.0, tol=1e-7)
    back = I.Injection(fwd["id"].copy(), fwd["A"].copy(), fwd["Z"].copy(), fwd["E"].copy(),
                       fwd["x"].copy(), -fwd["u"], np.full(n, L))
    bwd, _ = _run(O, w, I.GALACTIC_FIELD, back, charge_sign=-1, bnd_r=0.0, tol=1e-7)
    order = np.argsort(inj.id)
    start = inj.pos[order]
    assert np.all(bwd["L"] == L) and np.all(fwd["L"] == L)
    assert np.max(np.linalg.norm(bwd["x"] - start, axis=1)) < 1e-6 * L
    u0 = inj.dir[order]
    assert np.max(np.linalg.norm(bwd["u"] + u0, axis=1)) < 1e-5
    # the deflection was not trivial
    assert np.median(np.degrees(np.arccos(np.clip((fwd["u"] * fwd["u0"]).sum(1), -1, 1)))) > 2


def test_spherical_boundary_straight_lines(O):
    """No field: candidates leave the 20 kpc sphere on a straight line and stop
    at the first cycle end outside it (within one step of the sphere)."""
    w = I.W_GALBACK
    zero = {k: (0.0 if k.startswith("b_") else v) for k, v in I.GALACTIC_FIELD.items()}
    inj = w.make_injection(200)
    f, c = _run(O, w, zero, inj)
    assert c["boundary"] == 200 and c["max_traj"] == 0
    assert np.all(f["status"] == O.BOUNDARY)
    r = np.linalg.norm(f["x"], axis=1)
    assert np.all(r >= w.boundary_radius_m) and np.all(r < w.boundary_radius_m + w.hmax_m)
    # straight: the end point is the start plus L along the initial direction
    fo = np.argsort(inj.id)
    end = inj.pos[fo] + f["L"][:, None] * inj.dir[fo]
    assert np.max(np.linalg.norm(f["x"] - end, axis=1)) < 1e-9 * np.max(f["L"])
