"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module only *generates inputs*: the turbulent magnetic-field grid, the
per-nucleon interaction/loss tables, injection arrays and neural-field sample
points.  It contains none of the propagation arithmetic (no stepping, no
interpolation, no table lookup, no random-number stream of the method).

Units follow the C-ABI: metres, electron-volts, tesla, rates in 1/m.

The paper (section 6, benchmark tests) describes the 3D workload only as a
turbulent field of 1 nG RMS strength with protons of 1-1000 EeV; grid size,
spectrum band, table shapes and source geometry are this project's synthetic
stand-ins, stated in each function below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --- physical constants and units (SI-exact where defined) -----------------
C_LIGHT = 299792458.0                 # m/s
PC_M = 3.0856775814913673e16          # m
KPC_M = 1e3 * PC_M
MPC_M = 1e6 * PC_M
NG_T = 1e-13                          # tesla per nanogauss
EEV = 1e18                            # eV

# species table used by the mixed-composition workloads (id mod 4)
SPECIES_AZ = ((1, 1), (4, 2), (14, 7), (56, 26))


# --------------------------------------------------------------------------
# Turbulent field (section 6: "turbulent magnetic field of 1 nG B_rms").
# --------------------------------------------------------------------------
def turbulence_modes(n: int, nmin: float, nmax: float, exclude_nyquist: bool = True):
    """Representative lattice modes of the turbulence spectrum.

    Modes are integer wave vectors m (cycles per box) with nmin <= |m| <= nmax,
    no component on the Nyquist plane |m_a| = n/2, and the representative of
    each +/- pair has its first non-zero component positive.  Returned in
    lexicographic (C) order of (m_x, m_y, m_z).
    """
    r = int(math.floor(nmax))
    ax = np.arange(-r, r + 1)
    mx, my, mz = np.meshgrid(ax, ax, ax, indexing="ij")
    mx, my, mz = mx.ravel(), my.ravel(), mz.ravel()
    mag2 = mx * mx + my * my + mz * mz
    keep = (mag2 >= nmin * nmin) & (mag2 <= nmax * nmax)
    if exclude_nyquist and n % 2 == 0:
        h = n // 2
        keep &= (np.abs(mx) < h) & (np.abs(my) < h) & (np.abs(mz) < h)
    rep = (mx > 0) | ((mx == 0) & (my > 0)) | ((mx == 0) & (my == 0) & (mz > 0))
    keep &= rep
    return np.stack([mx[keep], my[keep], mz[keep]], axis=1).astype(np.int64)


def turbulence_coefficients(modes: np.ndarray, seed: int):
    """Complex vector amplitude of each representative mode.

    Amplitude |m|^(-11/6) (Kolmogorov: shell spectrum k^(-5/3), so per-mode
    power k^(-11/3)), polarisation cos(theta) e1 + sin(theta) e2 transverse to
    m (divergence-free), phase phi; theta and phi uniform on [0, 2 pi) drawn
    pairwise per mode from numpy's default_rng(seed) in the order given.
    """
    rng = np.random.default_rng(seed)
    ang = rng.random((modes.shape[0], 2)) * (2.0 * np.pi)
    theta, phi = ang[:, 0], ang[:, 1]
    m = modes.astype(np.float64)
    mag = np.sqrt((m * m).sum(axis=1))
    mhat = m / mag[:, None]
    zhat = np.array([0.0, 0.0, 1.0])
    xhat = np.array([1.0, 0.0, 0.0])
    par_z = (modes[:, 0] == 0) & (modes[:, 1] == 0)
    e1 = np.cross(m, zhat)
    e1[par_z] = np.cross(m[par_z], xhat)
    e1 /= np.sqrt((e1 * e1).sum(axis=1))[:, None]
    e2 = np.cross(mhat, e1)
    pol = np.cos(theta)[:, None] * e1 + np.sin(theta)[:, None] * e2
    amp = mag ** (-11.0 / 6.0)
    return (amp * np.exp(1j * phi))[:, None] * pol     # [M, 3] complex


def turbulent_grid(n: int, spacing_m: float, nmin: float, nmax: float,
                   brms_T: float, seed: int, dtype=np.float64, device=None):
    """Periodic divergence-free turbulent field on an n^3 vertex grid.

    Layout [n][n][n][3] (x slowest, component fastest), tesla.  Vertex (i,j,k)
    sits at (i,j,k)*spacing.  The field is rescaled so that the RMS of |B|
    over all vertices equals brms_T.  With ``device`` (a torch device) the
    inverse FFT runs through torch on that device and a torch tensor is
    returned; otherwise numpy on the host.
    """
    modes = turbulence_modes(n, nmin, nmax)
    coef = turbulence_coefficients(modes, seed)
    # m_z < 0 never occurs for representatives with m_x = m_y = 0; for the
    # others, a representative with m_z < 0 is stored through its partner -m
    # (which has m_z > 0) as conj(c).
    neg = modes[:, 2] < 0
    store_m = np.where(neg[:, None], -modes, modes)
    store_c = np.where(neg[:, None], np.conj(coef), coef)
    zero = store_m[:, 2] == 0
    ia = store_m % n
    ib = (-store_m[zero]) % n
    hz = n // 2 + 1
    if device is None:
        out = np.empty((n, n, n, 3), dtype=dtype)
        for comp in range(3):
            spec = np.zeros((n, n, hz), dtype=np.complex128)
            spec[ia[:, 0], ia[:, 1], ia[:, 2]] = store_c[:, comp]
            spec[ib[:, 0], ib[:, 1], ib[:, 2]] = np.conj(store_c[zero, comp])
            out[..., comp] = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2)) * float(n) ** 3
            del spec
        ms = 0.0
        for comp in range(3):
            ms += float(np.mean(out[..., comp].astype(np.float64) ** 2))
        scale = brms_T / math.sqrt(ms)
        out *= dtype(scale) if dtype == np.float32 else scale
        return out
    import torch
    out = torch.empty((n, n, n, 3), dtype=torch.float32 if dtype == np.float32 else torch.float64,
                      device=device)
    ia_t = torch.as_tensor(ia, device=device)
    ib_t = torch.as_tensor(ib, device=device)
    ms = 0.0
    for comp in range(3):
        spec = torch.zeros((n, n, hz), dtype=torch.complex128, device=device)
        spec[ia_t[:, 0], ia_t[:, 1], ia_t[:, 2]] = torch.as_tensor(store_c[:, comp], device=device)
        spec[ib_t[:, 0], ib_t[:, 1], ib_t[:, 2]] = torch.as_tensor(
            np.conj(store_c[zero, comp]), device=device)
        real = torch.fft.irfftn(spec, s=(n, n, n)) * float(n) ** 3
        del spec
        ms += float((real * real).mean().item())
        out[..., comp] = real.to(out.dtype)
        del real
    scale = brms_T / math.sqrt(ms)
    out.mul_(scale)
    return out


# --------------------------------------------------------------------------
# Synthetic rate / loss tables (per nucleon, at eps = E/A).
# --------------------------------------------------------------------------
def table_nodes(n: int = 200, lo_log10: float = 16.0, hi_log10: float = 23.0):
    """n log-spaced energy nodes from 10^lo to 10^hi eV (strictly increasing)."""
    j = np.arange(n, dtype=np.float64)
    return 10.0 ** (lo_log10 + (hi_log10 - lo_log10) * j / (n - 1))


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


@dataclass
class Tables:
    e_nodes: np.ndarray       # eV
    t_pi: np.ndarray          # 1/m, pion-production-like rate per nucleon
    t_n: np.ndarray           # 1/m, nucleon-loss-like rate per nucleon
    beta_p: np.ndarray        # 1/m, relative continuous loss rate of a proton


def tables_loss_only():
    """Smoothly rising pair-production-like loss table; no stochastic channels."""
    e = table_nodes()
    lg = np.log10(e)
    beta = (4e-3 * _sigmoid((lg - 18.6) / 0.25) + 1e-5) / MPC_M
    z = np.zeros_like(e)
    return Tables(e, z.copy(), z.copy(), beta)


def tables_full():
    """Loss table plus pion-production-like and nucleon-loss-like channels."""
    t = tables_loss_only()
    lg = np.log10(t.e_nodes)
    t.t_pi = 0.25 * _sigmoid((lg - 19.7) / 0.15) / MPC_M
    t.t_n = 0.05 * _sigmoid((lg - 18.7) / 0.20) / MPC_M
    return t


def tables_constant(e_nodes=None, t_pi=0.0, t_n=0.0, beta_p=0.0):
    """Energy-independent tables (used for closed-form checks)."""
    e = table_nodes() if e_nodes is None else e_nodes
    one = np.ones_like(e)
    return Tables(e, t_pi * one, t_n * one, beta_p * one)


# --------------------------------------------------------------------------
# Injection (the source class: position, spectrum, composition).
# --------------------------------------------------------------------------
@dataclass
class Injection:
    id: np.ndarray            # uint32
    A: np.ndarray             # int32
    Z: np.ndarray             # int32
    E: np.ndarray             # float64, eV
    pos: np.ndarray           # float64 [n,3], m
    dir: np.ndarray           # float64 [n,3], unit
    lmax: np.ndarray          # float64, m

    def __len__(self):
        return int(self.id.shape[0])

    def subset(self, sel):
        return Injection(self.id[sel], self.A[sel], self.Z[sel], self.E[sel],
                         self.pos[sel], self.dir[sel], self.lmax[sel])


def isotropic(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.sqrt((g * g).sum(axis=1))[:, None]


def powerlaw_energy(u, e1, e2):
    """Inverse CDF of dN/dE ~ E^-2 on [e1, e2] for uniform u in [0, 1)."""
    return 1.0 / (1.0 / e1 - u * (1.0 / e1 - 1.0 / e2))


def inject_protons_fixed(n=1000, energy_eV=1e19, lmax_m=10 * MPC_M, seed=101, id0=0):
    rng = np.random.default_rng(seed)
    d = isotropic(rng, n)
    return Injection(np.arange(id0, id0 + n, dtype=np.uint32), np.ones(n, np.int32),
                     np.ones(n, np.int32), np.full(n, energy_eV), np.zeros((n, 3)), d,
                     np.full(n, lmax_m))


def inject_mixed(n, seed, lmax_m=100 * MPC_M, e1=1e18, e2=1e21, id0=0):
    """Equal H/He/N/Fe fractions (species = id mod 4), E^-2, isotropic from the origin."""
    rng = np.random.default_rng(seed)
    ids = np.arange(id0, id0 + n, dtype=np.uint32)
    az = np.array(SPECIES_AZ, dtype=np.int32)[ids % 4]
    e = powerlaw_energy(rng.random(n), e1, e2)
    d = isotropic(rng, n)
    return Injection(ids, az[:, 0].copy(), az[:, 1].copy(), e, np.zeros((n, 3)), d,
                     np.full(n, lmax_m))


def inject_distances(n, seed, dmin_m=1 * MPC_M, dmax_m=1000 * MPC_M, e1=1e18, e2=1e21, id0=0):
    """Mixed composition at distance D ~ U[dmin, dmax] around an observer at the origin.

    Source at D * n_hat (n_hat isotropic); emission direction isotropic and
    independent; trajectory limit L_max = D.
    """
    rng = np.random.default_rng(seed)
    ids = np.arange(id0, id0 + n, dtype=np.uint32)
    az = np.array(SPECIES_AZ, dtype=np.int32)[ids % 4]
    e = powerlaw_energy(rng.random(n), e1, e2)
    dist = dmin_m + rng.random(n) * (dmax_m - dmin_m)
    pos = isotropic(rng, n) * dist[:, None]
    d = isotropic(rng, n)
    return Injection(ids, az[:, 0].copy(), az[:, 1].copy(), e, pos, d, dist)


def inject_protons_logflat(n, seed, e1=1e18, e2=1e21, lmax_m=1000 * MPC_M, id0=0):
    """Protons, log-flat spectrum (the paper's 3D benchmark composition)."""
    rng = np.random.default_rng(seed)
    e = 10.0 ** (np.log10(e1) + rng.random(n) * (np.log10(e2) - np.log10(e1)))
    d = isotropic(rng, n)
    return Injection(np.arange(id0, id0 + n, dtype=np.uint32), np.ones(n, np.int32),
                     np.ones(n, np.int32), e, np.zeros((n, 3)), d, np.full(n, lmax_m))


# --------------------------------------------------------------------------
# Galactic propagation (section 4): a synthetic analytic field and observed
# events to backtrack.
# --------------------------------------------------------------------------
MICROGAUSS_T = 1e-10
EARTH_KPC = (-8.5, 0.0, 0.02)          # galactocentric position of the observer

# Disk / halo / X-field model of the JF12 structure with rational profiles
# (the JF12 fit parameters are not available); galactocentric, axis z.
GALACTIC_FIELD = {
    "center": (0.0, 0.0, 0.0),
    "b_disk": 6.0 * MICROGAUSS_T, "r_disk": 5.0 * KPC_M, "h_disk": 0.4 * KPC_M,
    "b_halo": 4.0 * MICROGAUSS_T, "r_halo": 6.0 * KPC_M, "h_halo": 2.0 * KPC_M,
    "b_x": 1.5 * MICROGAUSS_T, "r_x": 4.0 * KPC_M, "h_x": 3.0 * KPC_M,
}


def inject_galactic(n, seed, e1=1e18, e2=1e20, lmax_m=100 * KPC_M, id0=0):
    """Events observed at Earth, to be backtracked: H/He/N/Fe (id mod 4),
    log-flat energies on [e1, e2], isotropic directions (the reversed arrival
    directions), all starting at the observer's position."""
    rng = np.random.default_rng(seed)
    ids = np.arange(id0, id0 + n, dtype=np.uint32)
    az = np.array(SPECIES_AZ, dtype=np.int32)[ids % 4]
    e = 10.0 ** (np.log10(e1) + rng.random(n) * (np.log10(e2) - np.log10(e1)))
    pos = np.tile(np.array(EARTH_KPC) * KPC_M, (n, 1))
    d = isotropic(rng, n)
    return Injection(ids, az[:, 0].copy(), az[:, 1].copy(), e, pos, d, np.full(n, lmax_m))


# --------------------------------------------------------------------------
# Workload descriptions.
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    grid_n: int
    spacing_m: float
    band: tuple               # (nmin, nmax) cycles per box
    grid_seed: int
    grid_dtype: type
    tables: str               # 'loss' | 'full'
    inject: str               # 'protons' | 'mixed' | 'distances'
    n_candidates: int
    inject_seed: int
    lmax_m: float
    observer: tuple = (0.0, 0.0, 0.0)
    obs_radius_m: float = 0.0
    philox_seed: int = 1
    tol: float = 1e-4
    hmin_m: float = 10 * KPC_M
    hmax_m: float = 1 * MPC_M
    brms_T: float = 1 * NG_T
    extra: dict = field(default_factory=dict)
    charge_sign: int = 1                  # -1: backtracking (antiparticle)
    boundary_center: tuple = (0.0, 0.0, 0.0)
    boundary_radius_m: float = 0.0        # spherical boundary (0: none)
    field: str = "grid"                   # 'grid' | 'analytic'

    def make_tables(self):
        if self.tables == "none":
            return tables_constant()
        return tables_full() if self.tables == "full" else tables_loss_only()

    def make_injection(self, n=None, id0=0):
        n = self.n_candidates if n is None else n
        if self.inject == "protons":
            return inject_protons_fixed(n, 1e19, self.lmax_m, self.inject_seed, id0)
        if self.inject == "mixed":
            return inject_mixed(n, self.inject_seed, self.lmax_m, id0=id0)
        if self.inject == "distances":
            return inject_distances(n, self.inject_seed, id0=id0)
        if self.inject == "logflat":
            return inject_protons_logflat(n, self.inject_seed, lmax_m=self.lmax_m, id0=id0)
        if self.inject == "galactic":
            return inject_galactic(n, self.inject_seed, lmax_m=self.lmax_m, id0=id0)
        raise ValueError(self.inject)

    def make_grid(self, device=None):
        return turbulent_grid(self.grid_n, self.spacing_m, self.band[0], self.band[1],
                              self.brms_T, self.grid_seed, self.grid_dtype, device)


# 1000 protons, 32^3 FP64 grid of 100 kpc cells, band 2..16 cells, 10 Mpc.
W_SMALL = Workload("p1e3_grid32_fp64", 32, 100 * KPC_M, (2.0, 16.0), 1, np.float64,
                   "loss", "protons", 1000, 101, 10 * MPC_M, philox_seed=1)
# 1e6 mixed nuclei, 256^3 FP64 grid of 50 kpc cells, band 2..16 cells,
# 100 Mpc or a 1 Mpc observer sphere at (50,0,0) Mpc.
W_MIXED256 = Workload("mixed1e6_grid256_fp64", 256, 50 * KPC_M, (16.0, 128.0), 2, np.float64,
                      "full", "mixed", 1_000_000, 202, 100 * MPC_M,
                      observer=(50 * MPC_M, 0.0, 0.0), obs_radius_m=1 * MPC_M, philox_seed=2)
# 1e7 mixed nuclei, 1024^3 FP32 grid of 10 kpc cells, band 2..16 cycles/box.
W_MIXED1024 = Workload("mixed1e7_grid1024_fp32", 1024, 10 * KPC_M, (2.0, 16.0), 3, np.float32,
                       "full", "mixed", 10_000_000, 303, 100 * MPC_M,
                       observer=(50 * MPC_M, 0.0, 0.0), obs_radius_m=1 * MPC_M, philox_seed=3)
# 1e7-candidate batches at distances 1..1000 Mpc around an observer at the origin.
W_DIST1024 = Workload("dist1e7_grid1024_fp32", 1024, 10 * KPC_M, (2.0, 16.0), 3, np.float32,
                      "full", "distances", 10_000_000, 404, 1000 * MPC_M,
                      observer=(0.0, 0.0, 0.0), obs_radius_m=1 * MPC_M, philox_seed=4)

# The shape of the paper's 3D benchmark (section 6): protons with a log-flat
# spectrum over 1-1000 EeV, 1 Gpc trajectories, energy losses off, here on the
# 256^3 FP64 turbulent grid (1 nG RMS).
W_PAPER256 = Workload("p_logflat_1gpc_grid256_fp64", 256, 50 * KPC_M, (16.0, 128.0), 2,
                      np.float64, "none", "logflat", 1_000_000, 606, 1000 * MPC_M, philox_seed=6)

# Galactic backtracking: observed events at Earth traced back (charge -Z,
# reversed direction) through the analytic field to a 20 kpc sphere.
W_GALBACK = Workload("galback1e6_analytic", 1, 1.0, (0.0, 0.0), 0, np.float64, "none",
                     "galactic", 1_000_000, 707, 100 * KPC_M, philox_seed=7,
                     hmin_m=1e-3 * KPC_M, hmax_m=1.0 * KPC_M, charge_sign=-1,
                     boundary_radius_m=20.0 * KPC_M, field="analytic")

WORKLOADS = {w.name: w for w in (W_SMALL, W_MIXED256, W_MIXED1024, W_DIST1024, W_PAPER256,
                                 W_GALBACK)}


# --------------------------------------------------------------------------
# Neural-field inputs: Fourier frequency matrix and sample points.
# --------------------------------------------------------------------------
def nf_frequencies(nfeat=64, nmin=2.0, nmax=16.0, seed=505):
    """Integer frequency vectors (cycles per box) for the Fourier embedding.

    Drawn without replacement from the representative modes of the field's
    band with probability proportional to the per-mode power |m|^(-11/3), so
    the low, energetic modes are favoured.  A band with fewer than nfeat modes
    gives all of them, and the rest is drawn the same way from the next shell
    nmax < |m| <= nmax + 1.
    """
    modes = turbulence_modes(0, nmin, nmax, exclude_nyquist=False)
    rng = np.random.default_rng(seed)

    def draw(cand, k):
        mag = np.sqrt((cand.astype(np.float64) ** 2).sum(axis=1))
        p = mag ** (-11.0 / 3.0)
        p /= p.sum()
        return cand[rng.choice(cand.shape[0], size=k, replace=False, p=p)]

    if modes.shape[0] >= nfeat:
        pick = draw(modes, nfeat)
    else:
        outer = turbulence_modes(0, nmax, nmax + 1.0, exclude_nyquist=False)
        mag = np.sqrt((outer.astype(np.float64) ** 2).sum(axis=1))
        outer = outer[mag > nmax]
        pick = np.concatenate([modes, draw(outer, nfeat - modes.shape[0])])
    order = np.lexsort(pick.T[::-1])
    return pick[order].astype(np.int32)


def nf_init_weights(seed=509, width=128, depth=4, nout=3, nin=128):
    """He-uniform initial FP32 master weights, row-major W[out][in], zero biases."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    fan = nin
    for _ in range(depth):
        lim = math.sqrt(6.0 / fan)
        ws.append(rng.uniform(-lim, lim, (width, fan)).astype(np.float32))
        bs.append(np.zeros(width, np.float32))
        fan = width
    lim = math.sqrt(3.0 / fan)
    ws.append(rng.uniform(-lim, lim, (nout, fan)).astype(np.float32))
    bs.append(np.zeros(nout, np.float32))
    return ws, bs


def nf_init_flat(seed=509):
    """The same initial parameters as one flat FP32 vector in the library's
    order W1, b1, ..., W4, b4, W5, b5 (each W row-major [out][in])."""
    ws, bs = nf_init_weights(seed)
    parts = []
    for W, b in zip(ws, bs):
        parts.append(np.asarray(W, np.float32).ravel())
        parts.append(np.asarray(b, np.float32).ravel())
    return np.concatenate(parts)


def uniform_points(n, box_m, seed, origin=(0.0, 0.0, 0.0)):
    """Uniform sample positions in one period of the field box, metres."""
    rng = np.random.default_rng(seed)
    return np.asarray(origin)[None, :] + rng.random((n, 3)) * box_m
