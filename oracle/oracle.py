"""ctypes wrapper of the FP64 CPU oracle (liboracle.so) -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
this module.  It shares no code with the GPU library; both sides only read the
same input arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "crp_oracle.c")

FP64, MIX = 0, 1
GRID_F32, GRID_F64 = 0, 1
ACTIVE, OBSERVED, MAX_TRAJ, ENERGY_FLOOR, BOUNDARY = 0, 1, 2, 3, 4
CHAN_PI, CHAN_N = 0, 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: FP64 IEEE, no contraction, OpenMP."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=gnu11", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_P = C.POINTER


class Config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("renormalize", C.c_int32), ("tol", C.c_double),
                ("hmin", C.c_double), ("hmax", C.c_double), ("eps_loss", C.c_double),
                ("kappa_pi", C.c_double), ("e_floor", C.c_double), ("obs", C.c_double * 3),
                ("obs_r", C.c_double), ("seed", C.c_uint64), ("max_cycles", C.c_int64),
                ("charge_sign", C.c_int32), ("pad_", C.c_int32), ("bnd_center", C.c_double * 3),
                ("bnd_r", C.c_double), ("traj_every", C.c_int32), ("traj_ids", C.c_uint32)]


class Analytic(C.Structure):
    _fields_ = [("center", C.c_double * 3)] + [(k, C.c_double) for k in (
        "b_disk", "r_disk", "h_disk", "b_halo", "r_halo", "h_halo", "b_x", "r_x", "h_x")]


class Patch(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n", C.c_int64 * 3), ("offset", C.c_int64 * 3),
                ("refine", C.c_int32), ("pad_", C.c_int32)]


FIELD_CB = C.CFUNCTYPE(None, C.c_void_p, _P(C.c_double), _P(C.c_double))


class Grid(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("pad_", C.c_int32),
                ("n", C.c_int64 * 3), ("spacing", C.c_double), ("origin", C.c_double * 3),
                ("analytic", _P(Analytic)), ("n_patches", C.c_int32), ("pad2_", C.c_int32),
                ("patches", _P(Patch)), ("field_cb", FIELD_CB), ("cb_user", C.c_void_p)]


class Tables(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad_", C.c_int32), ("e", _P(C.c_double)),
                ("tpi", _P(C.c_double)), ("tn", _P(C.c_double)), ("bp", _P(C.c_double))]


class Finished(C.Structure):
    _fields_ = [("cap", C.c_int64)] + [(k, _P(C.c_uint32)) for k in
                                       ("id", "lineage", "m", "nsteps", "nrej")] + \
               [(k, _P(C.c_int32)) for k in ("status", "A", "Z")] + \
               [(k, _P(C.c_double)) for k in ("E", "x", "u", "L", "u0", "E0")]


class Neutral(C.Structure):
    _fields_ = [("cap", C.c_int64), ("id", _P(C.c_uint32)), ("lineage", _P(C.c_uint32)),
                ("m", _P(C.c_uint32)), ("chan", _P(C.c_int32)), ("E", _P(C.c_double)),
                ("x", _P(C.c_double)), ("u", _P(C.c_double))]


class Traj(C.Structure):
    _fields_ = [("cap", C.c_int64), ("id", _P(C.c_uint32)), ("lineage", _P(C.c_uint32)),
                ("n", _P(C.c_uint32)), ("A", _P(C.c_int32)), ("L", _P(C.c_double)),
                ("E", _P(C.c_double)), ("x", _P(C.c_double))]


COUNT_FIELDS = ("finished", "observed", "max_traj", "energy_floor", "still_active", "steps",
                "attempts", "rejects", "forced", "events", "null_events", "inter_pi",
                "inter_n", "charged_sec", "neutral_sec", "fin_dropped", "neu_dropped",
                "boundary", "traj_dropped")


class Counts(C.Structure):
    _fields_ = [(k, C.c_int64) for k in COUNT_FIELDS]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.oracle_propagate.restype = C.c_int
        L.oracle_propagate.argtypes = [
            _P(Config), _P(Grid), _P(Tables), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, _P(Finished), _P(Neutral),
            _P(Counts), _P(C.c_int64), _P(C.c_int64)]
        L.oracle_propagate_traj.restype = C.c_int
        L.oracle_propagate_traj.argtypes = L.oracle_propagate.argtypes + [_P(Traj),
                                                                          _P(C.c_int64)]
        L.oracle_eval_field.restype = None
        L.oracle_eval_field.argtypes = [_P(Grid), C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]
        L.oracle_ck_attempt.restype = None
        L.oracle_ck_attempt.argtypes = [_P(Grid), C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_double, C.c_void_p, C.c_void_p, _P(C.c_double)]
        L.oracle_philox4x64.restype = None
        L.oracle_philox4x64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_table_lookup.restype = C.c_double
        L.oracle_table_lookup.argtypes = [_P(Tables), C.c_int32, C.c_double]
        L.oracle_rates.restype = None
        L.oracle_rates.argtypes = [_P(Tables), C.c_int32, C.c_int32, C.c_double, C.c_void_p]
        L.oracle_texp.restype = C.c_double
        L.oracle_texp.argtypes = [C.c_uint64]
        L.oracle_ctrl_k.restype = C.c_int32
        L.oracle_ctrl_k.argtypes = [C.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class GridRef:
    """Keeps the numpy array alive while the C struct points into it."""

    def __init__(self, data, spacing, origin=(0.0, 0.0, 0.0), patches=()):
        """patches: refinement patches, each a dict with data ([n0][n1][n2][3] of
        the base grid's dtype), offset (base vertex index of its first vertex)
        and refine (base cells per patch cell)."""
        data = np.asarray(data)
        if data.dtype not in (np.float32, np.float64) or data.ndim != 4 or data.shape[3] != 3:
            raise ValueError("grid must be [nx][ny][nz][3] float32/float64")
        self.arr = np.ascontiguousarray(data)
        self.s = Grid()
        self.s.data = self.arr.ctypes.data
        self.s.dtype = GRID_F64 if self.arr.dtype == np.float64 else GRID_F32
        for a in range(3):
            self.s.n[a] = self.arr.shape[a]
            self.s.origin[a] = float(origin[a])
        self.s.spacing = float(spacing)
        self.patch_arrs = [np.ascontiguousarray(q["data"], self.arr.dtype) for q in patches]
        if patches:
            self.ps = (Patch * len(patches))()
            for k, q in enumerate(patches):
                a = self.patch_arrs[k]
                assert a.ndim == 4 and a.shape[3] == 3
                self.ps[k].data = a.ctypes.data
                for ax in range(3):
                    self.ps[k].n[ax] = a.shape[ax]
                    self.ps[k].offset[ax] = int(q["offset"][ax])
                self.ps[k].refine = int(q["refine"])
            self.s.n_patches = len(patches)
            self.s.patches = C.cast(self.ps, _P(Patch))


class AnalyticRef:
    """The analytic galactic field as a field source (no grid array)."""

    def __init__(self, model):
        self.a = Analytic()
        for a in range(3):
            self.a.center[a] = float(model["center"][a])
        for k in ("b_disk", "r_disk", "h_disk", "b_halo", "r_halo", "h_halo", "b_x", "r_x",
                  "h_x"):
            setattr(self.a, k, float(model[k]))
        self.s = Grid()
        self.s.data = None
        self.s.dtype = GRID_F64
        for a in range(3):
            self.s.n[a] = 1
        self.s.spacing = 1.0
        self.s.analytic = C.pointer(self.a)


class FieldRef:
    """A Python function as the field source: fn(p) -> B for one position p
    (numpy [3], metres) returning [3] tesla in FP64.  Propagation with it runs
    on one thread."""

    def __init__(self, fn):
        self.fn = fn

        def cb(_user, p, B):
            b = fn(np.array([p[0], p[1], p[2]]))
            B[0], B[1], B[2] = float(b[0]), float(b[1]), float(b[2])

        self.cb = FIELD_CB(cb)          # kept alive with this object
        self.s = Grid()
        self.s.data = None
        self.s.dtype = GRID_F64
        for a in range(3):
            self.s.n[a] = 1
        self.s.spacing = 1.0
        self.s.field_cb = self.cb


class TablesRef:
    def __init__(self, t):
        self.arrs = [np.ascontiguousarray(np.asarray(a, np.float64))
                     for a in (t.e_nodes, t.t_pi, t.t_n, t.beta_p)]
        self.s = Tables()
        self.s.n = len(self.arrs[0])
        self.s.e, self.s.tpi, self.s.tn, self.s.bp = [
            a.ctypes.data_as(_P(C.c_double)) for a in self.arrs]


def make_config(precision=FP64, tol=1e-4, hmin=None, hmax=None, eps_loss=0.1, kappa_pi=0.2,
                e_floor=1e16, observer=(0.0, 0.0, 0.0), obs_r=0.0, seed=1, renormalize=1,
                max_cycles=0, charge_sign=1, bnd_center=(0.0, 0.0, 0.0), bnd_r=0.0,
                traj_every=0, traj_ids=0):
    kpc = 3.0856775814913673e19
    c = Config()
    c.precision = precision
    c.renormalize = renormalize
    c.tol = tol
    c.hmin = 10 * kpc if hmin is None else hmin
    c.hmax = 1000 * kpc if hmax is None else hmax
    c.eps_loss = eps_loss
    c.kappa_pi = kappa_pi
    c.e_floor = e_floor
    for a in range(3):
        c.obs[a] = observer[a]
    c.obs_r = obs_r
    c.seed = seed
    c.max_cycles = max_cycles
    c.charge_sign = charge_sign
    for a in range(3):
        c.bnd_center[a] = bnd_center[a]
    c.bnd_r = bnd_r
    c.traj_every = traj_every
    c.traj_ids = traj_ids
    return c


def config_for(workload, precision=FP64, **kw):
    args = dict(precision=precision, tol=workload.tol, hmin=workload.hmin_m,
                hmax=workload.hmax_m, observer=workload.observer, obs_r=workload.obs_radius_m,
                seed=workload.philox_seed, charge_sign=workload.charge_sign,
                bnd_center=workload.boundary_center, bnd_r=workload.boundary_radius_m)
    args.update(kw)
    return make_config(**args)


FIN_FIELDS = {"id": np.uint32, "lineage": np.uint32, "m": np.uint32, "nsteps": np.uint32,
              "nrej": np.uint32, "status": np.int32, "A": np.int32, "Z": np.int32,
              "E": np.float64, "x": np.float64, "u": np.float64, "L": np.float64,
              "u0": np.float64, "E0": np.float64}
NEU_FIELDS = {"id": np.uint32, "lineage": np.uint32, "m": np.uint32, "chan": np.int32,
              "E": np.float64, "x": np.float64, "u": np.float64}
TRAJ_FIELDS = {"id": np.uint32, "lineage": np.uint32, "n": np.uint32, "A": np.int32,
               "L": np.float64, "E": np.float64, "x": np.float64}
VEC3 = ("x", "u", "u0")


def _alloc(fields, cap):
    out = {}
    for k, dt in fields.items():
        out[k] = np.zeros((max(cap, 1), 3) if k in VEC3 else max(cap, 1), dtype=dt)
    return out


def propagate(cfg, grid: GridRef, tables: TablesRef, inj, nthreads=0, fin_cap=None,
              neu_cap=None):
    """Run the oracle; returns (finished dict, neutral dict, counts dict, threads)."""
    fin, neu, counts, used, _ = _run(cfg, grid, tables, inj, nthreads, fin_cap, neu_cap, None)
    return fin, neu, counts, used


def propagate_traj(cfg, grid: GridRef, tables: TablesRef, inj, traj_cap, nthreads=0,
                   fin_cap=None, neu_cap=None):
    """Run the oracle with per-step trajectory output (config traj_every /
    traj_ids); returns (finished, neutral, counts, trajectory points), the
    points as a dict of arrays (id, lineage, n, A, L, E, x)."""
    fin, neu, counts, _, traj = _run(cfg, grid, tables, inj, nthreads, fin_cap, neu_cap,
                                     int(traj_cap))
    return fin, neu, counts, traj


def _run(cfg, grid, tables, inj, nthreads, fin_cap, neu_cap, traj_cap):
    n = len(inj)
    fin_cap = fin_cap if fin_cap is not None else max(16, 64 * n)
    neu_cap = neu_cap if neu_cap is not None else max(16, 64 * n)
    fin = _alloc(FIN_FIELDS, fin_cap)
    neu = _alloc(NEU_FIELDS, neu_cap)
    fs = Finished()
    fs.cap = fin_cap
    for k in FIN_FIELDS:
        setattr(fs, k, fin[k].ctypes.data_as(dict(Finished._fields_)[k]))
    ns = Neutral()
    ns.cap = neu_cap
    for k in NEU_FIELDS:
        setattr(ns, k, neu[k].ctypes.data_as(dict(Neutral._fields_)[k]))
    ids = np.ascontiguousarray(inj.id, np.uint32)
    A = np.ascontiguousarray(inj.A, np.int32)
    Z = np.ascontiguousarray(inj.Z, np.int32)
    E = np.ascontiguousarray(inj.E, np.float64)
    pos = np.ascontiguousarray(inj.pos, np.float64)
    d = np.ascontiguousarray(inj.dir, np.float64)
    lm = np.ascontiguousarray(inj.lmax, np.float64)
    cnt = Counts()
    nf = C.c_int64(0)
    nn = C.c_int64(0)
    args = [C.byref(cfg), C.byref(grid.s), C.byref(tables.s), n, _ptr(ids), _ptr(A), _ptr(Z),
            _ptr(E), _ptr(pos), _ptr(d), _ptr(lm), int(nthreads), C.byref(fs), C.byref(ns),
            C.byref(cnt), C.byref(nf), C.byref(nn)]
    traj = None
    if traj_cap is None:
        used = lib().oracle_propagate(*args)
    else:
        traj = _alloc(TRAJ_FIELDS, traj_cap)
        ts = Traj()
        ts.cap = traj_cap
        for k in TRAJ_FIELDS:
            setattr(ts, k, traj[k].ctypes.data_as(dict(Traj._fields_)[k]))
        nt = C.c_int64(0)
        used = lib().oracle_propagate_traj(*args, C.byref(ts), C.byref(nt))
        nt = min(nt.value, traj_cap)
        traj = {k: v[:nt] for k, v in traj.items()}
    nf = min(nf.value, fin_cap)
    nn = min(nn.value, neu_cap)
    fin = {k: v[:nf] for k, v in fin.items()}
    neu = {k: v[:nn] for k, v in neu.items()}
    counts = {k: getattr(cnt, k) for k in COUNT_FIELDS}
    return fin, neu, counts, used, traj


def eval_field(grid: GridRef, pos, mode=FP64):
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    out = np.empty_like(pos)
    lib().oracle_eval_field(C.byref(grid.s), mode, pos.shape[0], _ptr(pos), _ptr(out))
    return out


def ck_attempt(grid: GridRef, x, u, kappa, h, mode=FP64):
    x = np.ascontiguousarray(x, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    x5 = np.empty(3)
    u5 = np.empty(3)
    err = C.c_double(0)
    lib().oracle_ck_attempt(C.byref(grid.s), mode, _ptr(x), _ptr(u), kappa, h, _ptr(x5),
                            _ptr(u5), C.byref(err))
    return x5, u5, err.value


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.empty(4, np.uint64)
    lib().oracle_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def table_lookup(tables: TablesRef, which, eps):
    return lib().oracle_table_lookup(C.byref(tables.s), which, eps)


def rates(tables: TablesRef, A, Z, E):
    out = np.empty(4)
    lib().oracle_rates(C.byref(tables.s), A, Z, E, _ptr(out))
    return out


def texp(w):
    return lib().oracle_texp(int(w))


def ctrl_k(r):
    return lib().oracle_ctrl_k(r)


def sort_finished(fin):
    """Order finished records by their key (id, lineage)."""
    order = np.lexsort((fin["lineage"], fin["id"]))
    return {k: v[order] for k, v in fin.items()}


def sort_traj(tr):
    """Order trajectory points by (id, lineage, step)."""
    order = np.lexsort((tr["n"], tr["lineage"], tr["id"]))
    return {k: v[order] for k, v in tr.items()}


def sort_neutral(neu):
    order = np.lexsort((neu["m"], neu["lineage"], neu["id"]))
    return {k: v[order] for k, v in neu.items()}
