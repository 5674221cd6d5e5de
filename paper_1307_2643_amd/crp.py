"""Thin ctypes binding of libcrp.so (include/crp.h): argument marshalling only.

Every step of the propagation runs in the HIP kernels of libcrp; this module
converts numpy arrays / torch tensors into pointers and status codes into
exceptions.  PyTorch is used only for device memory and the HIP stream.  If the
library is missing the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrp.so")

OK, INCOMPLETE, EOVERFLOW = 0, 1, 2
STATUS_NAMES = {0: "CRP_OK", 1: "CRP_INCOMPLETE", 2: "CRP_EOVERFLOW", -1: "CRP_EINVAL",
                -2: "CRP_EDEVICE", -3: "CRP_ENOMEM", -4: "CRP_ESTATE", -5: "CRP_EQUEUE"}
FP64, MIX = 0, 1
FIELD_GRID, FIELD_NEURAL, FIELD_ANALYTIC = 0, 1, 2
EVAL_NEURAL = 16 + FIELD_NEURAL
EVAL_ANALYTIC = 16 + FIELD_ANALYTIC
EVAL_NOALLOC_MAX = 262144          # CRP_EVAL_NOALLOC_MAX
F32, F64 = 0, 1
LAYOUT_LINEAR, LAYOUT_CORNER = 0, 1
ORDER_LONGEST_FIRST, ORDER_AS_GIVEN = 0, 1
ACTIVE, OBSERVED, MAX_TRAJ, ENERGY_FLOOR, BOUNDARY = 0, 1, 2, 3, 4
NF_NPARAM = 66435

EXPORTS = ("crp_create", "crp_destroy", "crp_set_field_grid", "crp_set_field_patches",
           "crp_set_field_analytic",
           "crp_set_tables", "crp_inject",
           "crp_propagate", "crp_read_finished", "crp_read_neutral", "crp_read_trajectory",
           "crp_set_observables", "crp_observe", "crp_read_observables", "crp_lens_build",
           "crp_lens_read", "crp_lens_apply", "crp_peek_pending",
           "crp_counts", "crp_reset_counters", "crp_eval_field", "crp_eval_field_noalloc",
           "crp_set_launch",
           "crp_get_launch", "crp_tune", "crp_last_timing", "crp_gather_ceiling",
           "crp_snapshot", "crp_restore",
           "crp_free", "crp_nf_init", "crp_nf_get_params", "crp_nf_loss_grad", "crp_nf_adam_step",
           "crp_nf_train",
           "crp_last_error")


class CrpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("field_mode", C.c_int32), ("renormalize", C.c_int32),
                ("device", C.c_int32), ("tol", C.c_double), ("hmin", C.c_double),
                ("hmax", C.c_double), ("eps_loss", C.c_double), ("kappa_pi", C.c_double),
                ("e_floor", C.c_double), ("obs_center", C.c_double * 3),
                ("obs_radius", C.c_double), ("seed", C.c_uint64),
                ("queue_capacity", C.c_int64), ("neutral_capacity", C.c_int64),
                ("charge_sign", C.c_int32), ("inject_order", C.c_int32),
                ("boundary_center", C.c_double * 3), ("boundary_radius", C.c_double),
                ("traj_every", C.c_int32), ("traj_ids", C.c_uint32),
                ("traj_capacity", C.c_int64)]


class AnalyticField(C.Structure):
    _fields_ = [("center", C.c_double * 3)] + [(k, C.c_double) for k in (
        "b_disk", "r_disk", "h_disk", "b_halo", "r_halo", "h_halo", "b_x", "r_x", "h_x")]


class GridPatch(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n", C.c_int64 * 3), ("offset", C.c_int64 * 3),
                ("refine", C.c_int32), ("on_device", C.c_int32)]


class Launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("refill", C.c_int32),
                ("layout", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.POINTER


class FinishedSoA(C.Structure):
    _fields_ = [(k, _P(C.c_uint32)) for k in ("id", "lineage", "m", "nsteps", "nrej")] + \
               [(k, _P(C.c_int32)) for k in ("status", "A", "Z")] + \
               [(k, _P(C.c_double)) for k in ("E", "x", "u", "L", "u0", "E0")]


class NeutralSoA(C.Structure):
    _fields_ = [("id", _P(C.c_uint32)), ("lineage", _P(C.c_uint32)), ("m", _P(C.c_uint32)),
                ("chan", _P(C.c_int32)), ("E", _P(C.c_double)), ("x", _P(C.c_double)),
                ("u", _P(C.c_double))]


class TrajSoA(C.Structure):
    _fields_ = [("id", _P(C.c_uint32)), ("lineage", _P(C.c_uint32)), ("n", _P(C.c_uint32)),
                ("A", _P(C.c_int32)), ("L", _P(C.c_double)), ("E", _P(C.c_double)),
                ("x", _P(C.c_double))]


class Observables(C.Structure):
    _fields_ = [("n_e", C.c_int32), ("n_groups", C.c_int32), ("e_edges", _P(C.c_double)),
                ("a_edges", _P(C.c_int32)), ("status_mask", C.c_int32), ("sky_n", C.c_int32),
                ("sky_sign", C.c_double), ("e_ref", C.c_double), ("gamma", C.c_double)]


class LensSpec(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("sky_n", C.c_int32), ("r_edges", _P(C.c_double)),
                ("status_mask", C.c_int32), ("pad_", C.c_int32)]


COUNT_FIELDS = ("finished", "observed", "max_traj", "energy_floor", "steps", "attempts",
                "rejects", "forced", "events", "null_events", "inter_pi", "inter_n",
                "charged_sec", "neutral_sec", "queue_deferred", "neutral_deferred", "pending",
                "finished_unread", "neutral_unread", "lane_slots", "boundary", "traj_points",
                "traj_dropped", "traj_unread")


class Counters(C.Structure):
    _fields_ = [(k, C.c_int64) for k in COUNT_FIELDS]


_lib = None


def load():
    """Loads libcrp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1307_2643_amd.build` (no CPU fallback exists)")
    # One HIP runtime per process: PyTorch carries its own copy, and of two
    # copies loaded side by side the second finds no GPU.  Importing torch
    # first makes the library bind to torch's copy (same soname).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sig = {
        "crp_create": ([_P(Config), vp, _P(vp)], C.c_int),
        "crp_destroy": ([vp], None),
        "crp_set_field_grid": ([vp, vp, i32, i32, i64, i64, i64, dbl, vp], C.c_int),
        "crp_set_field_analytic": ([vp, _P(AnalyticField)], C.c_int),
        "crp_set_field_patches": ([vp, i32, _P(GridPatch)], C.c_int),
        "crp_set_tables": ([vp, i32, vp, vp, vp, vp], C.c_int),
        "crp_inject": ([vp, i64, vp, vp, vp, vp, vp, vp, vp, i32], C.c_int),
        "crp_propagate": ([vp, i64], C.c_int),
        "crp_read_finished": ([vp, i64, _P(FinishedSoA), _P(i64)], C.c_int),
        "crp_read_neutral": ([vp, i64, _P(NeutralSoA), _P(i64)], C.c_int),
        "crp_read_trajectory": ([vp, i64, _P(TrajSoA), _P(i64)], C.c_int),
        "crp_set_observables": ([vp, _P(Observables)], C.c_int),
        "crp_observe": ([vp, _P(dbl)], C.c_int),
        "crp_read_observables": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "crp_lens_build": ([vp, _P(LensSpec), _P(i64), _P(dbl)], C.c_int),
        "crp_lens_read": ([vp, vp, vp, vp, vp], C.c_int),
        "crp_lens_apply": ([vp, i32, vp, vp, i32, _P(dbl)], C.c_int),
        "crp_peek_pending": ([vp, i64, _P(FinishedSoA), _P(i64)], C.c_int),
        "crp_counts": ([vp, _P(Counters)], C.c_int),
        "crp_reset_counters": ([vp], C.c_int),
        "crp_eval_field": ([vp, i64, vp, vp, i32, i32], C.c_int),
        "crp_eval_field_noalloc": ([vp, i64, vp, vp, i32], C.c_int),
        "crp_set_launch": ([vp, _P(Launch)], C.c_int),
        "crp_get_launch": ([vp, _P(Launch)], C.c_int),
        "crp_tune": ([vp, i64, C.c_char_p, _P(Launch), _P(dbl)], C.c_int),
        "crp_last_timing": ([vp, _P(dbl), _P(i64)], C.c_int),
        "crp_gather_ceiling": ([vp, i32, _P(dbl)], C.c_int),
        "crp_snapshot": ([vp, _P(vp), _P(C.c_size_t)], C.c_int),
        "crp_restore": ([vp, vp, C.c_size_t], C.c_int),
        "crp_free": ([vp], None),
        "crp_nf_init": ([vp, vp, vp, dbl], C.c_int),
        "crp_nf_get_params": ([vp, vp], C.c_int),
        "crp_nf_loss_grad": ([vp, i64, vp, vp, vp, vp, _P(dbl)], C.c_int),
        "crp_nf_adam_step": ([vp, vp, dbl], C.c_int),
        "crp_nf_train": ([vp, i64, i64, dbl, dbl, C.c_uint64, vp], C.c_int),
        "crp_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(a):
    """Pointer of a numpy array or torch tensor (host or device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _is_dev(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _shape_ok(got, want, what):
    if len(got) != len(want) or any(w is not None and g != w for g, w in zip(got, want)):
        exp = tuple("*" if w is None else w for w in want)
        raise ValueError(f"{what}: shape {tuple(got)}, expected {exp}")


def _host(a, dtype, shape, what):
    """`a` as a C-contiguous host array of `dtype` whose shape matches `shape`
    (None matches any extent).  The library reads exactly the sizes it is
    given, so every shape is checked here before a pointer is passed."""
    if hasattr(a, "is_cuda"):
        raise ValueError(f"{what}: a host array is expected here, got a torch tensor")
    a = np.ascontiguousarray(a, dtype)
    _shape_ok(a.shape, shape, what)
    return a


def _dev(a, dtype, shape, what, device):
    """`a` checked as a contiguous torch tensor on GPU `device` of `dtype`
    (uint32 data may come as int32 tensors) with a shape matching `shape`."""
    if not _is_dev(a):
        raise ValueError(f"{what}: a torch tensor on the GPU is expected here")
    import torch
    ok = {np.float64: (torch.float64,), np.float32: (torch.float32,),
          np.int32: (torch.int32,), np.uint32: (torch.int32, torch.uint32)}[dtype]
    if a.dtype not in ok:
        raise ValueError(f"{what}: dtype {a.dtype}, expected {ok[0]}")
    if not a.is_contiguous():
        raise ValueError(f"{what}: the tensor must be contiguous")
    if a.device.index != device:
        raise ValueError(f"{what}: tensor on {a.device}, the context uses cuda:{device}")
    _shape_ok(tuple(a.shape), shape, what)
    return a


FIN_FIELDS = {"id": np.uint32, "lineage": np.uint32, "m": np.uint32, "nsteps": np.uint32,
              "nrej": np.uint32, "status": np.int32, "A": np.int32, "Z": np.int32,
              "E": np.float64, "x": np.float64, "u": np.float64, "L": np.float64,
              "u0": np.float64, "E0": np.float64}
NEU_FIELDS = {"id": np.uint32, "lineage": np.uint32, "m": np.uint32, "chan": np.int32,
              "E": np.float64, "x": np.float64, "u": np.float64}
TRAJ_FIELDS = {"id": np.uint32, "lineage": np.uint32, "n": np.uint32, "A": np.int32,
               "L": np.float64, "E": np.float64, "x": np.float64}
VEC3 = ("x", "u", "u0")


def _alloc(fields, n):
    return {k: np.zeros((n, 3) if k in VEC3 else n, dtype=dt) for k, dt in fields.items()}


def _fill(struct_cls, arrs):
    s = struct_cls()
    for k, t in struct_cls._fields_:
        setattr(s, k, arrs[k].ctypes.data_as(t))
    return s


@dataclass
class Params:
    precision: int = FP64
    field_mode: int = FIELD_GRID
    renormalize: int = 1
    device: int = 0
    tol: float = 1e-4
    hmin: float = 3.0856775814913673e20      # 10 kpc
    hmax: float = 3.0856775814913673e22      # 1 Mpc
    eps_loss: float = 0.1
    kappa_pi: float = 0.2
    e_floor: float = 1e16
    obs_center: tuple = (0.0, 0.0, 0.0)
    obs_radius: float = 0.0
    seed: int = 1
    queue_capacity: int = 1 << 16
    neutral_capacity: int = 1 << 16
    charge_sign: int = 1
    inject_order: int = 0                    # ORDER_LONGEST_FIRST
    boundary_center: tuple = (0.0, 0.0, 0.0)
    boundary_radius: float = 0.0
    traj_every: int = 0
    traj_ids: int = 0
    traj_capacity: int = 0


class Context:
    """One libcrp context.  `stream`: a torch.cuda.Stream (or None: default)."""

    def __init__(self, params: Params, stream=None):
        self.L = load()
        c = Config()
        for k, _ in Config._fields_:
            v = getattr(params, k)
            if k in ("obs_center", "boundary_center"):
                for a in range(3):
                    getattr(c, k)[a] = float(v[a])
            else:
                setattr(c, k, v)
        self.params = params
        h = C.c_void_p()
        sp = None if stream is None else C.c_void_p(stream.cuda_stream)
        self._keep = []
        st = self.L.crp_create(C.byref(c), sp, C.byref(h))
        if st != OK:
            raise CrpError(st, "crp_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.crp_destroy(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st, ok=(OK,)):
        if st not in ok:
            msg = self.L.crp_last_error(self.h)
            raise CrpError(st, msg.decode() if msg else "")
        return st

    # -- inputs -------------------------------------------------------------
    def set_field_grid(self, grid, spacing, origin=(0.0, 0.0, 0.0)):
        """grid: [nx][ny][nz][3] float32/float64 numpy array (copied) or a
        contiguous torch device tensor (used in place; kept alive here)."""
        on_dev = _is_dev(grid)
        if on_dev:
            import torch
            dt = F32 if grid.dtype == torch.float32 else F64
            _dev(grid, np.float32 if dt == F32 else np.float64, (None, None, None, 3), "grid",
                 self.params.device)
            self._keep = [grid]
        else:
            dt = F32 if np.asarray(grid).dtype == np.float32 else F64
            grid = _host(grid, np.float32 if dt == F32 else np.float64, (None, None, None, 3),
                         "grid")
        org = (C.c_double * 3)(*[float(v) for v in origin])
        self._check(self.L.crp_set_field_grid(self.h, _ptr(grid), dt, int(on_dev),
                                              grid.shape[0], grid.shape[1], grid.shape[2],
                                              float(spacing), org))
        self._grid_dtype = np.float32 if dt == F32 else np.float64

    def set_field_patches(self, patches):
        """Refinement patches of the grid: dicts with data ([n0][n1][n2][3] numpy
        array, copied, or a contiguous torch device tensor, used in place and
        kept alive here), offset (base vertex index) and refine.  Patch values
        have the base grid's type (host arrays are converted to it)."""
        gdt = getattr(self, "_grid_dtype", np.float64)
        arr = (GridPatch * max(len(patches), 1))()
        keep = []
        for k, q in enumerate(patches):
            d = q["data"]
            on_dev = _is_dev(d)
            if on_dev:
                d = _dev(d, gdt, (None, None, None, 3), f"patch {k}", self.params.device)
            else:
                d = _host(d, gdt, (None, None, None, 3), f"patch {k}")
            keep.append(d)
            arr[k].data = _ptr(d)
            for a in range(3):
                arr[k].n[a] = int(d.shape[a])
                arr[k].offset[a] = int(q["offset"][a])
            arr[k].refine = int(q["refine"])
            arr[k].on_device = int(on_dev)
        self._check(self.L.crp_set_field_patches(self.h, len(patches), arr))
        self._patches_keep = [d for d in keep if hasattr(d, "is_cuda")]

    def set_field_analytic(self, model):
        """The analytic galactic field: a dict with center (3, m), b_disk, r_disk,
        h_disk, b_halo, r_halo, h_halo, b_x, r_x, h_x (tesla, metres)."""
        f = AnalyticField()
        for a in range(3):
            f.center[a] = float(model["center"][a])
        for k, _ in AnalyticField._fields_[1:]:
            setattr(f, k, float(model[k]))
        self._check(self.L.crp_set_field_analytic(self.h, C.byref(f)))

    def set_tables(self, tables):
        n = len(tables.e_nodes)
        arrs = [_host(a, np.float64, (n,), "tables") for a in
                (tables.e_nodes, tables.t_pi, tables.t_n, tables.beta_p)]
        self._check(self.L.crp_set_tables(self.h, len(arrs[0]), *[_ptr(a) for a in arrs]))

    def inject(self, inj=None, *, id=None, A=None, Z=None, E=None, pos=None, dir=None,
               lmax=None, on_device=False):
        if inj is not None:
            id, A, Z, E, pos, dir, lmax = inj.id, inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax
        n = int(len(id))
        spec = ((id, np.uint32, (n,), "id"), (A, np.int32, (n,), "A"), (Z, np.int32, (n,), "Z"),
                (E, np.float64, (n,), "E"), (pos, np.float64, (n, 3), "pos"),
                (dir, np.float64, (n, 3), "dir"), (lmax, np.float64, (n,), "lmax"))
        if on_device:
            arrs = [_dev(a, dt, sh, w, self.params.device) for a, dt, sh, w in spec]
        else:
            arrs = [_host(a, dt, sh, w) for a, dt, sh, w in spec]
        self._check(self.L.crp_inject(self.h, n, *[_ptr(a) for a in arrs], int(on_device)))

    # -- the hot path ---------------------------------------------------------
    def propagate(self, max_cycles=0):
        """Returns True when complete, False when candidates remain pending.
        Raises CrpError with status EOVERFLOW when candidates wait for room in
        the full neutral-record buffer: read neutral records, then call again
        (nothing is lost)."""
        st = self._check(self.L.crp_propagate(self.h, int(max_cycles)), ok=(OK, INCOMPLETE))
        return st == OK

    # -- outputs ------------------------------------------------------------
    def counts(self):
        c = Counters()
        self._check(self.L.crp_counts(self.h, C.byref(c)))
        return {k: getattr(c, k) for k in COUNT_FIELDS}

    def reset_counters(self):
        self._check(self.L.crp_reset_counters(self.h))

    def read_finished(self, cap=None):
        cap = self.counts()["finished_unread"] if cap is None else cap
        arrs = _alloc(FIN_FIELDS, cap)
        s = _fill(FinishedSoA, arrs)
        n = C.c_int64(0)
        self._check(self.L.crp_read_finished(self.h, cap, C.byref(s), C.byref(n)),
                    ok=(OK, EOVERFLOW))
        return {k: v[:n.value] for k, v in arrs.items()}

    def discard_finished(self):
        n = C.c_int64(0)
        self._check(self.L.crp_read_finished(self.h, 1 << 62, None, C.byref(n)),
                    ok=(OK, EOVERFLOW))
        m = C.c_int64(0)
        self._check(self.L.crp_read_neutral(self.h, 1 << 62, None, C.byref(m)),
                    ok=(OK, EOVERFLOW))
        return n.value, m.value

    def read_neutral(self, cap=None):
        cap = self.counts()["neutral_unread"] if cap is None else cap
        arrs = _alloc(NEU_FIELDS, cap)
        s = _fill(NeutralSoA, arrs)
        n = C.c_int64(0)
        self._check(self.L.crp_read_neutral(self.h, cap, C.byref(s), C.byref(n)),
                    ok=(OK, EOVERFLOW))
        return {k: v[:n.value] for k, v in arrs.items()}

    def read_trajectory(self, cap=None):
        """Trajectory points (dict: id, lineage, n, A, L, E, x [n][3])."""
        cap = self.counts()["traj_unread"] if cap is None else cap
        arrs = _alloc(TRAJ_FIELDS, cap)
        s = _fill(TrajSoA, arrs)
        n = C.c_int64(0)
        self._check(self.L.crp_read_trajectory(self.h, cap, C.byref(s), C.byref(n)),
                    ok=(OK, EOVERFLOW))
        return {k: v[:n.value] for k, v in arrs.items()}

    def discard_trajectory(self):
        n = C.c_int64(0)
        self._check(self.L.crp_read_trajectory(self.h, 1 << 62, None, C.byref(n)),
                    ok=(OK, EOVERFLOW))
        return n.value

    # -- observables ----------------------------------------------------------
    def set_observables(self, spec):
        """spec: dict with e_edges, a_edges, status_mask, sky_n, sky_sign, e_ref,
        gamma (the fields of crp_observables); clears the sums."""
        ee = np.ascontiguousarray(spec["e_edges"], np.float64)
        ae = np.ascontiguousarray(spec["a_edges"], np.int32)
        o = Observables(len(ee) - 1, len(ae) - 1, ee.ctypes.data_as(_P(C.c_double)),
                        ae.ctypes.data_as(_P(C.c_int32)), int(spec["status_mask"]),
                        int(spec["sky_n"]), float(spec["sky_sign"]), float(spec["e_ref"]),
                        float(spec["gamma"]))
        self._check(self.L.crp_set_observables(self.h, C.byref(o)))
        self._obs_shape = (len(ae) - 1, len(ee) - 1, 6 * int(spec["sky_n"]) ** 2)

    def observe(self):
        """Adds the unread finished records to the sums; returns the kernel ms."""
        ms = C.c_double(0)
        self._check(self.L.crp_observe(self.h, C.byref(ms)))
        return ms.value

    def read_observables(self):
        if getattr(self, "_obs_shape", None) is None:      # the library reports the state
            self._check(self.L.crp_read_observables(self.h, None, None, None, None, None))
        ng, ne, npix = self._obs_shape
        out = dict(counts=np.zeros((ng, ne), np.uint64), wsum=np.zeros((ng, ne)),
                   defl=np.zeros((ng, ne), np.uint64), sky=np.zeros((ng, ne, npix), np.uint64))
        outside = np.zeros(1, np.uint64)
        self._check(self.L.crp_read_observables(self.h, _ptr(out["counts"]), _ptr(out["wsum"]),
                                                _ptr(out["defl"]), _ptr(out["sky"]),
                                                _ptr(outside)))
        out["outside"] = int(outside[0])
        return out

    # -- galactic lenses --------------------------------------------------------
    def lens_build(self, spec):
        """spec: dict with r_edges, sky_n, status_mask.  Returns (nnz, ms)."""
        re_ = np.ascontiguousarray(spec["r_edges"], np.float64)
        ls = LensSpec(len(re_) - 1, int(spec["sky_n"]), re_.ctypes.data_as(_P(C.c_double)),
                      int(spec["status_mask"]), 0)
        nnz = C.c_int64(0)
        ms = C.c_double(0)
        self._check(self.L.crp_lens_build(self.h, C.byref(ls), C.byref(nnz), C.byref(ms)))
        self._lens_shape = (len(re_) - 1, 6 * int(spec["sky_n"]) ** 2, nnz.value)
        return nnz.value, ms.value

    def lens_read(self):
        if getattr(self, "_lens_shape", None) is None:     # the library reports the state
            self._check(self.L.crp_lens_read(self.h, None, None, None, None))
        nr, npix, nnz = self._lens_shape
        out = dict(rowptr=np.zeros(nr * npix + 1, np.int64), col=np.zeros(nnz, np.int32),
                   val=np.zeros(nnz), count=np.zeros(nnz, np.uint64))
        self._check(self.L.crp_lens_read(self.h, _ptr(out["rowptr"]), _ptr(out["col"]),
                                         _ptr(out["val"]), _ptr(out["count"])))
        out.update(npix=npix, n_r=nr)
        return out

    def lens_apply(self, x, y=None):
        """x: [n_maps][n_r][Np] float64 numpy array (or a torch device tensor,
        then y too).  Returns (y, kernel ms)."""
        if getattr(self, "_lens_shape", None) is None:
            self._check(self.L.crp_lens_apply(self.h, 0, None, None, 0, None))
        nr, npix, _ = self._lens_shape
        shape = (None, nr, npix)
        on_dev = _is_dev(x)
        if on_dev:
            import torch
            x = _dev(x, np.float64, shape, "x", self.params.device)
            y = torch.empty_like(x) if y is None else y
            _dev(y, np.float64, tuple(x.shape), "y", self.params.device)
        else:
            x = _host(x, np.float64, shape, "x")
            y = np.empty_like(x)
        ms = C.c_double(0)
        self._check(self.L.crp_lens_apply(self.h, int(x.shape[0]), _ptr(x), _ptr(y),
                                          int(on_dev), C.byref(ms)))
        return y, ms.value

    def peek_pending(self, cap=None):
        cap = self.counts()["pending"] if cap is None else cap
        arrs = _alloc(FIN_FIELDS, cap)
        s = _fill(FinishedSoA, arrs)
        n = C.c_int64(0)
        self._check(self.L.crp_peek_pending(self.h, cap, C.byref(s), C.byref(n)))
        return {k: v[:n.value] for k, v in arrs.items()}

    def eval_field(self, pos, mode=FP64):
        on_dev = _is_dev(pos)
        if on_dev:
            import torch
            pos = _dev(pos, np.float64, (None, 3), "pos", self.params.device)
            out = torch.empty_like(pos)
        else:
            pos = _host(np.asarray(pos, np.float64).reshape(-1, 3), np.float64, (None, 3), "pos")
            out = np.empty_like(pos)
        self._check(self.L.crp_eval_field(self.h, pos.shape[0], _ptr(pos), _ptr(out), mode,
                                          int(on_dev)))
        return out

    def eval_field_noalloc(self, pos, mode=FP64, out=None):
        """crp_eval_field for host arrays through the library's static staging
        (no device allocation; at most EVAL_NOALLOC_MAX points).  `out`, if
        given, is a C-contiguous float64 [n][3] array written in place."""
        pos = _host(np.asarray(pos, np.float64).reshape(-1, 3), np.float64, (None, 3), "pos")
        if out is None:
            out = np.empty_like(pos)
        elif not (isinstance(out, np.ndarray) and out.dtype == np.float64 and
                  out.flags.c_contiguous and out.shape == pos.shape):
            raise ValueError("out: a C-contiguous float64 [n][3] host array is expected")
        self._check(self.L.crp_eval_field_noalloc(self.h, pos.shape[0], _ptr(pos), _ptr(out),
                                                  mode))
        return out

    # -- launch shape / tuning / timing ---------------------------------------
    def set_launch(self, block=128, blocks_per_cu=0, refill=4, layout=LAYOUT_LINEAR):
        lch = Launch(block, blocks_per_cu, refill, layout)
        self._check(self.L.crp_set_launch(self.h, C.byref(lch)))

    def get_launch(self):
        lch = Launch()
        self._check(self.L.crp_get_launch(self.h, C.byref(lch)))
        return lch.as_dict()

    def tune(self, max_cycles=64, cache_path=None):
        best = Launch()
        rate = C.c_double(0)
        cp = cache_path.encode() if cache_path else None
        self._check(self.L.crp_tune(self.h, int(max_cycles), cp, C.byref(best), C.byref(rate)))
        return best.as_dict(), rate.value

    def last_timing(self):
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._check(self.L.crp_last_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # -- checkpoint -----------------------------------------------------------
    def gather_ceiling(self, iters=2000):
        """Records/s of the cooperative field gather alone (diagnostic)."""
        r = C.c_double(0)
        self._check(self.L.crp_gather_ceiling(self.h, int(iters), C.byref(r)))
        return r.value

    def snapshot(self) -> bytes:
        p = C.c_void_p()
        n = C.c_size_t(0)
        self._check(self.L.crp_snapshot(self.h, C.byref(p), C.byref(n)))
        try:
            return C.string_at(p, n.value)
        finally:
            self.L.crp_free(p)

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.L.crp_restore(self.h, buf, len(blob)))

    # -- neural field ---------------------------------------------------------
    def nf_init(self, freq, params, b_scale):
        f = _host(freq, np.int32, (64, 3), "freq")
        p = _host(params, np.float32, (NF_NPARAM,), "params")
        self._check(self.L.crp_nf_init(self.h, _ptr(f), _ptr(p), float(b_scale)))

    def nf_get_params(self):
        p = np.empty(NF_NPARAM, np.float32)
        self._check(self.L.crp_nf_get_params(self.h, _ptr(p)))
        return p

    def nf_loss_grad(self, pos, target):
        pos = _host(np.asarray(pos, np.float64).reshape(-1, 3), np.float64, (None, 3), "pos")
        t = _host(np.asarray(target, np.float32).reshape(-1, 3), np.float32,
                  (pos.shape[0], 3), "target")
        out = np.empty(t.shape, np.float32)
        g = np.empty(NF_NPARAM, np.float32)
        loss = C.c_double(0)
        self._check(self.L.crp_nf_loss_grad(self.h, pos.shape[0], _ptr(pos), _ptr(t), _ptr(out),
                                            _ptr(g), C.byref(loss)))
        return out, g, loss.value

    def nf_adam_step(self, grad, lr):
        g = _host(grad, np.float32, (NF_NPARAM,), "grad")
        self._check(self.L.crp_nf_adam_step(self.h, _ptr(g), float(lr)))

    def nf_train(self, steps, batch, lr0, lr1, seed):
        losses = np.empty(max(int(steps), 1), np.float32)
        self._check(self.L.crp_nf_train(self.h, int(steps), int(batch), float(lr0), float(lr1),
                                        int(seed), _ptr(losses)))
        return losses[:steps]


def params_for(workload, precision=FP64, **kw):
    """Params matching a workload description (see crp_inputs.Workload)."""
    p = Params(precision=precision, tol=workload.tol, hmin=workload.hmin_m,
               hmax=workload.hmax_m, obs_center=workload.observer,
               obs_radius=workload.obs_radius_m, seed=workload.philox_seed,
               charge_sign=workload.charge_sign, boundary_center=workload.boundary_center,
               boundary_radius=workload.boundary_radius_m,
               field_mode=FIELD_ANALYTIC if workload.field == "analytic" else FIELD_GRID)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def sort_finished(fin):
    order = np.lexsort((fin["lineage"], fin["id"]))
    return {k: v[order] for k, v in fin.items()}


def sort_traj(tr):
    order = np.lexsort((tr["n"], tr["lineage"], tr["id"]))
    return {k: v[order] for k, v in tr.items()}


def sort_neutral(neu):
    order = np.lexsort((neu["m"], neu["lineage"], neu["id"]))
    return {k: v[order] for k, v in neu.items()}
