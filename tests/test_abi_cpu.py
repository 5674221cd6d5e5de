"""CPU-side checks of the C-ABI library: it loads, exports every function that
include/crp.h declares, and the binding marshals the declared structs with the
same sizes as the header (no compute calls: there is no GPU here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(crp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("crp_create", "crp_set_field_grid", "crp_set_tables", "crp_inject",
                 "crp_propagate", "crp_read_finished", "crp_read_neutral", "crp_counts",
                 "crp_eval_field", "crp_snapshot", "crp_restore", "crp_tune", "crp_nf_train"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1307_2643_amd import crp
    lib = crp.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    assert set(declared_functions()) == set(crp.EXPORTS)


def test_library_is_built_for_gfx950():
    """The library built here embeds a gfx950 code object."""
    from paper_1307_2643_amd import crp
    blob = open(crp.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def _c_struct_size(decl, name):
    """Size of a struct from crp.h as compiled by the host C compiler."""
    prog = '#include "crp.h"\n#include <stdio.h>\nint main(void){printf("%%zu", sizeof(%s));}\n' % name
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), src, "-o", exe])
        return int(subprocess.check_output([exe]).decode())


@pytest.mark.parametrize("cname,pyname", [("crp_config", "Config"), ("crp_launch", "Launch"),
                                          ("crp_finished_soa", "FinishedSoA"),
                                          ("crp_neutral_soa", "NeutralSoA"),
                                          ("crp_counters", "Counters"),
                                          ("crp_analytic_field", "AnalyticField"),
                                          ("crp_traj_soa", "TrajSoA"),
                                          ("crp_observables", "Observables"),
                                          ("crp_grid_patch", "GridPatch"),
                                          ("crp_lens_spec", "LensSpec")])
def test_binding_struct_sizes_match_header(cname, pyname):
    from paper_1307_2643_amd import crp
    assert C.sizeof(getattr(crp, pyname)) == _c_struct_size(HEADER, cname)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1307_2643_amd import crp
    monkeypatch.setattr(crp, "_lib", None)
    monkeypatch.setattr(crp, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        crp.load()


def test_create_rejects_bad_configs_before_any_device_call():
    """crp_create validates the configuration on the host: every bad field is
    CRP_EINVAL without touching a device (a good one reaches the device, which
    this container lacks: CRP_EDEVICE, or a context where there is a GPU)."""
    import math
    from paper_1307_2643_amd import crp
    lib = crp.load()

    def status(**kw):
        p = crp.Params()
        for k, v in kw.items():
            setattr(p, k, v)
        c = crp.Config()
        for k, _ in crp.Config._fields_:
            v = getattr(p, k)
            if k in ("obs_center", "boundary_center"):
                for a in range(3):
                    getattr(c, k)[a] = float(v[a])
            else:
                setattr(c, k, v)
        h = C.c_void_p()
        st = lib.crp_create(C.byref(c), None, C.byref(h))
        if h.value:
            lib.crp_destroy(h)
        return st

    bad = [dict(precision=2), dict(field_mode=7), dict(charge_sign=2), dict(tol=0.0),
           dict(tol=math.inf), dict(hmin=0.0), dict(hmax=1.0), dict(hmax=math.inf),
           dict(eps_loss=math.nan), dict(kappa_pi=1.0), dict(e_floor=math.inf),
           dict(obs_radius=-1.0), dict(obs_center=(0.0, math.nan, 0.0)),
           dict(boundary_radius=math.inf), dict(queue_capacity=0),
           dict(neutral_capacity=(1 << 40) + 1), dict(traj_every=1, traj_capacity=0),
           dict(field_mode=crp.FIELD_NEURAL, precision=crp.FP64), dict(inject_order=2),
           dict(inject_order=-1)]
    for kw in bad:
        assert status(**kw) == -1, kw
    assert status() in (0, -2)
