"""Comparison helpers shared by the GPU parity tests (GPU records versus the
oracle's records for the same candidates)."""
import sys

import numpy as np

INT_FIELDS = ("id", "lineage", "m", "nsteps", "nrej", "status", "A", "Z")
CNT_KEYS = ("finished", "observed", "max_traj", "energy_floor", "steps", "attempts", "rejects",
            "forced", "events", "null_events", "inter_pi", "inter_n", "charged_sec",
            "neutral_sec")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_ctx(P, w, grid, tables, precision, qcap=1 << 16, ncap=1 << 16, **kw):
    prm = P.params_for(w, precision, queue_capacity=qcap, neutral_capacity=ncap, **kw)
    ctx = P.Context(prm)
    ctx.set_field_grid(grid, w.spacing_m)
    ctx.set_tables(tables)
    return ctx


def run_gpu(ctx, inj, max_cycles=0):
    ctx.inject(inj)
    done = ctx.propagate(max_cycles)
    return done, ctx.read_finished(), ctx.read_neutral(), ctx.counts()


def compare_records(fg, fo, what, x_tol=1e-9, e_tol=1e-6):
    from paper_1307_2643_amd import crp
    fg = crp.sort_finished(fg)
    fo = crp.sort_finished(fo)
    assert len(fg["id"]) == len(fo["id"]), what
    for k in INT_FIELDS:
        bad = np.nonzero(fg[k] != fo[k])[0]
        assert bad.size == 0, f"{what}: field {k} differs at {bad[:5]}"
    scale = np.maximum(fo["L"], np.linalg.norm(fo["x"], axis=1))
    dx = np.linalg.norm(fg["x"] - fo["x"], axis=1)
    assert np.all(dx <= x_tol * np.maximum(scale, 1.0)), f"{what}: max dx/scale {np.max(dx / scale)}"
    assert np.all(np.abs(fg["E"] / fo["E"] - 1) <= e_tol), what
    assert np.all(np.abs(fg["L"] - fo["L"]) <= x_tol * np.maximum(fo["L"], 1.0)), what
    assert np.all(np.linalg.norm(fg["u"] - fo["u"], axis=1) <= 1e-7), what
    same = np.all(fg["x"] == fo["x"], axis=1) & np.all(fg["u"] == fo["u"], axis=1) & \
        (fg["E"] == fo["E"]) & (fg["L"] == fo["L"])
    say(f"{what}: {len(fg['id'])} records, bitwise identical {same.sum()} "
        f"({100.0 * same.mean():.3f}%)")
    return same


def compare_neutral(ng, no, what):
    from paper_1307_2643_amd import crp
    ng = crp.sort_neutral(ng)
    no = crp.sort_neutral(no)
    assert len(ng["id"]) == len(no["id"]), what
    for k in ("id", "lineage", "m", "chan"):
        assert np.array_equal(ng[k], no[k]), f"{what}: {k}"
    assert np.allclose(ng["E"], no["E"], rtol=1e-6, atol=0), what
    assert np.allclose(ng["x"], no["x"], rtol=0, atol=1e-9 * 1e26), what


def compare_counts(cg, co, what):
    for k in CNT_KEYS:
        assert cg[k] == co[k], f"{what}: count {k}: gpu {cg[k]} oracle {co[k]}"
