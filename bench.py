"""Benchmark of the propagation hot path on one MI355X.

One bench step = inject one batch of synthetic candidates (already resident in
HBM) and propagate every candidate and spawned secondary to completion.  The
workload is the 1024^3 FP32 turbulent grid (10 kpc cells, 1 nG RMS) with 1e7
mixed H/He/N/Fe candidates on an E^-2 spectrum from the origin, interaction
and loss tables, a 1 Mpc observer at (50,0,0) Mpc and a 100 Mpc trajectory
limit.  The headline value is accepted candidate-steps per second of the
precision form; the FP64 method on the same grid is timed beside it, and the
precision form's error against the FP64 oracle is reported on a sample.

    python bench.py [--steps K] [--warmup W] [--n CANDIDATES] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GATHERS_PER_ATTEMPT = 6
RECORD_BYTES = 8 * 3 * 4          # algorithmic bytes of one gather: 8 corners x 3 x FP32
RECORD_BYTES_FP64 = 8 * 3 * 8     # the same for an FP64 grid
TUNE_CYCLES_FP64 = 256
TUNE_N_HEADLINE = 5_000_000       # candidates of the timed batch the headline's tuning runs            # cycles per autotuner trial on the FP64-grid workloads


def gathers(cnt):
    """Field gathers of a run: six per Cash-Karp attempt, except that the retry
    after a rejection keeps the first-stage field of its unchanged position
    (one gather fewer per rejected attempt)."""
    return GATHERS_PER_ATTEMPT * cnt["attempts"] - cnt["rejects"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("crp_device.hpp", "crp_kernels.hip", "crp_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1307_2643_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="candidates per batch (default 1e7)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-method variant")
    ap.add_argument("--launch", type=str, default=None,
                    help="force the launch shape BLOCK,BLOCKS_PER_CU,REFILL,LAYOUT (no tuner)")
    ap.add_argument("--no-sample", action="store_true",
                    help="skip the error sample against the oracle")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration)")
    ap.add_argument("--summarize-pmc", type=str, default=None, metavar="DIR",
                    help="offline: per-launch HBM traffic from rocprofv3 --pmc CSV output")
    ap.add_argument("--pmc-kernel", type=str, default=None,
                    help="with --summarize-pmc: kernel-name prefix of the instantiation to "
                         "summarize (default: the headline's)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-nf", action="store_true", help="skip the neural-field variant")
    ap.add_argument("--nf-candidates", type=int, default=1_000_000)
    ap.add_argument("--nf-narrow-steps", type=int, default=45780,
                    help="training steps of the network on the narrow-band field "
                         "(45780 steps = 3e9 points; 0 skips that point)")
    ap.add_argument("--nf-steps", type=int, default=1526,
                    help="training steps of 65536 points (1526 steps = 1e8 points)")
    ap.add_argument("--no-outputs", action="store_true",
                    help="skip the output-module variants (trajectory points, observables)")
    ap.add_argument("--no-nested", action="store_true",
                    help="skip the multi-resolution grid variant")
    ap.add_argument("--no-galactic", action="store_true",
                    help="skip the galactic backtracking variant (analytic field)")
    ap.add_argument("--gal-n", type=int, default=10_000_000)
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper-shaped context run (protons, 1 Gpc, 256^3 grid)")
    ap.add_argument("--paper-n", type=int, default=1_000_000)
    ap.add_argument("--nf-only", action="store_true",
                    help="diagnostic: only the neural-field variant (training, field error, "
                         "surrogate vs grid); prints that variant's JSON")
    ap.add_argument("--batching", type=int, default=10, metavar="NBATCH",
                    help="batches of 1e7 candidates at distances 1..1000 Mpc in the batching "
                         "form (10 = the 1e8-candidate stream; 0 skips it)")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="autotuner cache file (default: a new file for this run); the "
                         "headline's shape is kept in FILE.headline, the batching form's and "
                         "the FP64-grid workloads' in FILE")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the FP64 lines of the 32^3 and 256^3 workloads")
    ap.add_argument("--fp64-grid-only", action="store_true",
                    help="diagnostic: only the FP64 lines of the 32^3 and 256^3 workloads "
                         "(for profiling them); prints their JSON")
    ap.add_argument("--fp64-launch", type=str, default=None,
                    help="force the launch of the FP64-grid workloads "
                         "BLOCK,BLOCKS_PER_CU,REFILL,LAYOUT (no tuner)")
    ap.add_argument("--nf-sweep", type=str, default=None, metavar="NMAX,..:STEPS,..:LR",
                    help="diagnostic: neural-field RMS error on the 1024^3 grid against the "
                         "field band's n_max (band 2..n_max cycles per box) and the training "
                         "length (steps of 65536 points, one cosine schedule each, from lr LR "
                         "to 1e-5); one JSON line per point")
    args = ap.parse_args()
    if args.tune_cache is None:
        import tempfile
        args.tune_cache = os.path.join(tempfile.mkdtemp(prefix="crp_bench_"), "tune_cache.txt")

    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.pmc_kernel)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the propagation "
              "shards by candidate id across GPUs without communication, but this build "
              "measures one GPU's share.", file=sys.stderr)
        sys.exit(2)

    import torch

    import crp_inputs as I
    from paper_1307_2643_amd import crp

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)                       # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b

    if args.nf_sweep:
        nf_sweep(args.nf_sweep, crp, I, torch, dev, stream)
        return

    if args.fp64_grid_only:
        out = {"fp64_grid32": small_config_variant(args, crp, I, torch, stream, I.W_SMALL, None),
               "fp64_grid256": small_config_variant(args, crp, I, torch, stream, I.W_MIXED256,
                                                    10_000)}
        print(json.dumps({"variant": "fp64_grid", **out}), flush=True)
        return

    w = I.W_MIXED1024
    n = args.n or w.n_candidates
    log(f"[bench] workload {w.name}: n={n}, grid {w.grid_n}^3 fp32")
    t0 = time.time()
    grid = w.make_grid(device=dev)                     # [1024]^3 x 3 float32, 12.9 GB
    torch.cuda.synchronize()
    log(f"[bench] grid generated in {time.time() - t0:.1f}s")
    tables = w.make_tables()
    inj = w.make_injection(n)
    d_inj = [torch.as_tensor(a, device=dev) for a in
             (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]

    if args.nf_only:
        lch = dict(block=128, blocks_per_cu=4, refill=32, layout=1)
        if args.launch:
            b, bpc, rf, lay = [int(v) for v in args.launch.split(",")]
            lch = dict(block=b, blocks_per_cu=bpc, refill=rf, layout=lay)
        nf = neural_variant(args, crp, I, torch, w, grid, tables, stream, lch)
        print(json.dumps({"variant": "nf", **nf}), flush=True)
        return

    def context(precision, **kw):
        prm = crp.params_for(w, precision, device=0, queue_capacity=2 * n,
                             neutral_capacity=max(n, 1 << 20), **kw)
        ctx = crp.Context(prm, stream)
        ctx.set_field_grid(grid, w.spacing_m)
        ctx.set_tables(tables)
        return ctx

    def inject(ctx, count=None):
        if count is None:
            ctx.inject(id=d_inj[0], A=d_inj[1], Z=d_inj[2], E=d_inj[3], pos=d_inj[4],
                       dir=d_inj[5], lmax=d_inj[6], on_device=True)
        else:
            ctx.inject(id=d_inj[0][:count], A=d_inj[1][:count], Z=d_inj[2][:count],
                       E=d_inj[3][:count], pos=d_inj[4][:count], dir=d_inj[5][:count],
                       lmax=d_inj[6][:count], on_device=True)

    # ---- precision form: tune (untimed), warm up, time K steps ---------------
    ctx = context(crp.MIX)
    tuned = None
    if args.launch:
        b, bpc, rf, lay = [int(v) for v in args.launch.split(",")]
        ctx.set_launch(block=b, blocks_per_cu=bpc, refill=rf, layout=lay)
    elif not args.no_tune:
        t0 = time.time()
        # the timed workload's own launch: the autotuner on the batch's first
        # TUNE_N_HEADLINE candidates (the same mix, spectrum and field), every
        # trial run to completion, tail and secondaries included; its cache file
        # is its own (the batching form tunes on its own distribution)
        inject(ctx, min(TUNE_N_HEADLINE, n))
        tuned, rate = ctx.tune(max_cycles=0, cache_path=args.tune_cache + ".headline")
        while not ctx.propagate(0):
            pass
        ctx.discard_finished()
        log(f"[bench] autotuner picked {tuned} ({rate:.3e} steps/s on the batch's first "
            f"{min(TUNE_N_HEADLINE, n)} candidates) in {time.time() - t0:.1f}s")
    launch = ctx.get_launch()

    def one_step(c):
        inject(c)
        c.propagate(0)
        ms, nl = c.last_timing()
        cnt = c.counts()
        c.discard_finished()
        return ms, cnt

    for i in range(args.warmup):
        ctx.reset_counters()
        ms, cnt = one_step(ctx)
        log(f"[bench] warmup {i}: kernel {ms:.1f} ms, {cnt['steps']} steps")
    ctx.reset_counters()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ms, cnt = one_step(ctx)
        kms.append(ms)
        log(f"[bench] step {i}: kernel {ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = ctx.counts()
    steps_total = cnt["steps"]
    attempts_total = cnt["attempts"]
    value = steps_total / wall
    ms_per_step = 1000.0 * wall / args.steps
    kernel_ms = sum(kms) / len(kms)
    attempts_per_launch = attempts_total / args.steps
    gathers_per_launch = gathers(cnt) / args.steps
    alg_bytes = gathers_per_launch * RECORD_BYTES
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    log(f"[bench] precision form: {value:.4e} steps/s, {ms_per_step:.1f} ms/step, "
        f"kernel {kernel_ms:.1f} ms, {achieved:.1f} GB/s algorithmic")

    # ---- the same step across the host boundary (not the headline) ---------
    # host arrays in, finished and neutral records back to host arrays: the
    # rate a caller that keeps its data on the host sees (PCIe and host-side
    # record conversion included)
    ctx.reset_counters()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.inject(inj)
    ctx.propagate(0)
    hf = ctx.read_finished()
    hn = ctx.read_neutral()
    torch.cuda.synchronize()
    host_wall = time.perf_counter() - t1
    host_rate = ctx.counts()["steps"] / host_wall
    log(f"[bench] across the host boundary: {host_rate:.4e} steps/s ({host_wall:.2f} s, "
        f"{len(hf['id'])} finished and {len(hn['id'])} neutral records read back)")
    del hf, hn

    # ---- a plain device copy: the HBM bandwidth this machine reaches -----------
    copy_gbs = copy_bandwidth(torch, dev)
    log(f"[bench] device copy of 4 GiB: {copy_gbs:.0f} GB/s (read + write)")

    # ---- the gather pattern alone on the same corner records (diagnostic) ---
    ceiling = None
    if launch["layout"] == crp.LAYOUT_CORNER:
        rec_s = ctx.gather_ceiling(20000)
        ceiling = {"records_per_s": rec_s, "algorithmic_GBps": rec_s * RECORD_BYTES / 1e9,
                   "line_GBps": rec_s * 128 / 1e9,
                   "kernel_frac_of_ceiling": achieved / (rec_s * RECORD_BYTES / 1e9)}
        log(f"[bench] gather pattern alone: {rec_s:.3e} records/s = "
            f"{rec_s * RECORD_BYTES / 1e9:.0f} GB/s algorithmic ({rec_s * 128 / 1e9:.0f} GB/s "
            f"in 128-byte lines); the propagation gathers "
            f"{gathers_per_launch / (kernel_ms * 1e-3):.3e} records/s")

    # ---- sample for the stated error: MIX (GPU) vs FP64 oracle --------------
    nsample = 0 if args.no_sample else min(n, 10_000)   # the 1e4-candidate error subset
    horizon = 16
    if nsample:
        ctx.reset_counters()
        inject(ctx, nsample)
        ctx.propagate(0)
        mix_fin = crp.sort_finished(ctx.read_finished())
        ctx.discard_finished()
        # the same candidates after their first `horizon` cycles
        inject(ctx, nsample)
        ctx.propagate(horizon)
        part = ctx.read_finished()
        pend = ctx.peek_pending()
        mix_short = crp.sort_finished({k: np.concatenate([part[k], pend[k]]) for k in part})
        while not ctx.propagate(0):
            pass
        ctx.discard_finished()
    ctx.close()

    variants = {"mix": {"steps_per_s": value, "kernel_ms": kernel_ms, "launch": launch,
                        "attempts_per_launch": attempts_per_launch,
                        "lane_utilisation": attempts_total / max(cnt["lane_slots"], 1),
                        "host_boundary_steps_per_s": host_rate}}

    # ---- FP64 method on the same FP32 grid ("plain grid") ----------------------
    fp64_fin = None
    if not args.no_fp64:
        c64 = context(crp.FP64)
        c64.set_launch(**launch)
        one_step(c64)                    # untimed: builds this context's grid records
        c64.reset_counters()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms64, cnt64 = one_step(c64)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t1
        variants["fp64"] = {"steps_per_s": cnt64["steps"] / wall64, "kernel_ms": ms64}
        log(f"[bench] FP64 method: {cnt64['steps'] / wall64:.4e} steps/s")
        if nsample:
            c64.reset_counters()
            inject(c64, nsample)
            c64.propagate(0)
            fp64_fin = crp.sort_finished(c64.read_finished())
        c64.close()

    # ---- output modules: per-step trajectory points and observables ---------
    if not args.no_outputs:
        variants["outputs"] = outputs_variant(args, crp, w, n, context, inject, launch, value)

    # ---- multi-resolution grid: a refined patch inside the 1024^3 grid -------
    if not args.no_nested:
        variants["nested"] = nested_variant(args, crp, I, torch, w, n, grid, tables, stream, inj)

    # ---- CPU oracle baseline and error of the precision form ----------------
    cpu = None
    err = None
    if not args.no_cpu and nsample:
        from oracle import oracle as O
        host_grid = grid.cpu().numpy()
        G = O.GridRef(host_grid, w.spacing_m)
        T = O.TablesRef(tables)
        threads = len(os.sched_getaffinity(0))
        fo, _, co, used = O.propagate(O.config_for(w), G, T, inj.subset(slice(0, nsample)),
                                      nthreads=threads)
        fo = O.sort_finished(fo)
        err = {"full_run": error_report(mix_fin, fo)}
        fs, _, _, _ = O.propagate(O.config_for(w, max_cycles=horizon), G, T,
                                  inj.subset(slice(0, nsample)), nthreads=threads)
        err[f"after_{horizon}_cycles"] = error_report(mix_short, O.sort_finished(fs))
        if fp64_fin is not None:
            if len(fp64_fin["id"]) == len(fo["id"]):
                same = int(np.sum(np.all(fp64_fin["x"] == fo["x"], axis=1) &
                                  (fp64_fin["E"] == fo["E"])))
                err["fp64_gpu_vs_fp64_oracle_bitwise"] = f"{same}/{len(fo['id'])}"
            else:
                err["fp64_gpu_vs_fp64_oracle_bitwise"] = "record counts differ"
        # time the oracle's precision form on a bounded sample of the workload
        probe = 256
        t1 = time.perf_counter()
        _, _, cp, used = O.propagate(O.config_for(w, precision=O.MIX), G, T,
                                     inj.subset(slice(0, probe)), nthreads=threads)
        tp = time.perf_counter() - t1
        m = int(min(n, max(probe, probe * args.cpu_seconds / max(tp, 1e-3))))
        t1 = time.perf_counter()
        _, _, cp, used = O.propagate(O.config_for(w, precision=O.MIX), G, T,
                                     inj.subset(slice(0, m)), nthreads=threads)
        tc = time.perf_counter() - t1
        cpu = {"value": cp["steps"] / tc, "unit": "candidate-steps/s", "cores": used,
               "kind": "oracle",
               "sample": f"first {m} candidates of the same batch (precision form), "
                         f"{cp['steps']} steps in {tc:.1f}s"}
        log(f"[bench] CPU oracle: {cpu['value']:.3e} steps/s on {used} threads")
        del host_grid

    # ---- the FP64 method on the small and mid-size workloads ----------------
    if not args.no_small:
        variants["fp64_grid32"] = small_config_variant(args, crp, I, torch, stream, I.W_SMALL,
                                                       None)
        variants["fp64_grid256"] = small_config_variant(args, crp, I, torch, stream,
                                                        I.W_MIXED256, 10_000)

    # ---- galactic backtracking through the analytic field --------------------
    if not args.no_galactic:
        variants["galactic"] = galactic_variant(args, crp, I, torch, stream)

    # ---- the paper's own benchmark shape, for context ------------------------
    if not args.no_paper:
        variants["paper_comparable"] = paper_comparable(args, crp, I, torch, stream)

    # ---- batching form: a stream of 1e7-candidate batches -------------------
    if args.batching:
        variants["batching"] = batching_variant(args, crp, I, torch, grid, tables, stream)

    # ---- neural-field form: train on the grid, then replace the gather -------
    if not args.no_nf:
        variants["nf"] = neural_variant(args, crp, I, torch, w, grid, tables, stream, launch)

    traffic = None
    traffic_launch = None
    tpath = os.path.join(ROOT, "profiles", "propagate_mix_grid1024_traffic.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        # counters taken on this kernel source and grid layout (the block shape
        # changes the traffic by cache effects only)
        if (t.get("kernel_sources_sha") == kernel_sources_sha() and
                t.get("launch", {}).get("layout") == launch["layout"]):
            traffic = t.get("hbm_bytes_per_launch")
            traffic_launch = t.get("launch")

    out = {
        "metric": "candidate-steps/sec at 1024^3 grid: plain grid vs FP32/neural-field form "
                  "at stated error",
        "value": value,
        "unit": "candidate-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "candidates_per_step": n, "grid": "1024^3x3 fp32",
                   "cell_kpc": 10, "precision": "mix", "launch": launch},
        "variants": variants,
        "error_vs_fp64_oracle": err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_propagate<MIX,float,%s>" % ("corner-coop" if launch["layout"] else "linear"),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "bytes_per_gather": RECORD_BYTES,
                     "gathers_per_launch": gathers_per_launch,
                     "gather_ceiling": ceiling,
                     "attempts_per_launch": attempts_per_launch,
                     "rejects_per_launch": cnt["rejects"] / args.steps,
                     "copy_GBps_measured": copy_gbs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def copy_bandwidth(torch, dev, nbytes=1 << 32):
    """A plain device-to-device copy of nbytes timed with HIP events: bytes
    read plus bytes written per second (the best of three)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def tuned_fp64_launch(args, ctx):
    """The launch of an FP64-grid workload: the autotuner's pick on the
    context's pending work, each trial cut to TUNE_CYCLES_FP64 cycles (about a
    tenth of the 256^3 workload's run; the cache answers for a grid of the same
    shape, element type and method), the one --fp64-launch names, or the
    context's default with --no-tune.
    The pending work is unchanged."""
    if args.fp64_launch:
        b, bpc, rf, lay = [int(v) for v in args.fp64_launch.split(",")]
        ctx.set_launch(block=b, blocks_per_cu=bpc, refill=rf, layout=lay)
    elif not args.no_tune:
        ctx.tune(max_cycles=TUNE_CYCLES_FP64, cache_path=args.tune_cache)
    return ctx.get_launch()


def small_config_variant(args, crp, I, torch, stream, w, subset):
    """The FP64 method on a workload whose grid is FP64 and small: all of its
    candidates on the GPU (timed with the library's HIP events and by wall
    clock), and the oracle on the host beside it -- the whole workload, or
    its first `subset` candidates (ids 0.. , all species alike), whose records
    are also compared with the GPU's records of the same candidates."""
    grid = w.make_grid()
    tables = w.make_tables()
    n = w.n_candidates
    inj = w.make_injection(n)
    dev = torch.device("cuda:0")
    d = [torch.as_tensor(a, device=dev) for a in
         (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
    prm = crp.params_for(w, crp.FP64, device=0, queue_capacity=2 * n,
                         neutral_capacity=max(n, 1 << 16))
    ctx = crp.Context(prm, stream)
    ctx.set_field_grid(torch.as_tensor(grid, device=dev), w.spacing_m)
    ctx.set_tables(tables)

    def inject():
        ctx.reset_counters()
        ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=d[4], dir=d[5], lmax=d[6],
                   on_device=True)
        torch.cuda.synchronize()

    # untimed first run, in the launch the autotuner picks for this workload
    inject()
    launch = tuned_fp64_launch(args, ctx)
    ctx.propagate(0)
    ctx.discard_finished()
    inject()
    t0 = time.perf_counter()
    ctx.propagate(0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, _ = ctx.last_timing()
    c = ctx.counts()
    fin = crp.sort_finished(ctx.read_finished())
    ctx.discard_finished()
    ctx.close()
    out = {"workload": f"{w.name} ({n} candidates, FP64 method, {w.grid_n}^3 FP64 grid)",
           "launch": launch,
           "steps_per_s": c["steps"] / wall, "steps_per_s_kernel": c["steps"] / (ms * 1e-3),
           "wall_s": wall, "kernel_ms": ms, "steps": c["steps"], "attempts": c["attempts"],
           "finished": c["finished"], "charged_sec": c["charged_sec"],
           "neutral_sec": c["neutral_sec"]}
    # the gathers' algorithmic bytes (8 corners x 3 x FP64 = 192 B each, whether a
    # record comes from HBM or from a cache) over the kernel time
    gbs = gathers(c) * RECORD_BYTES_FP64 / (ms * 1e-3) / 1e9
    out["gather_algorithmic_GBps"] = gbs
    out["gather_frac_of_hbm_peak"] = gbs / HBM_PEAK_GBS
    log(f"[bench] {w.name}: {out['steps_per_s']:.3e} steps/s ({wall * 1e3:.1f} ms wall, "
        f"kernel {ms:.1f} ms, {gbs:.0f} GB/s algorithmic gather bandwidth, launch {launch})")
    if not args.no_cpu:
        from oracle import oracle as O
        m = n if subset is None else subset
        sub = inj.subset(slice(0, m))
        threads = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        fo, _, co, used = O.propagate(O.config_for(w), O.GridRef(grid, w.spacing_m),
                                      O.TablesRef(tables), sub, nthreads=threads)
        tc = time.perf_counter() - t0
        out["oracle"] = {"steps_per_s": co["steps"] / tc, "cores": used, "wall_s": tc,
                         "sample": "the whole workload" if subset is None else
                         f"first {m} candidates (ids 0..{m - 1})"}
        fo = O.sort_finished(fo)
        mine = fin["id"] < m
        fg = {k: v[mine] for k, v in fin.items()}
        same = 0
        if len(fg["id"]) == len(fo["id"]) and np.array_equal(fg["id"], fo["id"]) and \
                np.array_equal(fg["lineage"], fo["lineage"]):
            same = int(np.sum(np.all(fg["x"] == fo["x"], axis=1) & (fg["E"] == fo["E"]) &
                              (fg["nsteps"] == fo["nsteps"])))
        out["parity"] = {"records": int(len(fo["id"])), "gpu_records": int(len(fg["id"])),
                         "bitwise_identical": same}
        log(f"[bench] {w.name} oracle: {co['steps'] / tc:.3e} steps/s on {used} threads; "
            f"{same}/{len(fo['id'])} records bitwise identical to the GPU's")
    return out


# Bytes the observable reduction reads per record: the status of every record,
# and energy, mass number, source energy and both directions of a record that
# takes part.
OBS_BYTES_STATUS = 4
OBS_BYTES_SELECTED = 8 + 4 + 8 + 24 + 24
TRAJ_POINT_BYTES = 3 * 8 + 8 + 8 + 4 + 4 + 4 + 4


def outputs_variant(args, crp, w, n, context, inject, launch, headline):
    """The headline batch with per-step trajectory output for the first 1e5
    candidate ids, then the observable reduction over its finished records."""
    traj_ids = min(n, 100_000)
    ctx = context(crp.MIX, traj_every=1, traj_ids=traj_ids, traj_capacity=150_000_000)
    ctx.set_launch(**launch)
    inject(ctx)                          # untimed: builds this context's grid records
    ctx.propagate(0)
    ctx.discard_finished()
    ctx.discard_trajectory()
    ctx.reset_counters()
    inject(ctx)
    ctx.propagate(0)
    ms, _ = ctx.last_timing()
    cnt = ctx.counts()
    rate = cnt["steps"] / (ms * 1e-3)
    traj = {"ids_recorded": traj_ids, "every": 1, "points": cnt["traj_points"],
            "dropped": cnt["traj_dropped"], "kernel_ms": ms, "steps_per_s_kernel": rate,
            "point_bytes": TRAJ_POINT_BYTES}
    log(f"[bench] with per-step output of {traj_ids} candidates: {cnt['traj_points']} points, "
        f"kernel {ms:.1f} ms ({rate:.4e} steps/s by kernel time)")
    edges = 10.0 ** np.linspace(16.0, 22.0, 25)
    spec = dict(e_edges=edges, a_edges=np.array([1, 2, 5, 15, 57]), status_mask=0b11110,
                sky_n=64, sky_sign=-1.0, e_ref=1e18, gamma=-1.5)
    ctx.set_observables(spec)
    ctx.observe()                        # warm
    ctx.set_observables(spec)
    oms = ctx.observe()
    ob = ctx.read_observables()
    nrec = cnt["finished_unread"]
    nsel = int(ob["counts"].sum()) + ob["outside"]
    obytes = OBS_BYTES_STATUS * nrec + OBS_BYTES_SELECTED * nsel
    gbs = obytes / (oms * 1e-3) / 1e9
    log(f"[bench] observables over {nrec} records: {oms:.3f} ms, {gbs:.0f} GB/s algorithmic")
    ctx.close()
    oracle = None
    if not args.no_cpu:
        # the oracle's reduction on a bounded synthetic sample of records
        from oracle import observables as OB
        m = 1_000_000
        rng = np.random.default_rng(72)
        recs = dict(status=rng.integers(1, 5, m).astype(np.int32),
                    A=rng.choice([1, 4, 14, 56], m).astype(np.int32),
                    E=10.0 ** rng.uniform(16.0, 22.0, m), E0=10.0 ** rng.uniform(18.0, 21.0, m),
                    u=rng.standard_normal((m, 3)), u0=rng.standard_normal((m, 3)))
        sp = dict(spec, e_edges=np.asarray(edges), a_edges=np.asarray(spec["a_edges"]))
        t0 = time.perf_counter()
        OB.observe(sp, recs)
        t1 = time.perf_counter() - t0
        oracle = {"records_per_s": m / t1, "cores": 1, "sample": f"{m} synthetic records"}
        log(f"[bench] observables oracle: {m / t1:.3e} records/s (one core)")
    obs = {"records": nrec, "selected": nsel, "kernel_ms": oms, "oracle": oracle,
           "bins": int(ob["counts"].size), "sky_pixels": int(ob["sky"].shape[-1]),
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": obytes}}
    return {"trajectory": traj, "observe": obs}


def nested_variant(args, crp, I, torch, w, n, grid, tables, stream, inj):
    """The 1e7 mixed-nuclei batch started at the centre of a 512^3 refinement
    patch (4x finer: 2.5 kpc cells over a 1.28 Mpc cube) inside the 1024^3
    grid, against the same batch on the plain grid, both from corner records
    gathered by the whole wave."""
    nside, refine, off = 512, 4, 448
    dev = grid.device
    t0 = time.time()
    patch = I.turbulent_grid(nside, w.spacing_m / refine, 2.0, 64.0, w.brms_T, 31, np.float32,
                             device=dev)
    torch.cuda.synchronize()
    centre = (off + nside / refine / 2) * w.spacing_m
    pos = torch.full((n, 3), centre, dtype=torch.float64, device=dev)
    d = [torch.as_tensor(a, device=dev) for a in
         (inj.id.view(np.int32), inj.A, inj.Z, inj.E)] + \
        [pos] + [torch.as_tensor(a, device=dev) for a in (inj.dir, inj.lmax)]
    log(f"[bench] nested: patch {nside}^3 x{refine} generated in {time.time() - t0:.1f}s")
    out = {"patch": f"{nside}^3 fp32, refine {refine} ({w.spacing_m / refine / I.KPC_M:g} kpc "
                    f"cells), offset {off}", "workload": f"{w.name} started at the patch centre"}
    for name, patches in (("nested", [dict(data=patch, offset=(off, off, off), refine=refine)]),
                          ("plain", [])):
        prm = crp.params_for(w, crp.MIX, device=0, queue_capacity=2 * n,
                             neutral_capacity=max(n, 1 << 20))
        ctx = crp.Context(prm, stream)
        ctx.set_field_grid(grid, w.spacing_m)
        ctx.set_tables(tables)
        if patches:
            ctx.set_field_patches(patches)
        ctx.set_launch(block=128, blocks_per_cu=0, refill=4, layout=crp.LAYOUT_CORNER)
        ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=d[4], dir=d[5], lmax=d[6],
                   on_device=True)
        ctx.propagate(0)
        ms, _ = ctx.last_timing()
        cnt = ctx.counts()
        ctx.close()
        rate = cnt["steps"] / (ms * 1e-3)
        gbs = gathers(cnt) * RECORD_BYTES / (ms * 1e-3) / 1e9
        out[name] = {"steps_per_s": rate, "kernel_ms": ms, "steps": cnt["steps"],
                     "attempts": cnt["attempts"], "rejects": cnt["rejects"],
                     "algorithmic_GBps": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS}
        log(f"[bench] {name}: {rate:.4e} steps/s, kernel {ms:.1f} ms, {gbs:.0f} GB/s algorithmic")
    if not args.no_cpu:
        # the oracle on the first candidates of the same batch, both levels on the host
        from oracle import oracle as O
        m = 64
        G = O.GridRef(grid.cpu().numpy(), w.spacing_m,
                      patches=[dict(data=patch.cpu().numpy(), offset=(off, off, off),
                                    refine=refine)])
        sub = I.Injection(inj.id[:m], inj.A[:m], inj.Z[:m], inj.E[:m],
                          np.full((m, 3), centre), inj.dir[:m], inj.lmax[:m])
        t1 = time.perf_counter()
        _, _, co, used = O.propagate(O.config_for(w, precision=O.MIX), G, O.TablesRef(tables),
                                     sub, nthreads=len(os.sched_getaffinity(0)))
        tc = time.perf_counter() - t1
        out["oracle"] = {"steps_per_s": co["steps"] / tc, "cores": used,
                         "sample": f"first {m} candidates of the batch, precision form"}
        log(f"[bench] nested oracle: {co['steps'] / tc:.3e} steps/s on {used} threads")
        del G
    del patch, pos, d
    torch.cuda.empty_cache()
    return out


# FP64 operations of one Cash-Karp attempt of the FP64 method with the analytic
# field: 6 field evaluations x 47 (3 differences, 3 for r^2, 1 for z^2, 6 for the
# disk denominator X, 2 + 5 for the halo denominator Y, 7 for g including its
# division, 4 for D, 1 + 1 for 1/D and its square, 3 for q, 3 + 3 + 5 for B)
# plus the stages: 6 x 12 derivative, 210 stage sums, 54 fifth-order sum, 34
# error estimate.
ANALYTIC_FLOP_PER_ATTEMPT = 6 * 47 + 6 * 12 + 210 + 54 + 34
FP64_VECTOR_PEAK_TFLOPS = 78.6


def galactic_variant(args, crp, I, torch, stream):
    """Galactic backtracking (section 4): observed events at Earth traced back
    as antiparticles through the analytic disk/halo/X-field model to a 20 kpc
    sphere; ALU-bound (no field memory)."""
    w = I.W_GALBACK
    n = args.gal_n
    inj = w.make_injection(n)
    dev = torch.device("cuda:0")
    d = [torch.as_tensor(a, device=dev) for a in
         (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
    out = {"workload": f"{w.name} x {n} events (H/He/N/Fe, 1-100 EeV, 20 kpc sphere)"}
    for name, prec in (("fp64", crp.FP64), ("mix", crp.MIX)):
        prm = crp.params_for(w, prec, device=0, queue_capacity=2 * n, neutral_capacity=1 << 16)
        ctx = crp.Context(prm, stream)
        ctx.set_field_analytic(I.GALACTIC_FIELD)
        ctx.set_tables(w.make_tables())
        rate = None
        for rep in range(2):                     # the first run is untimed
            ctx.reset_counters()
            ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=d[4], dir=d[5], lmax=d[6],
                       on_device=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.propagate(0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms, _ = ctx.last_timing()
            c = ctx.counts()
            if prec == crp.FP64 and rep == 1:
                out["lens"] = lens_measure(crp, torch, ctx)
            ctx.discard_finished()
        ctx.close()
        r = {"steps_per_s": c["steps"] / wall, "events_per_s": n / wall, "kernel_ms": ms,
             "steps": c["steps"], "attempts": c["attempts"], "boundary": c["boundary"],
             "max_traj": c["max_traj"]}
        if prec == crp.FP64:
            achieved = c["attempts"] * ANALYTIC_FLOP_PER_ATTEMPT / (ms * 1e-3) / 1e12
            r["roofline"] = {"bound": "alu", "flop_per_attempt": ANALYTIC_FLOP_PER_ATTEMPT,
                             "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS}
        out[name] = r
        log(f"[bench] galactic backtracking ({name}): {c['steps'] / wall:.3e} steps/s, "
            f"{n / wall:.3e} events/s, kernel {ms:.1f} ms")
    if not args.no_cpu:
        from oracle import oracle as O
        m = 20000
        t0 = time.perf_counter()
        fo, _, co, used = O.propagate(O.config_for(w), O.AnalyticRef(I.GALACTIC_FIELD),
                                      O.TablesRef(w.make_tables()), inj.subset(slice(0, m)),
                                      nthreads=len(os.sched_getaffinity(0)))
        t1 = time.perf_counter() - t0
        out["oracle"] = {"steps_per_s": co["steps"] / t1, "cores": used,
                         "sample": f"first {m} events, FP64"}
        log(f"[bench] galactic backtracking oracle: {co['steps'] / t1:.3e} steps/s on {used} "
            f"threads")
        if "lens" in out:
            # the oracle's lens construction and application on its own records
            from oracle import lens as LN
            sp = LN.spec(10.0 ** np.linspace(16.5, 20.0, 8), sky_n=32)
            t0 = time.perf_counter()
            L = LN.build(sp, fo)
            tb = time.perf_counter() - t0
            x = np.random.default_rng(71).uniform(0.0, 1.0, (16, 7, 6144))
            t0 = time.perf_counter()
            LN.apply(L, x)
            ta = time.perf_counter() - t0
            out["lens"]["oracle"] = {"build_records_per_s": len(fo["id"]) / tb,
                                     "apply_entries_per_s": 16 * len(L["col"]) / ta,
                                     "cores": 1, "sample": f"the oracle's {m} events"}
            log(f"[bench] lens oracle: build {len(fo['id']) / tb:.3e} records/s, apply "
                f"{16 * len(L['col']) / ta:.3e} entries/s (one core)")
    return out


def lens_measure(crp, torch, ctx, sky_n=32, n_maps=16):
    """Galactic lenses (section 4) from the backtracked events still unread in
    ctx: build time, then the application to n_maps random border maps, priced
    at its algorithmic bytes: the matrix once (12 bytes per entry for column
    and value, 8 per row pointer) and each border map read and each Earth map
    written once (8 + 8 bytes per row and map)."""
    edges = 10.0 ** np.linspace(16.5, 20.0, 8)
    spec = dict(r_edges=edges, sky_n=sky_n, status_mask=1 << crp.BOUNDARY)
    _, first_ms = ctx.lens_build(spec)                  # allocates the construction scratch
    nnz, bms = ctx.lens_build(spec)
    nr, npix = len(edges) - 1, 6 * sky_n * sky_n
    nrows = nr * npix
    g = torch.Generator(device="cuda:0")
    g.manual_seed(71)
    x = torch.rand((n_maps, nr, npix), dtype=torch.float64, device="cuda:0", generator=g)
    y = torch.empty_like(x)
    ctx.lens_apply(x, y)                                # warm
    _, ams = ctx.lens_apply(x, y)
    # algorithmic bytes: the matrix once (column and value per entry, the row
    # pointers) and every border map read and Earth map written once
    app_bytes = 12 * nnz + 8 * (nrows + 1) + n_maps * 16 * nrows
    per_map = app_bytes / n_maps
    gbs = app_bytes / (ams * 1e-3) / 1e9
    log(f"[bench] lenses: {nr} rigidity bins x {npix} pixels, {nnz} entries, built in "
        f"{bms:.2f} ms; {n_maps} maps applied in {ams:.3f} ms = {gbs:.0f} GB/s algorithmic")
    return {"rigidity_bins": nr, "pixels": npix, "nnz": nnz, "build_ms": bms,
            "first_build_ms": first_ms,
            "maps": n_maps, "apply_ms": ams, "bytes_per_map": per_map,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS}}


def paper_comparable(args, crp, I, torch, stream):
    """The shape of the paper's 3D benchmark (section 6: protons, log-flat
    1-1000 EeV, 1 Gpc, losses off; here the 256^3 FP64 grid and the FP64
    method): GPU trajectories per second, and the oracle's single-core time
    per trajectory beside the paper's 1.0 ms (Intel i5-3317U, 1.7 GHz)."""
    w = I.W_PAPER256
    n = args.paper_n
    grid = w.make_grid()
    tables = w.make_tables()
    inj = w.make_injection(n)
    dev = torch.device("cuda:0")
    d = [torch.as_tensor(a, device=dev) for a in
         (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir, inj.lmax)]
    prm = crp.params_for(w, crp.FP64, device=0, queue_capacity=2 * n, neutral_capacity=1 << 16)
    ctx = crp.Context(prm, stream)
    ctx.set_field_grid(grid, w.spacing_m)
    ctx.set_tables(tables)

    def run(tune):
        ctx.reset_counters()
        ctx.inject(id=d[0], A=d[1], Z=d[2], E=d[3], pos=d[4], dir=d[5], lmax=d[6],
                   on_device=True)
        torch.cuda.synchronize()
        if tune:
            tuned_fp64_launch(args, ctx)
        t0 = time.perf_counter()
        ctx.propagate(0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        c = ctx.counts()
        ctx.discard_finished()
        return wall, c

    run(True)                                    # untimed first run (tuned launch)
    wall, c = run(False)
    launch = ctx.get_launch()
    ctx.close()
    out = {"workload": f"{w.name} ({n} protons, FP64 method)", "launch": launch,
           "gpu_trajectories_per_s": n / wall,
           "gpu_us_per_trajectory": 1e6 * wall / n, "gpu_steps_per_s": c["steps"] / wall,
           "steps_per_trajectory": c["steps"] / n,
           "paper_ms_per_trajectory": 1.0,
           "paper_hardware": "Intel Core i5-3317U @ 1.7 GHz, Python steering (section 6)"}
    log(f"[bench] paper-shaped 3D workload: GPU {n / wall:.3e} trajectories/s "
        f"({1e6 * wall / n:.3f} us each, {c['steps'] / n:.0f} steps per trajectory)")
    if not args.no_cpu:
        from oracle import oracle as O
        G = O.GridRef(grid, w.spacing_m)
        T = O.TablesRef(tables)
        m = 200
        t0 = time.perf_counter()
        _, _, co, used = O.propagate(O.config_for(w), G, T, inj.subset(slice(0, m)), nthreads=1)
        t1 = time.perf_counter() - t0
        out["oracle_ms_per_trajectory_one_core"] = 1e3 * t1 / m
        out["oracle_sample"] = f"first {m} trajectories, {co['steps']} steps, 1 thread"
        log(f"[bench] oracle on one host core: {1e3 * t1 / m:.2f} ms per trajectory "
            f"(paper: 1.0 ms on an i5-3317U)")
    return out


def batching_variant(args, crp, I, torch, grid, tables, stream):
    """Batches of 1e7 candidates (distances U[1, 1000] Mpc around an observer at the
    origin, seeds 404 + b, ids b*1e7 ...), each run to completion by the persistent
    kernel in the launch the autotuner picks for this workload.  Inputs are
    generated and uploaded before the timed region; finished and secondary
    records are drained on the device (counted, not copied to the host)."""
    w = I.W_DIST1024
    nb = args.batching
    per = w.n_candidates
    dev = grid.device
    log(f"[bench] batching form: {nb} batches of {per}")
    batches = []
    for b in range(nb):
        inj = I.inject_distances(per, 404 + b, id0=b * per)
        batches.append([torch.as_tensor(a, device=dev) for a in
                        (inj.id.view(np.int32), inj.A, inj.Z, inj.E, inj.pos, inj.dir,
                         inj.lmax)])
    prm = crp.params_for(w, crp.MIX, device=0, queue_capacity=2 * per,
                         neutral_capacity=max(per, 1 << 20))
    ctx = crp.Context(prm, stream)
    ctx.set_field_grid(grid, w.spacing_m)
    ctx.set_tables(tables)

    def inject(d, k=None):
        s = slice(0, k)
        ctx.inject(id=d[0][s], A=d[1][s], Z=d[2][s], E=d[3][s], pos=d[4][s], dir=d[5][s],
                   lmax=d[6][s], on_device=True)

    # the launch shape tuned on this workload's calibration batch (from the
    # tuner cache when an earlier run with the same cache file tuned it; else
    # tuned here), then that batch once more, untimed, as a warm-up
    log("[bench] batching: inputs on the device; tuning on 1e6 candidates")
    inject(batches[0], 1_000_000)
    tuned, rate = ctx.tune(max_cycles=0, cache_path=args.tune_cache)
    ctx.discard_finished()
    while not ctx.propagate(0):
        pass
    ctx.discard_finished()
    log(f"[bench] batching: launch {tuned}")
    ctx.reset_counters()
    torch.cuda.synchronize()
    per_batch = []
    t0 = time.perf_counter()
    for b in range(nb):
        inject(batches[b])
        ctx.propagate(0)
        ms, _ = ctx.last_timing()
        ctx.discard_finished()
        per_batch.append(ms)
        log(f"[bench] batching: batch {b}: kernel {ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = ctx.counts()
    ctx.close()
    out = {"workload": f"{w.name} x {nb} batches", "candidates": nb * per,
           "steps_per_s": cnt["steps"] / wall, "wall_s": wall, "steps": cnt["steps"],
           "attempts": cnt["attempts"], "kernel_ms_per_batch": per_batch,
           "kernel_share_of_wall": sum(per_batch) * 1e-3 / wall, "launch": tuned,
           "finished": cnt["finished"], "observed": cnt["observed"],
           "charged_sec": cnt["charged_sec"], "neutral_sec": cnt["neutral_sec"],
           "queue_deferred": cnt["queue_deferred"],
           "neutral_deferred": cnt["neutral_deferred"]}
    log(f"[bench] batching form: {out['steps_per_s']:.4e} steps/s over {nb * per} candidates "
        f"({wall:.1f} s)")
    return out


def neural_variant(args, crp, I, torch, w, grid, tables, stream, launch):
    """The learned form at two points of its capacity curve.  'c3_band': the
    network trained (1e8 points, lr 1e-3 -> 1e-5) on the 1024^3 grid of the
    timed batch (band 2..16 cycles per box), far from its 1% target.
    'narrow_band': the same network on a 1024^3 field of the band 2..3 cycles
    per box (seed 3, 1 nG RMS), trained until its RMS error falls below 1%
    (3e9 points, lr 3e-3 -> 1e-5).  At each point: the RMS field error on 1e6
    held-out points, and the surrogate against the grid on 1e6 candidates of
    the distance workload (sources at 1-1000 Mpc, secondaries on)."""
    out = {"c3_band": nf_point(args, crp, I, torch, grid, tables, stream, launch,
                               band=(2.0, 16.0), steps=args.nf_steps, lr0=1e-3)}
    if args.nf_narrow_steps > 0:
        g3 = I.turbulent_grid(w.grid_n, w.spacing_m, 2.0, 3.0, w.brms_T, 3, np.float32,
                              grid.device)
        out["narrow_band"] = nf_point(args, crp, I, torch, g3, tables, stream, launch,
                                      band=(2.0, 3.0), steps=args.nf_narrow_steps, lr0=3e-3)
        del g3
        torch.cuda.empty_cache()
    return out


def nf_point(args, crp, I, torch, grid, tables, stream, launch, band, steps, lr0):
    """Trains the Fourier-feature network on `grid` (its 64 frequencies drawn
    from `band`) with the library's own kernels and compares the surrogate with
    the grid path on a batch of the distance workload."""
    wd = I.W_DIST1024
    nprm = crp.params_for(wd, crp.MIX, device=0, field_mode=crp.FIELD_NEURAL,
                          queue_capacity=2 * args.nf_candidates,
                          neutral_capacity=max(args.nf_candidates, 1 << 20))
    cnf = crp.Context(nprm, stream)
    cnf.set_field_grid(grid, wd.spacing_m)
    cnf.set_tables(tables)
    cnf.nf_init(I.nf_frequencies(nmin=band[0], nmax=band[1], seed=505), I.nf_init_flat(509),
                wd.brms_T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = cnf.nf_train(steps, 65536, lr0, 1e-5, 506)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"[bench] NF (band {band[0]:g}..{band[1]:g}) trained on {steps * 65536:.3g} points "
        f"in {train_s:.1f}s, loss {losses[0]:.4f} -> {losses[-1]:.5f}")
    # field error on held-out points (the grid path is the reference)
    box = wd.grid_n * wd.spacing_m
    pos = I.uniform_points(1_000_000, box, 507)
    Bn = cnf.eval_field(pos, crp.EVAL_NEURAL)
    Bg = cnf.eval_field(pos, crp.MIX)
    rms = float(np.sqrt(((Bn - Bg) ** 2).sum(1).mean()) / wd.brms_T)
    log(f"[bench] NF RMS field error {rms:.4f} of B_rms")
    inj = I.inject_distances(args.nf_candidates, 508)

    def run(ctx):
        ctx.reset_counters()
        ctx.inject(inj)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.propagate(0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ms, _ = ctx.last_timing()
        fin = ctx.read_finished()
        ctx.discard_finished()
        c = ctx.counts()
        return fin, c["steps"] / dt, ms, c

    fin_nf, rate_nf, ms_nf, c_nf = run(cnf)
    cnf.close()
    gprm = crp.params_for(wd, crp.MIX, device=0, queue_capacity=2 * args.nf_candidates,
                          neutral_capacity=max(args.nf_candidates, 1 << 20))
    cg = crp.Context(gprm, stream)
    cg.set_field_grid(grid, wd.spacing_m)
    cg.set_tables(tables)
    cg.set_launch(**launch)
    run(cg)                                     # untimed: builds the grid records
    fin_g, rate_g, ms_g, c_g = run(cg)
    cg.close()

    def hist(f):
        th = np.degrees(np.arccos(np.clip((f["u"] * f["u0"]).sum(1), -1, 1)))
        return np.histogram(th, bins=36, range=(0, 180))[0] / max(len(th), 1), th

    hn, thn = hist(fin_nf)
    hg, thg = hist(fin_g)
    from scipy import stats
    ks = float(stats.ks_2samp(thn, thg).statistic)
    out = {"band_cycles_per_box": list(band), "steps_per_s": rate_nf, "kernel_ms": ms_nf,
           "grid_steps_per_s_same_batch": rate_g,
           "speedup_vs_grid": rate_nf / rate_g, "rms_field_error": rms,
           "deflection_hist_distance": float(0.5 * np.abs(hn - hg).sum()), "deflection_ks": ks,
           "train_points": steps * 65536, "train_lr0": lr0, "train_s": train_s,
           "final_train_loss": float(losses[-1]), "field_bytes_network": 66435 * 2,
           "field_bytes_grid": int(grid.numel() * 4),
           "workload": f"{wd.name} subset of {args.nf_candidates} candidates (seed 508)",
           "steps": {"nf": c_nf["steps"], "grid": c_g["steps"]},
           "attempts": {"nf": c_nf["attempts"], "grid": c_g["attempts"]},
           "kernel_time_ratio_nf_over_grid": ms_nf / ms_g}
    # MFMA work of the network: four 128x128 layers per evaluation, six
    # evaluations per Cash-Karp attempt (the 128->3 output layer is not counted)
    flop = 6 * 4 * 2 * 128 * 128
    achieved = c_nf["attempts"] * flop / (ms_nf * 1e-3) / 1e12
    out["mfma"] = {"bound": "mfma", "flop_per_attempt": flop, "achieved": achieved,
                   "peak": 2500.0, "unit": "TFLOP/s", "frac": achieved / 2500.0}
    log(f"[bench] NF form: {rate_nf:.3e} steps/s vs grid {rate_g:.3e} on the same batch; "
        f"deflection histogram distance {out['deflection_hist_distance']:.4f}, KS {ks:.4f}")
    return out


def nf_sweep(spec, crp, I, torch, dev, stream):
    """Field error of the network against the band of the turbulent field and
    the training length: for each n_max a 1024^3 FP32 grid of the band
    2..n_max cycles per box (seed 3, 1 nG RMS, 10 kpc cells), the network's 64
    frequencies drawn from that band (seed 505), then for each length a fresh
    network (seed 509) trained with one cosine schedule (lr LR -> 1e-5, batch
    65536, Philox seed 506) and its RMS error on 1e6 held-out points (seed 507)."""
    nmaxes, steps_list, lr0 = spec.split(":")
    w = I.W_DIST1024
    box = w.grid_n * w.spacing_m
    pos = I.uniform_points(1_000_000, box, 507)
    for nmax in [float(v) for v in nmaxes.split(",")]:
        grid = I.turbulent_grid(w.grid_n, w.spacing_m, 2.0, nmax, w.brms_T, 3, np.float32, dev)
        prm = crp.params_for(w, crp.MIX, device=0, field_mode=crp.FIELD_NEURAL,
                             queue_capacity=1 << 16, neutral_capacity=1 << 16)
        ctx = crp.Context(prm, stream)
        ctx.set_field_grid(grid, w.spacing_m)
        ctx.set_tables(w.make_tables())
        F = I.nf_frequencies(nmin=2.0, nmax=nmax, seed=505)
        Bg = ctx.eval_field(pos, crp.MIX)
        for steps in [int(v) for v in steps_list.split(",")]:
            ctx.nf_init(F, I.nf_init_flat(509), w.brms_T)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = ctx.nf_train(steps, 65536, float(lr0), 1e-5, 506)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            Bn = ctx.eval_field(pos, crp.EVAL_NEURAL)
            rms = float(np.sqrt(((Bn - Bg) ** 2).sum(1).mean()) / w.brms_T)
            print(json.dumps({"nmax": nmax, "band_modes": int(len(I.turbulence_modes(
                0, 2.0, nmax, exclude_nyquist=False))), "steps": steps,
                "points": steps * 65536, "lr0": float(lr0), "rms": rms, "train_s": dt,
                "final_loss": float(np.mean(losses[-20:]))}), flush=True)
        ctx.close()
        del grid
        torch.cuda.empty_cache()


def summarize_pmc(d, kernel=None):
    """Per-launch HBM read/write bytes of the propagation kernel from two
    rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each
    scaled by what the same counter reads for the 1 GiB copy (--calib-copy).
    kernel: the kernel-name prefix of the instantiation to summarize (default:
    the precision form on the FP32 grid's corner records, the headline's)."""
    kernel = kernel or "k_propagate<1, float, 2,"
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            c, k = r["Counter_Name"], r["Kernel_Name"]
            if c not in ("FETCH_SIZE", "WRITE_SIZE"):
                continue
            # the timed propagation kernel: the precision form on the FP32 grid
            # (other instantiations run in the same process for the variant
            # lines: FP64 grids, the analytic field, the neural field)
            grid_prop = kernel in k
            kind = "prop" if grid_prop else ("copy" if "copyBuffer" in k else None)
            if kind:
                vals.setdefault((kind, c), []).append((int(r["Dispatch_Id"]),
                                                       float(r["Counter_Value"])))
    gib = float(1 << 30)
    out = {"kernel_sources_sha": kernel_sources_sha(), "kernel": kernel}
    for c, key in (("FETCH_SIZE", "read"), ("WRITE_SIZE", "write")):
        # the 1 GiB copy of --calib-copy is the run's first copy dispatch (later
        # copies, e.g. the 4 GiB copy-bandwidth probe, have other sizes)
        copy = min(vals[("copy", c)])[1] * 1024.0       # bytes as counted
        vals[("prop", c)] = [v for _, v in vals[("prop", c)]]
        prop = max(vals[("prop", c)]) * 1024.0          # the largest (timed) propagation launch
        factor = gib / copy
        out[f"{key}_scale_factor"] = factor
        out[f"{key}_bytes_per_launch"] = prop * factor
    out["hbm_bytes_per_launch"] = out["read_bytes_per_launch"] + out["write_bytes_per_launch"]
    print(json.dumps(out, indent=1))


def error_report(gpu, ref):
    """Per-output error of the precision form against the FP64 oracle, over
    the records present in both (keyed by (id, lineage))."""
    kg = gpu["id"].astype(np.uint64) << np.uint64(32) | gpu["lineage"].astype(np.uint64)
    kr = ref["id"].astype(np.uint64) << np.uint64(32) | ref["lineage"].astype(np.uint64)
    common, ig, ir = np.intersect1d(kg, kr, return_indices=True)
    only = int(len(kg) + len(kr) - 2 * len(common))
    gpu = {k: v[ig] for k, v in gpu.items()}
    ref = {k: v[ir] for k, v in ref.items()}
    scale = np.maximum(ref["L"], 1.0)
    dx = np.linalg.norm(gpu["x"] - ref["x"], axis=1) / scale
    cosang = np.clip((gpu["u"] * ref["u"]).sum(1), -1.0, 1.0)
    dang = np.degrees(np.arccos(cosang))
    dE = np.abs(gpu["E"] / ref["E"] - 1.0)
    dL = np.abs(gpu["L"] / ref["L"] - 1.0)

    def q(v):
        return {"median": float(np.median(v)), "p99": float(np.quantile(v, 0.99)),
                "max": float(np.max(v))}

    ints = {k: int(np.sum(gpu[k] != ref[k])) for k in ("status", "A", "Z", "m", "nsteps")}
    th_g = np.degrees(np.arccos(np.clip((gpu["u"] * gpu["u0"]).sum(1), -1, 1)))
    th_r = np.degrees(np.arccos(np.clip((ref["u"] * ref["u0"]).sum(1), -1, 1)))
    hg = np.histogram(th_g, bins=36, range=(0, 180))[0] / len(th_g)
    hr = np.histogram(th_r, bins=36, range=(0, 180))[0] / len(th_r)
    # the same, stratified by the record's rigidity E/Z (volts, the oracle's
    # final energy and charge): low rigidity means small gyroradii and chaotic
    # paths, where FP32 stage differences grow fastest
    lgR = np.log10(ref["E"] / ref["Z"])
    strata = {}
    for lo, hi in ((-np.inf, 18.0), (18.0, 19.0), (19.0, 20.0), (20.0, np.inf)):
        sel = (lgR >= lo) & (lgR < hi)
        if not sel.any():
            continue
        name = f"lgR[{lo:g},{hi:g})"
        strata[name] = {"records": int(sel.sum()), "position_rel": q(dx[sel]),
                        "direction_deg": q(dang[sel]), "energy_rel": q(dE[sel]),
                        "length_rel": q(dL[sel]),
                        "integer_mismatches": {k: int(np.sum(gpu[k][sel] != ref[k][sel]))
                                               for k in ("status", "A", "Z", "m", "nsteps")}}
    return {"records_compared": int(len(ref["id"])), "records_in_one_only": only,
            "position_rel": q(dx), "direction_deg": q(dang),
            "energy_rel": q(dE), "length_rel": q(dL), "integer_mismatches": ints,
            "deflection_hist_distance": float(0.5 * np.abs(hg - hr).sum()),
            "by_rigidity": strata}


if __name__ == "__main__":
    main()
