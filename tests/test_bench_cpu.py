"""Host-side logic of bench.py that needs no GPU: the refusal of more than one
GPU, and the traffic summary that scales the FETCH_SIZE / WRITE_SIZE counters
of the propagation launch by what the same counters read for a 1 GiB copy."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, cwd=ROOT, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, k, c, v in rows:
            f.write(f'{d},"{k}",{c},{v}\n')


def test_traffic_summary_scales_by_the_copy(tmp_path):
    prop = "void crp::k_propagate<1, float, 2, 128, false>(crp::PropParams const*)"
    other = "void crp::k_propagate<0, double, 4, 128, false>(crp::PropParams const*)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = float(1 << 20)
    (tmp_path / "fetch").mkdir()
    (tmp_path / "write").mkdir()
    # the copy reads half its bytes as counted (FETCH_SIZE), writes all of them;
    # two propagation launches (the larger is the timed one) and a kernel of
    # another instantiation that must be ignored
    # later copies (the 4 GiB copy-bandwidth probe, record read-backs) are
    # other sizes: the calibration is the run's first copy dispatch
    _csv(tmp_path / "fetch" / "fetch_counter_collection.csv",
         [(1, copy, "FETCH_SIZE", gib_kib / 2), (2, prop, "FETCH_SIZE", 1000.0),
          (3, prop, "FETCH_SIZE", 3000.0), (4, other, "FETCH_SIZE", 9e9),
          (5, copy, "FETCH_SIZE", 4 * gib_kib / 2), (6, copy, "FETCH_SIZE", 7.0)])
    _csv(tmp_path / "write" / "write_counter_collection.csv",
         [(1, copy, "WRITE_SIZE", gib_kib), (2, prop, "WRITE_SIZE", 10.0),
          (3, prop, "WRITE_SIZE", 20.0), (4, other, "WRITE_SIZE", 9e9),
          (5, copy, "WRITE_SIZE", 4 * gib_kib), (6, copy, "WRITE_SIZE", 7.0)])
    r = _run("--summarize-pmc", str(tmp_path))
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["read_scale_factor"] == 2.0 and out["write_scale_factor"] == 1.0
    assert out["read_bytes_per_launch"] == 3000.0 * 1024 * 2
    assert out["write_bytes_per_launch"] == 20.0 * 1024
    assert out["hbm_bytes_per_launch"] == 3000.0 * 1024 * 2 + 20.0 * 1024
    assert len(out["kernel_sources_sha"]) == 16


def test_error_report_keys_records_and_measures_differences():
    """The precision-form error summary pairs records by (id, lineage), counts
    records present on one side only, and measures known perturbations."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    n = 1000
    rng = np.random.default_rng(5)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    ref = dict(id=np.arange(n, dtype=np.uint32), lineage=np.zeros(n, np.uint32),
               x=rng.standard_normal((n, 3)) * 1e22, u=u, u0=u.copy(), E=np.full(n, 1e19),
               L=np.full(n, 1e23), status=np.full(n, 2, np.int32), A=np.ones(n, np.int32),
               Z=np.ones(n, np.int32), m=np.zeros(n, np.uint32), nsteps=np.full(n, 7, np.uint32))
    gpu = {k: v.copy() for k, v in ref.items()}
    gpu["E"] = gpu["E"] * (1.0 + 1e-9)                  # every energy off by 1e-9
    gpu["x"][:, 0] += 1e23 * 1e-6                       # every position off by 1e-6 of L
    gpu["status"][:3] = 3                               # three integer mismatches
    order = rng.permutation(n)[:-5]                     # shuffled, five records missing
    gpu = {k: v[order] for k, v in gpu.items()}
    r = bench.error_report(gpu, ref)
    assert r["records_compared"] == n - 5 and r["records_in_one_only"] == 5
    assert abs(r["energy_rel"]["median"] - 1e-9) < 1e-15
    assert abs(r["position_rel"]["max"] - 1e-6) < 1e-12
    assert r["direction_deg"]["max"] < 1e-5          # arccos of a dot product rounded near 1
    assert r["integer_mismatches"]["status"] == sum(1 for i in order if i < 3)
    assert r["deflection_hist_distance"] == 0.0


def test_error_report_strata_by_rigidity():
    """The strata split the records by log10(E/Z) of the reference record,
    partition them, and carry each stratum's own errors."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    n = 400
    rng = np.random.default_rng(6)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    Z = rng.choice([1, 2, 7, 26], n).astype(np.int32)
    E = 10.0 ** rng.uniform(17.5, 21.5, n)
    ref = dict(id=np.arange(n, dtype=np.uint32), lineage=np.zeros(n, np.uint32),
               x=rng.standard_normal((n, 3)) * 1e22, u=u, u0=u.copy(), E=E,
               L=np.full(n, 1e23), status=np.full(n, 2, np.int32), A=2 * Z, Z=Z,
               m=np.zeros(n, np.uint32), nsteps=np.full(n, 7, np.uint32))
    gpu = {k: v.copy() for k, v in ref.items()}
    low = np.log10(E / Z) < 18.0
    gpu["E"] = np.where(low, E * (1 + 1e-6), E)        # only the lowest stratum is off
    r = bench.error_report(gpu, ref)
    st = r["by_rigidity"]
    assert sum(v["records"] for v in st.values()) == n
    assert st["lgR[-inf,18)"]["records"] == int(low.sum()) > 0
    assert abs(st["lgR[-inf,18)"]["energy_rel"]["median"] - 1e-6) < 1e-12
    for k, v in st.items():
        if k != "lgR[-inf,18)":
            assert v["energy_rel"]["max"] == 0.0
