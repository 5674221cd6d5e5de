"""Host logic of the build script: the parallel command pool."""
import subprocess
import sys

import pytest


def test_parallel_pool_runs_all_and_reports_a_failure(tmp_path, monkeypatch):
    from paper_1307_2643_amd import build as B
    monkeypatch.setenv("CRP_BUILD_JOBS", "3")
    marks = [tmp_path / f"m{i}" for i in range(7)]
    cmds = [[sys.executable, "-c", f"open({str(m)!r}, 'w').close()"] for m in marks]
    B._run_parallel(cmds, verbose=False)
    assert all(m.exists() for m in marks)
    bad = [[sys.executable, "-c", "pass"], [sys.executable, "-c", "raise SystemExit(3)"]]
    with pytest.raises(subprocess.CalledProcessError) as ei:
        B._run_parallel(bad, verbose=False)
    assert ei.value.returncode == 3
