"""bench.py host logic on the CPU: argument contract and roofline arithmetic."""
import subprocess
import sys

import numpy as np

import bench
from paper_2409_05572_amd.api import SolveInfo


def _info(ms, by, fl, calls):
    return SolveInfo(0, 10, True, 1, 1, 1e-9, 1e-9, 100.0, 0, np.zeros((0, 8)),
                     tuple(ms), tuple(by), tuple(fl), tuple(calls))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "4"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stdout


def test_roofline_picks_dominant_class_and_divides_correctly():
    ms = [1.0, 2.0, 10.0, 0.5, 3.0, 1.0, 0.1, 0.0]
    by = [8e9, 1e9, 2e9, 1e9, 0, 0, 0, 0]
    fl = [1e9, 1e11, 5e11, 0, 0, 0, 0, 0]
    calls = [2, 4, 10, 2, 1, 1, 1, 0]
    roof, table = bench.roofline([_info(ms, by, fl, calls)])
    assert roof["kernel"] == "update" and roof["bound"] == "mfma"
    assert abs(roof["achieved"] - 5e11 / 1e-2 / 1e12) < 1e-9
    assert abs(roof["frac"] - roof["achieved"] / 78.6) < 1e-4
    assert roof["launches"] == 10 and abs(roof["avg_launch_us"] - 1000.0) < 1e-9
    assert abs(table["spmm"]["GB_s"] - 8e9 / 1e-3 / 1e9) < 1e-6


def test_traffic_figure_only_for_unchanged_kernel_source(tmp_path, monkeypatch):
    import hashlib

    import bench

    csrc = tmp_path / "paper_2409_05572_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "k.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha256(b"kernel v1\n").hexdigest()
    (tmp_path / "profiles" / "update_w_hbm_traffic.md").write_text(
        f"# t\n\nsource: k.hip\nsource_sha256: {sha}\nbytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("update", "w") == 1234.0
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("update", "w") is None
    assert bench.measured_traffic("gram", "w") is None


def test_cpu_baseline_leg_runs_every_solver_option():
    """The oracle leg of the benchmark accepts each solver with the options it
    forwards (expansion vectors, filter degree, preconditioner) and reports a
    bounded sample in the contract's fields."""
    import argparse

    import workloads as W

    A = W.laplacian_2d(12)
    X0 = W.gaussian_block(A.n, 8, 3)
    cases = [dict(solver="lobpcg", precond="jacobi"), dict(solver="sd", expand_vectors="random"),
             dict(solver="si", filter_degree=4, expand_vectors="powered"), dict(solver="tracemin")]
    for c in cases:
        args = argparse.Namespace(n_ev=4, n_extra=4, strategy="fix", cpu_seconds=5.0, cpu_iterations=5,
                                  x0_seed=3, expand_vectors="xdrop", filter_degree=0, precond="none")
        for k, v in c.items():
            setattr(args, k, v)
        out = bench.cpu_baseline(A, X0, args, 20, lambda *a: None)
        assert out["kind"] == "oracle" and out["value"] >= 0 and out["cores"] >= 1, c
        assert "iteration" in out["sample"]
        host = out["host"]
        assert host["nproc"] >= 1 and host["affinity"] >= 1 and out["cores"] >= 1, c


def test_cpu_baseline_times_iterations_after_the_initial_rayleigh_ritz():
    """The sample is the requested number of full iterations, timed from the
    oracle's timestamp at the start of the first one."""
    import argparse

    import workloads as W

    A = W.laplacian_3d(20)
    X0 = W.gaussian_block(A.n, 24, 3)
    args = argparse.Namespace(n_ev=16, n_extra=8, strategy="none", cpu_seconds=60.0, cpu_iterations=5,
                              x0_seed=3, expand_vectors="xdrop", filter_degree=0, precond="none",
                              solver="lobpcg")
    out = bench.cpu_baseline(A, X0, args, 100, lambda *a: None)
    assert out["sample"].startswith("5 FP64 LOBPCG iteration(s)")
    assert out["value"] > 0
