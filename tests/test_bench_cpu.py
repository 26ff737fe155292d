"""The benchmark's byte models and JSON fields, on the host (no GPU):

  - the per-sweep algorithmic bytes at the Chung-Lu workload come to
    402.8 MB (n = 2^20, 32M stored entries, R = 16, FP32, weighted), and
    the R-MAT BF16 and FP32 sweeps to 5.37 / 6.44 GB at 256e6 edges
    (5.57 GB in BF16 at the 2^28 edges run);
  - a step's sweeps follow the storage schedule (BF16, then FP32, then the
    FP64 tail) and reduce to the plain FP32 sweep with no tails;
  - the distance pass counts row pointers, columns, one edge id and one
    distance per edge, and the vector block once;
  - the roofline object divides algorithmic bytes by the average launch and
    by the 8 TB/s figure;
  - more than one GPU is refused with a message, before any GPU work.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sweep_bytes_at_the_stated_workloads():
    n, nnz, R = 1 << 20, 32_000_000, 16
    assert bench.sweep_bytes(n, nnz, R, 4, True) == 402_800_648          # "402.8 MB per FP32 sweep"
    nr = 1 << 24                        # R-MAT scale 24
    bf16 = bench.sweep_bytes(nr, 2 * 256_000_000, R, 2, True)
    f32 = bench.sweep_bytes(nr, 2 * 256_000_000, R, 4, True)
    assert round(bf16 / 1e9, 2) == 5.37 and round(f32 / 1e9, 2) == 6.44
    # the workload as run (2^28 edges): 5.57 / 6.64 GB
    assert round(bench.sweep_bytes(nr, 2 << 28, R, 2, True) / 1e9, 2) == 5.57
    assert bench.sweep_bytes(n, nnz, R, 4, False) == 402_800_648 - 4 * nnz   # unit weights: no weight stream


def test_relax_schedule_bytes():
    n, nnz, R, k = 1000, 8000, 16, 30
    plain = bench.relax_sweep_bytes(n, nnz, R, k, True, 4, k, 0)
    assert plain == [bench.sweep_bytes(n, nnz, R, 4, True)] * k
    mixed = bench.relax_sweep_bytes(n, nnz, R, k, True, 2, 12, 1)
    # x^(0) FP32 -> 18 BF16 sweeps -> 11 FP32 -> 1 FP64
    assert mixed[0] == bench.sweep_bytes(n, nnz, R, 4, True, 2)
    assert mixed[1:18] == [bench.sweep_bytes(n, nnz, R, 2, True)] * 17
    assert mixed[18] == bench.sweep_bytes(n, nnz, R, 2, True, 4)
    assert mixed[19:29] == [bench.sweep_bytes(n, nnz, R, 4, True)] * 10
    assert mixed[29] == bench.sweep_bytes(n, nnz, R, 4, True, 8)
    tail = bench.relax_sweep_bytes(n, nnz, R, 20, True, 4, 20, 3)
    assert tail[-3:] == [bench.sweep_bytes(n, nnz, R, 4, True, 8)] + [bench.sweep_bytes(n, nnz, R, 8, True)] * 2


def test_dist_bytes():
    n, m, R = 1 << 20, 16_000_000, 16
    nnz = 2 * m
    got = bench.dist_bytes(n, nnz, m, R, 8)
    assert got == (n + 1) * 8 + 4 * nnz + 4 * m + n * R * 8 + 4 * m


def test_roofline_fraction():
    kern = {"k_sweep": (20, 8.0)}                  # 20 launches, 8 ms in all
    roof = bench.roofline(kern, 4.0e8, None)
    assert roof["avg_launch_ms"] == pytest.approx(0.4)
    assert roof["achieved"] == pytest.approx(4.0e8 / 0.4e-3 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
