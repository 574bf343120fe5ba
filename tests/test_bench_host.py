"""Host logic of bench.py, without a GPU: the single-GPU contract, the flop
accounting of the fused cell kernel, and the gating of figures recorded from
counter runs by the sources they were measured on."""
import json
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1212_3585_amd", "csrc")


def test_more_than_one_gpu_is_refused():
    for extra in ([], ["--amr-only"], ["--traffic-probe"]):
        r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"] + extra, cwd=ROOT,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2, (extra, r.returncode, r.stderr)
        assert "exactly one GPU" in r.stderr


def test_flop_counts_of_2d_euler_at_m3():
    # 2D Euler point flux: d^2 + 5 d + 3 = 17 flops; dt/dx scaling d nv = 8;
    # per node and variable: two 4-term derivative products (16), the 4-term
    # time product (8) and the subtraction from w_hat (1); 64 space-time nodes
    assert bench.predictor_flops_per_cell_iteration(2, 3, 4) == 64 * (17 + 8 + 4 * 25) == 8000
    # first sweep from w_hat: fluxes, scaling and derivatives at the 16
    # spatial nodes; then a product and a subtraction per space-time value
    assert bench.predictor_flops_first_sweep(2, 3, 4) == 16 * (17 + 8 + 4 * 16) + 64 * 4 * 2
    # WENO line, M = 3 (four stencils of four cells): inverse 2 n^2 = 32;
    # sigma from 6 Legendre coefficients of 4 products each, squared and
    # summed (6 x 10 = 60); the weight (5); then per stencil 2 for the
    # normalisation and 2 n = 8 for the combination
    assert bench.weno_flops_per_line(3) == 4 * (32 + 60 + 5) + 4 * 2 + 4 * 8 == 428


def test_cell_kernel_flops_add_up():
    ncells, sweeps = 1000, 11500
    weno = ncells * 4 * (1 + 4) * 428          # one x line and four y lines per variable
    picard = (sweeps - ncells) * 8000 + ncells * 1936
    traces = ncells * 2 * 2 * 4 * 16 * 2 * 4   # 4 faces x nv x n^2 values, 2 n flops each
    assert bench.cell_kernel_flops(2, 3, 4, sweeps, ncells) == weno + picard + traces


def test_recorded_figures_follow_the_sources(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        traffic = json.load(f)
    with open(bench.CLOCK_FILE) as f:
        clock = json.load(f)
    monkeypatch.setattr(bench, "device_source_hash", lambda: traffic["device_source_sha256"])
    assert bench.recorded_traffic() == traffic["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "device_source_hash", lambda: clock["device_source_sha256"])
    assert bench.recorded_clock_ghz() == clock["measured_clock_ghz"]
    monkeypatch.setattr(bench, "device_source_hash", lambda: "0" * 64)
    assert bench.recorded_traffic() is None
    assert bench.recorded_clock_ghz() is None


def test_hashed_sources_cover_every_file_the_cell_kernels_include():
    seen, todo = set(), [n for n in os.listdir(CSRC) if n.startswith("cell2d_rows")
                         and n.endswith(".hip")] + ["impl2d.hip"]
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        seen.add(name)
        with open(os.path.join(CSRC, name)) as f:
            for inc in re.findall(r'#include "([^"]+)"', f.read()):
                base = os.path.basename(inc)
                if os.path.exists(os.path.join(CSRC, base)):
                    todo.append(base)
    missing = sorted(seen - set(bench.CELL_KERNEL_SOURCES))
    assert not missing, missing
