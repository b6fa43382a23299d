"""Host-side checks of bench.py: the one-GPU contract, the argument checks,
and the algorithmic work it divides by the measured kernel times (the
per-unit figures of the kernel design: 27 and 31 window flops per (point,
direction) pair for spreading and gathering with W = 4, the chunk grids and
projection tiles each moved once)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_unknown_form_is_refused():
    r = _run("--form", "no_such_form")
    assert r.returncode == 2 and "unknown form" in r.stderr


def test_form_names():
    names = [n for n, _ in bench.form_runners(3)]
    assert len(names) == len(set(names))
    for n in ("precision_sorted", "mmd_energy_sorted", "batched_256", "mmd_flow_energy_d3072"):
        assert n in names


def test_window_flops_per_pair():
    # position 2, offset squared 1, two tap pairs of (even Horner 4, odd
    # Horner 2, two taps 4), then 4 weight products (spread) or 8
    # interpolation flops (gather)
    assert bench.WINDOW_FLOPS == {"spread": 27, "gather": 31}


def test_algorithmic_work_of_the_headline_step():
    N = M = 60000
    d, P, nr, chunks, groups = 50, 3500, 824, 15, 17
    info = dict(grid_nr=nr, fused=1, last_spread_chunks=chunks, last_gather_groups=groups)
    tiles = -(-N // 16) * 2 * 2 * 1024               # two k-blocks of hi + lo, 1 KB each
    byts, flops, bound = bench.algorithmic("project", info, N, M, d, P, "fp32")
    assert bound == "hbm" and byts == 2 * (N * d * 4 + tiles) and flops == 0.0
    byts, flops, bound = bench.algorithmic("spread", info, N, M, d, P, "fp32")
    assert bound == "alu"
    assert byts == pytest.approx(tiles + N * 4 + chunks * P * nr * 4)
    assert flops == 27 * N * P
    byts, flops, bound = bench.algorithmic("fftconv", info, N, M, d, P, "fp32")
    assert bound == "hbm" and byts == (chunks + 1) * P * nr * 4
    byts, flops, bound = bench.algorithmic("gather", info, N, M, d, P, "fp32")
    assert bound == "alu" and flops == 31 * M * P
    assert byts == pytest.approx(tiles + P * nr * 4 + groups * M * 8)
    byts, _, bound = bench.algorithmic("reduce", info, N, M, d, P, "fp32")
    assert bound == "hbm" and byts == groups * M * 8 + M * 4


def test_roofline_peaks():
    r = bench.roofline_of("alu", 0.0, 78.6e12 * 1e-3, 1e-3)
    assert r["peak"] == 78.6 and r["achieved"] == pytest.approx(78.6)
    r = bench.roofline_of("hbm", 8e9, 0.0, 1e-3)
    assert r["unit"] == "GB/s" and r["achieved"] == pytest.approx(8000.0)


def test_committed_traffic_is_reported_only_for_its_kernel_source(monkeypatch):
    """Each counter summary under profiles/ names the kernel-source hash it
    was taken on; the bench reports its bytes only while the source still
    has that hash (traffic null otherwise)."""
    for phase in ("project", "spread", "fftconv", "gather", "reduce"):
        path = os.path.join(bench.PROFILES, f"{phase}_scale_d50_P3500_traffic.txt")
        vals = dict(l.split(":", 1) for l in open(path) if ":" in l and not l.startswith("#"))
        taken = vals["kernel_source_sha256_16"].strip()
        assert float(vals["hbm_bytes_per_launch"]) > 0
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: taken)
        assert bench.measured_traffic(phase, 3500) == float(vals["hbm_bytes_per_launch"])
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
        assert bench.measured_traffic(phase, 3500) is None
