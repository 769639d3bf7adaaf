"""Host logic of bench.py (no GPU): the one-GPU refusal, the grid and spectral sizes of the
byte model, properties that model must have, and the rule that counter traffic is reported only
for the kernel source it was measured on."""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402

KERNELS = ["ch_rhs", "weno_adv_fine", "fft_x_fwd_fine", "fft_y_fwd_fine", "zpass_ch", "fft_y_inv_fine",
           "fft_x_inv_fine", "restrict_g", "momentum_rhs", "fft_x_fwd_coarse", "fft_y_fwd_coarse",
           "zpass_ns", "fft_y_inv_coarse", "fft_x_inv_coarse", "fft_xy_fwd_coarse",
           "fft_xy_inv_coarse", "polymer_stage1", "polymer_stage2", "polymer_rk2"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_grid_sizes_follow_the_refinement():
    F, C = bench.grid_sizes(W.config("C2"))
    assert (F["nx"], F["ny"], F["nz"]) == (256, 256, 128)
    assert (C["nx"], C["ny"], C["nz"]) == (128, 128, 64)
    assert F["cells"] == 8 * C["cells"] == 8388608
    assert F["spec"] == 129 * 256 * 128 and C["spec"] == 65 * 128 * 64
    # single resolution: the phase field on the flow grid
    F, C = bench.grid_sizes(W.config("C2S"))
    assert F == C and F["nx"] == 256
    # 2D: no refinement across the single y cell
    F, C = bench.grid_sizes(W.config("C1"))
    assert F["ny"] == C["ny"] == 1 and F["cells"] == 4 * C["cells"]


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C3L", "C3P", "C2R", "C2S", "C4"])
def test_byte_model_properties(name):
    cfg = W.config(name)
    for k in KERNELS:
        b32, b64 = bench.alg_bytes(k, cfg, 4), bench.alg_bytes(k, cfg, 8)
        assert b64 == 2 * b32 >= 0, k
    # the polymer stages move bytes only when there is a polymer
    for k in ("polymer_stage1", "polymer_stage2", "polymer_rk2"):
        assert (bench.alg_bytes(k, cfg, 8) > 0) == bool(cfg.viscoelastic), k
    # y transforms only where there is a y direction
    for k in ("fft_y_fwd_fine", "fft_y_inv_fine", "fft_y_fwd_coarse", "fft_y_inv_coarse"):
        assert (bench.alg_bytes(k, cfg, 8) > 0) == (cfg.ny > 1), k


def test_weno_moves_the_velocity_reads_out_of_ch_rhs():
    central, weno = W.config("C3L"), W.config("C3P")
    F, C = bench.grid_sizes(central)
    assert bench.alg_bytes("weno_adv_fine", central, 8) == 0
    assert bench.alg_bytes("weno_adv_fine", weno, 8) > 0
    # with the advection precomputed ch_rhs reads it (one fine field) instead of six coarse ones
    diff = bench.alg_bytes("ch_rhs", weno, 8) - bench.alg_bytes("ch_rhs", central, 8)
    assert diff == 8 * (F["cells"] - 6 * C["cells"])


def test_traffic_is_reported_only_for_the_measured_source_and_workload(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_2111_04577_amd", "csrc"), root / "paper_2111_04577_amd" / "csrc")
    (root / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.traffic_entry("restrict_g", 32, "C5") is None  # no counter summary at all
    entry = {"source_sha": bench.source_sha("restrict_g"), "bytes_per_launch": 12345}
    (root / "profiles" / "traffic.json").write_text(json.dumps({"restrict_g/fp32/C5": entry}))
    assert bench.traffic_entry("restrict_g", 32, "C5") == 12345
    assert bench.traffic_entry("restrict_g", 64, "C5") is None
    # taken on another workload: not reported for this one
    assert bench.traffic_entry("restrict_g", 32, "C2") is None
    # a change to a shared header makes the stored figure stale
    hdr = root / "paper_2111_04577_amd" / "csrc" / "common.hpp"
    hdr.write_text(hdr.read_text() + "\n// edited\n")
    assert bench.traffic_entry("restrict_g", 32, "C5") is None


def test_compulsory_byte_model():
    """18.5 / 24.75 words per fine cell in 3D (Newtonian / viscoelastic), 21.5 / 28.25 in 2D."""
    assert bench.compulsory_bytes_per_cell(W.config("C2"), 4) == 74
    assert bench.compulsory_bytes_per_cell(W.config("C5"), 4) == 99
    assert bench.compulsory_bytes_per_cell(W.config("C5"), 8) == 198
    assert bench.compulsory_bytes_per_cell(W.config("C1"), 8) == 172
    assert bench.compulsory_bytes_per_cell(W.config("C4"), 8) == 226


def test_headline_defaults():
    """The headline workload is the largest single-GPU one, timed 10 + 200 by default."""
    import sys
    old = sys.argv
    sys.argv = ["bench.py"]
    try:
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.config == "C5" and a.steps == 200 and a.warmup == 10
    assert "C5" not in a.others.split(",")


def test_oracle_rates_record():
    """The oracle-rate leg times the oracle itself (fine cells x steps / seconds) on every CPU;
    checked on a short C1 run."""
    out = bench.oracle_rates(W, plan=(("C1", 2),))
    rec = out["C1"]
    F, _ = bench.grid_sizes(W.config("C1"))
    assert rec["steps"] == 2 and rec["cores"] == (os.cpu_count() or 1)
    # seconds carries two decimals: value x seconds is the cell-update count to within value x 0.005
    assert rec["value"] > 0 and abs(rec["value"] * rec["seconds"] - 2 * F["cells"]) <= rec["value"] * 0.0051
