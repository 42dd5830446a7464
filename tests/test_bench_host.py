"""Host side of bench.py (no GPU): the byte model of the roofline, the rule
that uses the committed HBM counter summary only for the kernel sources,
mesh size and launch shape it was taken on, and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_cell_update():
    # rho, e per cell and u, v, w per node, read and written once: 32 B per
    # cell plus 48 B per node, 80.45 B per cell-update at 320^3
    n = 320
    per_cell = bench.algorithmic_bytes(n) / n ** 3
    assert per_cell == pytest.approx(32 + 48 * (n + 1) ** 3 / n ** 3)
    assert round(per_cell, 2) == 80.45
    assert bench.algorithmic_bytes(n, esz=4) == bench.algorithmic_bytes(n) // 2


def test_compulsory_bytes_exceed_the_algorithmic_ones():
    n = 320
    comp = bench.compulsory_bytes(n)
    assert set(comp) >= {"k_lagrange", "k_remap"}
    # the hand-off between the two kernels is written once and read once
    assert comp["k_lagrange"] + comp["k_remap"] > bench.algorithmic_bytes(n)


def test_counter_summary_used_only_where_it_was_taken(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    f = tmp_path / "traffic.md"
    f.write_text("counted on: 320^3, launch shape 16,16,3072 (tile rows of the two kernels, z-split target)\n"
                 "FP64 step: traffic bytes per step (fp64): 9.5e+09\n"
                 f"kernel sources sha256[:16]: {digest}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    shape = {"rows_a": 16, "rows_b": 16, "target": 3072}
    assert bench.measured_traffic(320, shape)[0] == pytest.approx(9.5e9)
    # the automatic split of a mesh this large equals the 3072-block target
    assert bench.measured_traffic(320, dict(shape, target=0))[0] == pytest.approx(9.5e9)
    assert bench.measured_traffic(480, shape)[0] is None
    assert bench.measured_traffic(320, dict(shape, rows_b=8))[0] is None
    f.write_text(f.read_text().replace(digest, "0" * 16))
    value, why = bench.measured_traffic(320, shape)
    assert value is None and "changed" in why


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
