"""Host logic of bench.py (no GPU): the refusal of more than one GPU, the
algorithmic byte counts the roofline divides by, and the traffic summary's
copy calibration on synthetic counter databases."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("q,prec,qh,expect", [
    # read and write both distributions once and the carried phi:
    # (2 Q + 2 Qh + 2) values of the storage type
    (19, "fp64", None, (4 * 19 + 2) * 8), (19, "fp32", None, (4 * 19 + 2) * 4),
    (9, "fp64", None, (4 * 9 + 2) * 8), (19, "fp64", 7, (2 * 19 + 2 * 7 + 2) * 8),
    (7, "fp32", None, (4 * 7 + 2) * 4),
    # deviation formats: per distribution Q - 1 16-bit codes and an FP32 rest
    # population, read and written, plus FP32 phi and Lambda
    (19, "fp16dev", None, 2 * (2 * (18 * 2 + 4) + 4 + 4)),
    (9, "bf16dev", None, 2 * (2 * (8 * 2 + 4) + 4 + 4)),
    (19, "fp16dev", 7, 2 * ((18 * 2 + 4) + (6 * 2 + 4) + 4 + 4)),
    (7, "fp16dev", None, 2 * (2 * (6 * 2 + 4) + 4 + 4)),
])
def test_algorithmic_bytes(q, prec, qh, expect):
    assert bench.bytes_per_node_step(q, prec, qh) == expect


def test_adjoint_bytes():
    # on D2Q9: 58 FP64 values of the adjoint arrays and accumulators per node,
    # and 21 of the two forward states (2 x 9 H pulls, 3 phi reads)
    assert bench.adjoint_bytes_per_node(9, 2, "fp64") == 8 * 58 + 8 * 21 == 632
    assert bench.adjoint_bytes_per_node(9, 2, "fp32") == 8 * 58 + 4 * 21
    # a deviation state: per H read 8 codes, the rest population and Lambda
    assert bench.adjoint_bytes_per_node(9, 2, "fp16dev") == 8 * 58 + 2 * (8 * 2 + 4 + 4) + 3 * 4


def _counter_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_summary_calibration(tmp_path):
    """The 4 GiB calibration negation launched as two dispatches of 2 GiB:
    their counters are summed, so a counter that reads half of the true
    fetched bytes gives a fetch scale of 2 and the step's bytes come out
    right."""
    kib4 = 4 * (1 << 20)
    step = "void gplbm::k_fused3d<64, 6, 32>(...)"
    neg = "void at::native::vectorized_elementwise_kernel<neg_kernel_cuda>"
    f = tmp_path / "f.db"
    w = tmp_path / "w.db"
    _counter_db(f, [(neg, "FETCH_SIZE", kib4 / 4), (neg, "FETCH_SIZE", kib4 / 4),
                    (step, "FETCH_SIZE", 1000.0), (step, "FETCH_SIZE", 1200.0)])
    _counter_db(w, [(neg, "WRITE_SIZE", kib4 / 2), (neg, "WRITE_SIZE", kib4 / 2),
                    (step, "WRITE_SIZE", 700.0)])
    out = tmp_path / "t.json"
    bench.summarize_profile("traffic", [str(f), str(w)], str(out), "porous3d_512_d3q19", "fp64",
                            "fused")
    d = json.loads(out.read_text())
    assert d["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert d["calibration"]["write_scale"] == pytest.approx(1.0)
    k = d["kernels"][step]
    assert k["read_bytes"] == pytest.approx(1100.0 * 1024 * 2)   # mean over dispatches
    assert k["write_bytes"] == pytest.approx(700.0 * 1024)
    assert d["bytes_per_step"] == pytest.approx(1100.0 * 1024 * 2 + 700.0 * 1024)
    assert d["source_hash"] == bench.kernel_source_hash()
