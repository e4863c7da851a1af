"""Host logic of the benchmark line: the work each form is charged with, the
traffic record's validity check and the one-GPU contract (no GPU needed)."""
import dataclasses
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2509_16896_amd import workloads as W  # noqa: E402


def test_algorithmic_flops_of_the_method():
    w = W.cubic_r1000()
    # two products (x.x and x.f) of r multiply-adds for every ordered pair
    assert bench.alg_flops(w) == 2.0 * 65536 * 65536 * 1000 * 2
    w1 = dataclasses.replace(w, scales=(1.0,))
    assert bench.alg_flops(w1) == 2.0 * 65536 * 65536 * 1000


def test_screened_work():
    w = W.cubic_r1000()
    n2 = 65536.0 * 65536.0
    # nothing flagged: only the screen's product, over the coordinates it uses; one run of 256 target
    # blocks takes the symmetric screen: block A against source tiles 2A .. 511, 65792 tiles of 256 x 128
    sym_pairs = 256.0 * 128.0 * sum(512 - 2 * a for a in range(256))
    assert sym_pairs == 256.0 * 128.0 * 65792
    alg, ex = bench.screened_work(w, "bf16x3p", 0, 131072)
    assert alg == ex == 2.0 * sym_pairs * 64
    # r <= 32 (a screen over 32 coordinates): every ordered pair
    narrow = W.shrink(w, r=32)
    alg, ex = bench.screened_work(narrow, "bf16x3p", 0, 131072)
    assert alg == ex == 2.0 * n2 * 32
    alg, ex = bench.screened_work(w, "bf16x3s", 0, 131072)
    assert alg == ex == 2.0 * n2 * 1000
    # every tile flagged: the method's products on top, executed twice over by the split form
    alg, ex = bench.screened_work(w, "bf16x3p", 131072, 131072)
    assert alg == 2.0 * sym_pairs * 64 + bench.alg_flops(w)
    assert ex == 2.0 * sym_pairs * 64 + 2.0 * bench.alg_flops(w)
    # 32 target blocks or fewer: every ordered pair
    mid = W.shrink(w, n=8192)
    assert bench.screen_pairs(8192, "bf16x3p") == 8192.0 * 8192.0
    assert bench.screen_pairs(8193, "bf16x3p") == 256.0 * 128.0 * sum(65 - 2 * a for a in range(33))
    assert bench.screen_pairs(8193, "bf16x3p", r=32) == 8193.0 * 8193.0
    assert bench.screened_work(mid, "bf16x3p", 0, 1)[0] == 2.0 * 8192 * 8192 * 64
    # a run narrower than the prefix screens all its coordinates
    small = W.shrink(w, r=20, n=1024)
    assert bench.screened_work(small, "bf16x3p", 0, 32)[0] == 2.0 * 1024 * 1024 * 20


def test_paper_sizes_match_the_workloads():
    assert tuple(bench.PAPER_E1) == W.PAPER_E1_SIZES
    for r, n in W.PAPER_E1_SIZES:
        w = W.paper_e1(r)
        assert (w.r, w.n, w.K, w.dt, w.h_shift, w.R, w.restart_every) == (r, n, 1000, 0.01, 100.0, 0.3, 2)


def test_traffic_record_needs_matching_form_and_source(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    f.write_text("traffic_prec = bf16x3p\ntraffic_source_hash = %s\ntraffic_bytes_per_launch = 1.5e+08\n"
                 % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"bf16x3p": str(f), "bf16x3g": str(f)})
    assert bench.recorded_traffic("bf16x3p") == 1.5e8
    assert bench.recorded_traffic("bf16x3s") is None
    assert bench.recorded_traffic("bf16x3g") is None     # the record covers another form
    f.write_text("traffic_prec = bf16x3p\ntraffic_source_hash = 0000\ntraffic_bytes_per_launch = 1.5e+08\n")
    assert bench.recorded_traffic("bf16x3p") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
