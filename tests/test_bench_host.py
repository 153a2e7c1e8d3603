"""Host arithmetic of the benchmark (no GPU): the roofline of each kind of
plan against counts worked by hand, the paper's normalized errors (Results,
"Accuracy Analysis", Eq. (2) and Eq. (3)) on a small example worked by hand,
and the guard that keeps the benchmark on one GPU."""
import math
import os
import subprocess
import sys

import numpy as np

import bench

E, B, NG = 134217728, 64, 1136           # the 4x4 slice, passes of 64
VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9        # CUs x SIMDs x lanes x FMA x clock


def test_valu_plan_counts_24_flops_per_entry_update():
    t = 4.6e-3
    r = bench.roofline(E, NG, B, 16, 16, 1, t, variant=2)
    assert r["bound"] == "alu"
    assert r["algorithmic_flops_per_launch"] == 24 * E * B
    assert math.isclose(r["frac"], 24 * E * B / t / VALU_PEAK, rel_tol=1e-12)
    assert "mfma_direct" not in r and "all_flops_vs_valu_peak" not in r


def test_mfma_plan_reports_the_direct_term_against_the_matrix_peak():
    t = 4.6e-3
    r = bench.roofline(E, NG, B, 16, 16, 1, t, variant=4)
    assert r["bound"] == "alu"
    assert r["algorithmic_flops_per_launch"] == 16 * E * B           # exchange only
    assert r["mfma_direct"]["flops_per_launch"] == 8 * E * B
    assert math.isclose(r["mfma_direct"]["frac"], 8 * E * B / t / 157.3e12, rel_tol=1e-12)
    assert math.isclose(r["all_flops_vs_valu_peak"], 24 * E * B / t / VALU_PEAK, rel_tol=1e-12)
    # both PH channels: two direct terms on the matrix cores, both exchange sums counted
    r2 = bench.roofline(E, NG, B, 16, 16, 3, t, variant=4)
    assert r2["mfma_direct"]["flops_per_launch"] == 16 * E * B
    assert r2["algorithmic_flops_per_launch"] == 32 * E * B
    # a direct term computed in a separate pass: not counted in this launch at all
    r3 = bench.roofline(E, NG, B, 8, 16, 1, t, variant=2, direct_elsewhere=True)
    assert r3["algorithmic_flops_per_launch"] == 16 * E * B and "mfma_direct" not in r3


def test_plain_pass_is_bound_by_hbm():
    t = 0.95e-3
    r = bench.roofline(E, NG, 1, 16, 16, 1, t)
    want_bytes = 2 * 16 * E + 2 * NG * NG * 16          # accumulator both ways, both G once
    assert r["bound"] == "hbm"
    assert r["algorithmic_bytes_per_launch"] == want_bytes
    assert math.isclose(r["frac"], want_bytes / t / 8e12, rel_tol=1e-12)


def test_paper_errors_on_a_hand_example():
    want = np.array([1 + 2j, -3 + 0j, 0 + 4j])
    got = want + np.array([0.1 + 0j, 0 - 0.2j, 0.3 + 0.1j])
    e = bench.paper_errors(got, want)
    # Eq. (2): sum |got - want| / sum |want| on each part; Eq. (3): the same with 2-norms
    assert math.isclose(e["eq2_l1_re"], 0.4 / 4.0)
    assert math.isclose(e["eq2_l1_im"], 0.3 / 6.0)
    assert math.isclose(e["eq3_l2_re"], math.sqrt(0.10) / math.sqrt(10.0))
    assert math.isclose(e["eq3_l2_im"], math.sqrt(0.05) / math.sqrt(20.0))
    assert math.isclose(e["rel_fro_vs_fp64_oracle"], math.sqrt(0.15) / math.sqrt(30.0))


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""
