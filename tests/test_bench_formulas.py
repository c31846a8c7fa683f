"""The benchmark's roofline bookkeeping against the definitions it reports:
method flops 4P + 5 log2 N + 8 per complex pol-sample (4 for one
polarisation), algorithmic bytes = the int8 input (2 B per pol-sample) plus
the dumps (4 B per product and channel per dump), the per-kernel split of the
flops (the four-step twiddle is not method work), and the matrix-core dense
flops of the split-FP16 passes.  CPU only; no GPU is touched."""
import numpy as np

import bench


def test_step_flops_match_the_method_count():
    c3 = bench.WORKLOADS["c3"]
    assert bench.step_flops_per_pol_sample(c3) == 8 * 4 + 5 * 19 + 8 == 135
    c2 = bench.WORKLOADS["c2"]
    assert bench.step_flops_per_pol_sample(c2) == 32 + 75 + 8
    c1 = bench.WORKLOADS["c1"]
    assert bench.step_flops_per_pol_sample(c1) == 32 + 50 + 4
    direct = bench.WORKLOADS["c2-direct"]
    assert bench.step_flops_per_pol_sample(direct) == 75 + 8


def test_kernel_flops_add_up_to_the_step():
    w = bench.WORKLOADS["c3"]
    N1, N2 = 2048, 256
    parts = sum(bench.flops_per_pol_sample(k, w, N1, N2) for k in ("column_pass", "row_pass"))
    assert parts == bench.step_flops_per_pol_sample(w)
    assert bench.flops_per_pol_sample("column_pass", w, N1, N2) == 32 + 40   # no twiddle flops
    assert bench.flops_per_pol_sample("single_pass", bench.WORKLOADS["c1"], 1, 1024) == \
        bench.step_flops_per_pol_sample(bench.WORKLOADS["c1"])


def test_algorithmic_bytes_are_input_and_dumps():
    w = bench.WORKLOADS["c3"]
    # 2 B of int8 input per pol-sample; 4 products x 4 B per channel per dump of
    # n_int spectra, shared by the two polarisations
    dump = 4.0 * 4 / (w["n_int"] * 2)
    assert bench.alg_bytes_per_pol_sample("column_pass", w) == 2.0
    assert bench.alg_bytes_per_pol_sample("row_pass", w) == 0.0
    assert np.isclose(bench.alg_bytes_per_pol_sample("dump_reduce", w), dump)
    assert np.isclose(2.0 + dump, 2.125)


def test_matrix_core_flops_of_the_split_fp16_passes():
    w = bench.WORKLOADS["c3"]
    # 2048-point rows: one radix-8 pass in FP32 and two radix-16 passes on the
    # matrix cores, 6 products of 16x16x32 (16384 flops) per 256 points each
    assert bench.mfma_flops_per_pol_sample("row_pass", "mixed", w, 2048, 256) == 2 * 6 * 16384 / 256
    assert bench.mfma_flops_per_pol_sample("column_pass", "mixed", w, 2048, 256) == 0
    assert bench.mfma_flops_per_pol_sample("column_pass", "fp16x2", w, 2048, 256) == 768
    assert bench.mfma_flops_per_pol_sample("row_pass", "fp16", w, 2048, 256) == 2 * 2 * 16384 / 256
    assert bench.mfma_flops_per_pol_sample("row_pass", "fp32", w, 2048, 256) == 0


def test_bench_refuses_more_than_one_gpu():
    """The spectrometer runs on one GPU; asked for several, the benchmark
    exits with status 2 and says why, before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
