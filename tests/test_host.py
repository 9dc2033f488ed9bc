"""Host-side checks that need no GPU: the benchmark's one-GPU contract and the seeded
workload generators shared by the oracle and the HIP path."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1810_09891_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


@pytest.mark.parametrize("name", ["d1", "d2", "grad", "nnfft_d2"])
def test_workloads_are_seeded_and_in_range(name):
    a = W.workload(name)
    b = W.workload(name)
    for key in ("x", "f"):
        assert np.array_equal(a[key], b[key])
    x = a["x"]
    assert x.dtype == np.float64 and x.shape == (a["M"], len(a["N"]))
    assert np.all(x >= -0.5) and np.all(x < 0.5)
    if name == "nnfft_d2":
        v = a["v"]
        assert np.array_equal(v, b["v"])
        assert v.shape == (a["K"], 2) and a["fhat"].shape == (a["K"],)
        assert np.all(v >= -np.asarray(a["N"]) / 2) and np.all(v < np.asarray(a["N"]) / 2)
    else:
        assert a["fhat"].shape == tuple(a["N"])
    # a different stream draws different numbers
    c = W.workload(name, stream=1)
    assert not np.array_equal(a["x"], c["x"])


def test_complex_gaussian_moments():
    z = W.cgauss(np.random.default_rng(3), (200000,))
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.02
    assert abs(np.mean(z)) < 0.01


def test_bench_byte_model():
    """The byte model of the benchmark's roofline: window steps move the FP64 nodes, the
    values and the grid once; FFT passes their nonzero input and their output.  Pinned to
    the sizes of the d = 2 (N = 512^2, M = 262144) and d = 3 (N = 128^3, M = 2,097,152)
    workloads worked out by hand."""
    sys.path.insert(0, ROOT)
    import bench

    ab = bench.algorithmic_bytes
    # window: M (8 d + c) + |I_n| c
    assert ab("spread_own", 2, (512, 512), (1024, 1024), 262144, 8) == 262144 * 24 + 1024 ** 2 * 8 == 14680064
    assert ab("interp", 3, (128,) * 3, (256,) * 3, 2097152, 16) == 2097152 * 40 + 256 ** 3 * 16
    # FFT, complex64, d = 2: first pass 512 rows of (512 in, 1024 out), then 1024 columns
    assert ab("fft_fwd_deconv", 2, (512, 512), (1024, 1024), 1, 8) == 8 * 512 * (512 + 1024)
    assert ab("fft_fwd", 2, (512, 512), (1024, 1024), 1, 8) == 8 * 1024 * (512 + 1024)
    # d = 3: passes over dimension 2, 1, 0 total 352 MB per transform in complex64
    first = ab("fft_fwd_deconv", 3, (128,) * 3, (256,) * 3, 1, 8)
    rest = ab("fft_fwd", 3, (128,) * 3, (256,) * 3, 1, 8) * 2
    assert first == 8 * 128 * 128 * 384 and first + rest == 8 * 384 * (128 * 128 + 128 * 256 + 256 * 256)
    assert ab("fft_adj_deconv", 3, (128,) * 3, (256,) * 3, 1, 8) == first
    # VALU issue time of the d = 3 window step: 14^3 pairs x 2 slots per node
    assert abs(bench.valu_seconds(3, 2097152, 6, True) - 2097152 * 2744 * 2 / (256 * 64 * 2.4e9)) < 1e-12
    e = bench.roofline_entry("interp", 1.0, 3, (128,) * 3, (256,) * 3, 2097152, 6, 16, True)
    assert e["binding"] == "valu" and abs(e["binding_frac"] - 2097152 * 2744 * 2 / (256 * 64 * 2.4e9) / 1e-3) < 1e-3
    # the 3-D spreading by output tiles runs on the matrix cores: 4 flops per pair at the
    # dense FP64 (78.6 TFLOP/s) or FP32 (157.3 TFLOP/s) MFMA peak
    e = bench.roofline_entry("spread_own", 1.0, 3, (128,) * 3, (256,) * 3, 2097152, 6, 16, True)
    assert e["binding"] == "mfma" and abs(e["binding_frac"] - 2097152 * 2744 * 4 / 78.6e12 / 1e-3) < 1e-4
    e = bench.roofline_entry("spread_own", 1.0, 3, (128,) * 3, (256,) * 3, 2097152, 6, 8, False)
    assert abs(e["binding_frac"] - 2097152 * 2744 * 4 / 157.3e12 / 1e-3) < 1e-4
