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
