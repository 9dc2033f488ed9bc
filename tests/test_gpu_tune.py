"""Measured work decomposition (nfft_plan_tune, nfft_plan_create_params) through the C ABI.

The bin edges and work-item cap change only how the sums are split among workgroups, so a
plan created with tuned (or any accepted) parameters must agree with the default plan to
rounding and with the FP64 oracle to the usual bars.  The tuning cache answers a shape it
holds without timing, and keeps one line per shape.
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, host, parity_err, rel_l2
from oracle import oracle as O
from paper_1810_09891_amd import Plan, tune_plan_params, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
SAME = {C64: 1e-6, C128: 1e-14}


def _run(p, c, dtype):
    p.set_nodes(dev(c["x"], torch.float64))
    return host(p.trafo(dev(c["fhat"], dtype))), host(p.adjoint(dev(c["f"], dtype)))


@pytest.mark.parametrize("d,N,M,m,dtype,kind", [
    (2, (128, 128), 20000, 6, C64, "uniform"),
    (2, (96, 64), 8000, 8, C128, "clustered"),
    (3, (24, 32, 16), 6000, 4, C128, "uniform"),
    (1, (512,), 4000, 8, C64, "clustered"),
])
def test_tuned_parameters_agree_with_defaults(tmp_path, d, N, M, m, dtype, kind):
    announce("plan tune", d, N, M, m, dtype, kind)
    c = W.small_case(d, N, M, seed=600 + d + m, kind=kind)
    cache = str(tmp_path / "plans.txt")
    params, ms = tune_plan_params(N, M, dev(c["x"], torch.float64), m=m, dtype=dtype, cache=cache)
    assert ms > 0
    assert len(params["bin"]) == d and all(b >= 1 and b & (b - 1) == 0 for b in params["bin"])
    assert params["chunk_cap"] in (128, 256, 512, 1024)
    p = Plan(N, M, m=m, dtype=dtype, params=params)
    assert tuple(int(p.info.bin[t]) for t in range(d)) == tuple(params["bin"])
    assert int(p.info.chunk_cap) == params["chunk_cap"]
    f, h = _run(p, c, dtype)
    f0, h0 = _run(Plan(N, M, m=m, dtype=dtype), c, dtype)
    assert rel_l2(f0, f) <= SAME[dtype] and rel_l2(h0, h) <= SAME[dtype]
    n = tuple(int(v) for v in p.n)
    assert parity_err(O.nfft_trafo(c["x"], c["fhat"], n, m), f) < TOL[dtype]
    assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, n, m), h) < TOL[dtype]
    # the cache answers the same shape without timing, and holds one line for it
    again, ms2 = tune_plan_params(N, M, dev(c["x"], torch.float64), m=m, dtype=dtype, cache=cache)
    assert again == params and ms2 == 0.0
    lines = [l for l in open(cache).read().splitlines() if l and not l.startswith("#")]
    assert len(lines) == 1 and lines[0].split()[0].startswith("plan-d%d-" % d)


@pytest.mark.parametrize("bins,cap", [((8, 8), 128), ((16, 64), 1024), ((64, 16), 256), ((32, 32), 64)])
def test_every_accepted_decomposition_computes_the_same_sums(bins, cap):
    """Forced bin edges and caps (including ones the rule never picks) against the defaults."""
    N, M, m = (64, 64), 9000, 6
    announce("plan params", bins, cap)
    c = W.small_case(2, N, M, seed=640, kind="clustered")
    f, h = _run(Plan(N, M, m=m, dtype=C128, params={"bin": bins, "chunk_cap": cap}), c, C128)
    f0, h0 = _run(Plan(N, M, m=m, dtype=C128), c, C128)
    assert rel_l2(f0, f) <= 1e-14 and rel_l2(h0, h) <= 1e-14
    assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, (128, 128), m), h) < TOL[C128]
