"""Oversampled grid lengths that are any even number (not only powers of two).

The paper's n-sweeps (Sec. 4.3.1, Fig. 4.1(a) d = 1, N = 512, n = 514 ... 820; Fig. 4.2(a)
d = 2, N = 128^2, n = 130, 154, 180) use lengths with large odd prime factors (514 = 2 * 257,
614 = 2 * 307, 716 = 4 * 179, 820 = 4 * 5 * 41, 130 = 2 * 5 * 13, 154 = 2 * 7 * 11).  Checked
through the C ABI against the FP64 oracle at the same n (parity bar 1e-12 complex128,
5e-6 complex64), and the GPU's E_2 against the direct sums reproduces the oracle's value
stored for the figure.  Also: 3-D plans on and off the output-tile spreading path, line
lengths with several odd factors, the longest accepted line, batches mixing power-of-two
and other grids, and the node gradient.

Near n = N the deconvolution factors w_k = 1 / (n phi_hat(k)) span many orders of magnitude
(1.3e9 at n = 514, 1.3e16 over the 2-D grid at n = 130), and two FP64 evaluations of the same
algorithm that differ only in the rounding order of the FFT disagree by up to 2e-9 (n = 514)
or 0.1 (adjoint, n = 130) in plain relative l2: no implementation meets a 1e-12 relative bar
there.  Parity is therefore measured in the norms in which each last step is well-conditioned
(``error_scale``: the relative l2 error weighted by the forward error scale of each output,
and its element-wise form); two FP64 oracle evaluations meet these at 1e-13 on every grid of
the sweep.  Where n_t >= 2 N_t the plain relative bar is asserted as well.
"""
import json
import os

import numpy as np
import pytest
import torch

from error_scale import adjoint_errors, trafo_errors
from gpu_util import TOL, announce, dev, host, parity_err, rel_l2
from oracle import oracle as O
from paper_1810_09891_amd import NFFT_KEEP_GRID, Batch, Plan, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
# bars: e2 (the weighted relative l2 error) at the parity bar, emax (element-wise) at the
# parity bar in complex128 and 4x it in complex64, where the FP32 FFT's per-entry rounding
# reaches a few times its l2 average
EMAX = {C128: 1e-12, C64: 2e-5}
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_errors.json")))


def check(errs, dtype, what=""):
    e2, emax = errs
    assert e2 < TOL[dtype] and emax < EMAX[dtype], (what, e2, emax)


def _run(N, M, n, m, dtype, c):
    p = Plan(N, M, n=n, m=m, dtype=dtype)
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    return p, f, h


@pytest.mark.parametrize("n", [514, 614, 716, 820])
@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_fig_4_1_lengths_d1(n, dtype):
    """d = 1, N = 512, M = 1024 (the paper's test polynomial and node count), m = 8."""
    announce("grid sizes d1", n, dtype)
    w = W.paper_workload(1)
    N, M = w["N"], w["M"]
    r = np.random.default_rng(n)
    f_in = r.standard_normal(M) + 1j * r.standard_normal(M)
    c = {"x": w["x"], "fhat": w["fhat"], "f": f_in}
    p, f, h = _run(N, M, (n,), 8, dtype, c)
    check(trafo_errors(c["x"], c["fhat"], N, (n,), 8, f), dtype)
    check(adjoint_errors(c["x"], f_in, N, (n,), 8, h), dtype)
    if dtype == C128:
        # the approximation error of Fig. 4.1(a) against the direct sums, on the GPU
        ref = host(p.ndft_trafo(dev(c["fhat"], dtype)))
        e2 = rel_l2(ref, f)
        gold = GOLDEN["fig_4_1_E2"][str(n)]
        assert gold / 2 <= e2 <= gold * 2, (e2, gold)


@pytest.mark.parametrize("n", [130, 154, 180])
@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_fig_4_2_lengths_d2(n, dtype):
    """d = 2, N = (128, 128), M = 32768 (the paper's workload), m = 8."""
    announce("grid sizes d2", n, dtype)
    w = W.paper_workload(2)
    N, M = w["N"], w["M"]
    r = np.random.default_rng(n)
    f_in = r.standard_normal(M) + 1j * r.standard_normal(M)
    c = {"x": w["x"], "fhat": w["fhat"], "f": f_in}
    p, f, h = _run(N, M, (n, n), 8, dtype, c)
    check(trafo_errors(c["x"], c["fhat"], N, (n, n), 8, f), dtype)
    check(adjoint_errors(c["x"], f_in, N, (n, n), 8, h), dtype)
    # at n = 130 rounding (2.9e-3 between two FP64 evaluations) is as large as the
    # approximation error (1.7e-3), so the stored E_2 is not a property of the method there
    if dtype == C128 and n != 130:
        ref = host(p.ndft_trafo(dev(c["fhat"], dtype)))
        e2 = rel_l2(ref, f)
        gold = GOLDEN["fig_4_2_E2"][str(n)]
        assert gold / 2 <= e2 <= gold * 2, (e2, gold)


CASES = [
    # d, N, n, M, kind: odd factors 3, 5, 7, 11, 13 and mixed dimensions
    (1, (60,), (90,), 777, "uniform"),
    (1, (100,), (126,), 901, "uniform"),
    (1, (200,), (286,), 1500, "clustered"),
    (2, (40, 36), (50, 74), 2100, "uniform"),
    (2, (60, 44), (96, 70), 1999, "clustered"),
    (2, (20, 64), (42, 128), 1234, "uniform"),
    # 3-D, every n_t a multiple of 16: spreading by output tiles
    (3, (20, 20, 36), (32, 48, 80), 3001, "uniform"),
    (3, (24, 24, 24), (48, 48, 48), 2500, "clustered"),
    # 3-D, not multiples of 16: tile spreading
    (3, (20, 16, 14), (42, 38, 30), 1800, "uniform"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "d%d_n%s_%s" % (c[0], "x".join(map(str, c[2])), c[4]))
@pytest.mark.parametrize("dtype,m", [(C128, 4), (C128, 6), (C64, 4), (C64, 6)], ids=["c128m4", "c128m6", "c64m4", "c64m6"])
def test_trafo_adjoint_any_even_n(case, dtype, m):
    d, N, n, M, kind = case
    announce("grid sizes", d, N, n, M, kind, dtype, m)
    c = W.small_case(d, N, M, seed=400 + sum(n) + m, kind=kind)
    p, f, h = _run(N, M, n, m, dtype, c)
    check(trafo_errors(c["x"], c["fhat"], N, n, m, f), dtype)
    check(adjoint_errors(c["x"], c["f"], N, n, m, h), dtype)
    if all(nt >= 2 * Nt for nt, Nt in zip(n, N)):  # flat w_k: the plain relative bar holds too
        assert parity_err(O.nfft_trafo(c["x"], c["fhat"], n, m), f) < TOL[dtype]
        assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, n, m), h) < TOL[dtype]
    if d == 3 and all(v % 16 == 0 for v in n):
        assert p.info.own_tiles > 0


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_longest_line_with_large_prime_factor(dtype):
    """n = 4094 = 2 * 23 * 89, the longest accepted line length with an odd part."""
    N, n, M = (2000,), (4094,), 3000
    announce("grid sizes longest", n, dtype)
    c = W.small_case(1, N, M, seed=480)
    _, f, h = _run(N, M, n, 6, dtype, c)
    check(trafo_errors(c["x"], c["fhat"], N, n, 6, f), dtype)
    check(adjoint_errors(c["x"], c["f"], N, n, 6, h), dtype)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_batch_mixing_grid_kinds(dtype):
    """A batch whose plans have power-of-two and other grids: each batched result equals
    the per-plan call and agrees with the oracle."""
    specs = [((64, 64), (128, 128), 5000), ((60, 44), (130, 90), 4000), ((32, 32), (64, 64), 3000),
             ((50, 50), (154, 154), 6000), ((100, 20), (206, 42), 2500)]
    announce("grid sizes batch", dtype)
    plans, cases = [], []
    for i, (N, n, M) in enumerate(specs):
        c = W.small_case(2, N, M, seed=500 + i)
        p = Plan(N, M, n=n, m=6, dtype=dtype)
        p.set_nodes(dev(c["x"], torch.float64))
        plans.append(p)
        cases.append(c)
    fs = [host(p.trafo(dev(c["fhat"], dtype))) for p, c in zip(plans, cases)]
    hs = [host(p.adjoint(dev(c["f"], dtype))) for p, c in zip(plans, cases)]
    b = Batch(plans)
    bf = [host(v) for v in b.trafo([dev(c["fhat"], dtype) for c in cases])]
    bh = [host(v) for v in b.adjoint([dev(c["f"], dtype) for c in cases])]
    same = 1e-14 if dtype == C128 else 1e-6
    for i, (N, n, M) in enumerate(specs):
        assert rel_l2(fs[i], bf[i]) <= same, i
        assert rel_l2(hs[i], bh[i]) <= same, i
        check(trafo_errors(cases[i]["x"], cases[i]["fhat"], N, n, 6, bf[i]), dtype, i)
        check(adjoint_errors(cases[i]["x"], cases[i]["f"], N, n, 6, bh[i]), dtype, i)
    b.close()


@pytest.mark.parametrize("d,N,n,M", [(1, (50,), (126,), 300), (2, (30, 20), (70, 42), 600)])
def test_grad_x_any_even_n(d, N, n, M):
    announce("grid sizes grad_x", d, N, n)
    c = W.small_case(d, N, M, seed=520 + d)
    p = Plan(N, M, n=n, m=5, dtype=C128, flags=NFFT_KEEP_GRID)
    p.set_nodes(dev(c["x"], torch.float64))
    p.trafo(dev(c["fhat"], C128))
    g = p.grad_x(dev(c["f"], C128))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], n, 5), N, 5)
    ref = np.real(np.conj(c["f"])[:, None] * dfdx)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-12
