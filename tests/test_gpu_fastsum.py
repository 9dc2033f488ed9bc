"""Fast summation (nfft_fastsum) against the FP64 oracle.

g_j = sum_l alpha_l K(y_j - x_l) for K(z) = sum_k bhat_k e^{-2 pi i k.z}: the HIP path is
the adjoint NFFT at x with the product by bhat fused into its last FFT pass, then the NFFT
at y; the oracle writes the same sums out through the direct sums.  Tolerances as for the
transforms: 1e-12 (complex128, m = 8), 5e-6 (complex64).
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, host, parity_err
from oracle import oracle as O
from paper_1810_09891_amd import Plan, fastsum, gaussian_coefficients, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def _case(N, Mx, My, seed):
    r = np.random.default_rng(seed)
    d = len(N)
    return {"x": r.random((Mx, d)) - 0.5, "y": r.random((My, d)) - 0.5, "bhat": W.cgauss(r, N),
            "alpha": W.cgauss(r, (Mx,))}


@pytest.mark.parametrize("N,Mx,My", [((128,), 700, 500), ((32, 48), 1500, 900), ((16, 16, 12), 800, 600)],
                         ids=["d1", "d2", "d3"])
@pytest.mark.parametrize("dtype,m", [(C128, 8), (C64, 6)], ids=["c128m8", "c64m6"])
def test_fastsum_two_node_sets(N, Mx, My, dtype, m):
    announce("fastsum", N, Mx, My, dtype, m)
    c = _case(N, Mx, My, 200 + len(N))
    px = Plan(N, Mx, m=m, dtype=dtype).set_nodes(dev(c["x"], torch.float64))
    py = Plan(N, My, m=m, dtype=dtype).set_nodes(dev(c["y"], torch.float64))
    g = host(fastsum(px, py, dev(c["bhat"], dtype), dev(c["alpha"], dtype)))
    ref = O.fastsum(c["x"], c["y"], c["bhat"], c["alpha"])
    assert parity_err(ref, g) < TOL[dtype]


@pytest.mark.parametrize("dtype,m", [(C128, 8), (C64, 6)], ids=["c128m8", "c64m6"])
def test_fastsum_same_nodes(dtype, m):
    """y = x through one plan (the adjoint's grid is then reused by the forward step)."""
    announce("fastsum same nodes", dtype, m)
    N = (48, 32)
    c = _case(N, 1200, 1, 220)
    p = Plan(N, 1200, m=m, dtype=dtype).set_nodes(dev(c["x"], torch.float64))
    g = host(fastsum(p, p, dev(c["bhat"], dtype), dev(c["alpha"], dtype)))
    ref = O.fastsum(c["x"], c["x"], c["bhat"], c["alpha"])
    assert parity_err(ref, g) < TOL[dtype]
    # a plain transform afterwards still works on the same plan
    f = host(p.trafo(dev(c["bhat"], dtype)))
    assert parity_err(O.ndft_trafo(c["x"], c["bhat"]), f) < (1e-12 if dtype == C128 else 5e-6)


def test_fastsum_gaussian_kernel():
    """Gaussian kernel exp(-|z|^2/c^2), c = 0.08, N = 64^2 (omitted coefficients < 1e-28):
    the GPU sums equal sums of Gaussians over the nearest periodic images."""
    announce("fastsum gaussian")
    r = np.random.default_rng(230)
    N, cw = (64, 64), 0.08
    x = r.random((3000, 2)) - 0.5
    y = r.random((2000, 2)) - 0.5
    alpha = W.cgauss(r, (3000,))
    px = Plan(N, 3000, m=8, dtype=C128).set_nodes(dev(x, torch.float64))
    py = Plan(N, 2000, m=8, dtype=C128).set_nodes(dev(y, torch.float64))
    g = host(fastsum(px, py, gaussian_coefficients(N, cw), dev(alpha, C128)))
    sel = np.arange(0, 2000, 10)
    ref = np.zeros(len(sel), dtype=np.complex128)
    for m0 in (-1, 0, 1):
        for m1 in (-1, 0, 1):
            z = y[sel, None, :] - x[None, :, :] + np.array([m0, m1])
            ref += np.exp(-np.sum(z * z, -1) / (cw * cw)) @ alpha
    assert parity_err(ref, g[sel]) < 1e-11


def test_fastsum_rejects_mismatched_plans():
    px = Plan((16, 16), 10, m=4, dtype=C64).set_nodes(torch.zeros(10, 2, device="cuda", dtype=torch.float64))
    py = Plan((16, 32), 10, m=4, dtype=C64).set_nodes(torch.zeros(10, 2, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        fastsum(px, py, torch.zeros(16, 16, device="cuda", dtype=C64), torch.zeros(10, device="cuda", dtype=C64))
    lib = px._lib
    w = torch.zeros(16, 16, device="cuda", dtype=C64)
    a = torch.zeros(10, device="cuda", dtype=C64)
    st = lib.nfft_fastsum(px._h, py._h, ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                          ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(w.data_ptr()), None)
    assert st == -1  # NFFT_ERR_ARG, nothing enqueued
