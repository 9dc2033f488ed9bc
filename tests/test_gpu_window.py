"""Gaussian, B-spline and sinc window plans (NFFT_WINDOW_GAUSSIAN, _BSPLINE, _SINC) against the
FP64 oracle with the same window.

Tolerances as for the Kaiser-Bessel plans: 1e-12 in complex128, 5e-6 in complex64 (the
window's own error against the direct sums is larger -- the oracle pins it to the
literature bound -- but both sides evaluate the same approximation).
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, host, parity_err
from oracle import oracle as O
from paper_1810_09891_amd import NFFT_KEEP_GRID, Batch, Plan, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64

CASES = [(1, (256,), 1500, "uniform"), (2, (48, 64), 2500, "clustered"), (3, (16, 12, 16), 1200, "wide")]


@pytest.mark.parametrize("case", CASES, ids=["d1", "d2", "d3"])
@pytest.mark.parametrize("dtype,m", [(C128, 8), (C128, 4), (C64, 6)], ids=["c128m8", "c128m4", "c64m6"])
def test_gaussian_trafo_adjoint(case, dtype, m):
    d, N, M, kind = case
    announce("gaussian window", d, N, M, kind, dtype, m)
    c = W.small_case(d, N, M, seed=400 + d * 10 + m, kind=kind)
    p = Plan(N, M, m=m, dtype=dtype, window="gaussian")
    assert p.info.window == 1
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    with O.window("gaussian"):
        f_ref = O.nfft_trafo(c["x"], c["fhat"], p.n, m)
        h_ref = O.nfft_adjoint(c["x"], c["f"], N, p.n, m)
    assert parity_err(f_ref, f) < TOL[dtype]
    assert parity_err(h_ref, h) < TOL[dtype]


def test_gaussian_steps_carry_the_window_peak():
    """Single steps exchange grids scaled by S = prod_t (pi b_t)^{-1/2} for this window."""
    announce("gaussian steps")
    N, M, m = (32, 24), 900, 6
    c = W.small_case(2, N, M, seed=450)
    p = Plan(N, M, m=m, dtype=C128, window="gaussian")
    p.set_nodes(dev(c["x"], torch.float64))
    S = 1.0
    for Nt, nt in zip(N, p.n):
        S *= 1.0 / np.sqrt(np.pi * O.gauss_b(Nt, nt, m))
    assert abs(p.info.grid_scale - S) / S < 1e-14
    g = host(p.step_grid(dev(c["fhat"], C128)))
    with O.window("gaussian"):
        g_ref = O.nfft_grid(c["fhat"], p.n, m)
    assert parity_err(S * g_ref, g) < 1e-12


def test_gaussian_grad_x():
    announce("gaussian grad_x")
    N, M, m = (32, 16), 700, 5
    n = (64, 32)
    c = W.small_case(2, N, M, seed=460)
    p = Plan(N, M, n=n, m=m, dtype=C128, flags=NFFT_KEEP_GRID, window="gaussian")
    p.set_nodes(dev(c["x"], torch.float64))
    p.trafo(dev(c["fhat"], C128))
    g = p.grad_x(dev(c["f"], C128)).cpu().numpy()
    with O.window("gaussian"):
        dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], n, m), N, m)
    ref = np.real(np.conj(c["f"])[:, None] * dfdx)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-12


def test_batch_mixes_windows():
    """Kaiser-Bessel and Gaussian plans in one launch group give their per-plan results."""
    announce("batch mixed windows")
    specs = [((64, 32), 2000, "kaiser-bessel"), ((32, 64), 1500, "gaussian"), ((64, 64), 3000, "gaussian")]
    plans, cases = [], []
    for i, (N, M, win) in enumerate(specs):
        c = W.small_case(2, N, M, seed=470 + i)
        p = Plan(N, M, m=6, dtype=C64, window=win)
        p.set_nodes(dev(c["x"], torch.float64))
        plans.append(p)
        cases.append(c)
    b = Batch(plans)
    assert b.info.groups == 1
    fb = [host(f) for f in b.trafo([dev(c["fhat"], C64) for c in cases])]
    hb = [host(h) for h in b.adjoint([dev(c["f"], C64) for c in cases])]
    for p, c, f, h in zip(plans, cases, fb, hb):
        assert parity_err(host(p.trafo(dev(c["fhat"], C64))), f) <= 1e-6
        assert parity_err(host(p.adjoint(dev(c["f"], C64))), h) <= 1e-6


@pytest.mark.parametrize("window", ["bspline", "sinc"])
@pytest.mark.parametrize("case", CASES, ids=["d1", "d2", "d3"])
@pytest.mark.parametrize("dtype,m", [(C128, 8), (C128, 3), (C64, 6)], ids=["c128m8", "c128m3", "c64m6"])
def test_bspline_sinc_trafo_adjoint(window, case, dtype, m):
    d, N, M, kind = case
    announce(window, "window", d, N, M, kind, dtype, m)
    c = W.small_case(d, N, M, seed=480 + d * 10 + m, kind=kind)
    p = Plan(N, M, m=m, dtype=dtype, window=window)
    assert p.info.window == {"bspline": 2, "sinc": 3}[window]
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    with O.window(window):
        f_ref = O.nfft_trafo(c["x"], c["fhat"], p.n, m)
        h_ref = O.nfft_adjoint(c["x"], c["f"], N, p.n, m)
    assert parity_err(f_ref, f) < TOL[dtype]
    assert parity_err(h_ref, h) < TOL[dtype]


@pytest.mark.parametrize("window", ["bspline", "sinc"])
def test_bspline_sinc_grad_x(window):
    announce(window, "grad_x")
    N, M, m = (32, 16), 700, 5
    n = (64, 32)
    c = W.small_case(2, N, M, seed=490)
    p = Plan(N, M, n=n, m=m, dtype=C128, flags=NFFT_KEEP_GRID, window=window)
    p.set_nodes(dev(c["x"], torch.float64))
    p.trafo(dev(c["fhat"], C128))
    g = p.grad_x(dev(c["f"], C128)).cpu().numpy()
    with O.window(window):
        dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], n, m), N, m)
    ref = np.real(np.conj(c["f"])[:, None] * dfdx)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-12


def test_bspline_sinc_reach_direct_sums():
    """Complex128, m = 8, sigma = 2: both windows bring the NFFT within their error level of
    the direct sums (E_inf <= 4 * 3^-16 ||fhat||_1)."""
    announce("bspline/sinc vs ndft")
    N, M = (64, 48), 1500
    c = W.small_case(2, N, M, seed=495)
    for window in ("bspline", "sinc"):
        p = Plan(N, M, m=8, dtype=C128, window=window)
        p.set_nodes(dev(c["x"], torch.float64))
        f = host(p.trafo(dev(c["fhat"], C128)))
        ref = O.ndft_trafo(c["x"], c["fhat"])
        assert np.max(np.abs(f - ref)) / np.sum(np.abs(c["fhat"])) <= 4 * 3.0 ** -16, window
