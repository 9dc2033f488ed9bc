"""Window factors from lookup tables (NFFT_PRE_LIN_PSI, Sec. 3.1 Table 3.2) through the C ABI.

With the flag, nfft_set_nodes and nfft_grad_x take the window and its derivative from
tables of 4097 samples per stencil point in the offset delta, linearly interpolated.  Linear
interpolation with step h = 1/4096 has error at most h^2/8 max|d^2 phi/d delta^2| per factor
(the standard bound); the window's second derivative in delta is at most about b^2 times its
peak (b the window shape), so each factor carries a relative error below h^2 b^2 / 8 and a
d-fold product below d times that.  The bars below are that bound times 4 (for the sums over
the stencil and the FFT), checked against the FP64 oracle; in complex128 the result must
also differ from the closed-form plan by more than rounding (the tables are in use).
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, dev, host, parity_err, rel_l2
from oracle import oracle as O
from paper_1810_09891_amd import NFFT_KEEP_GRID, NFFT_PRE_LIN_PSI, Plan, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
H = 1.0 / 4096


def _bar(d, N, n, m, window):
    """4 d times the per-factor bound h^2/8 max|phi''| / max|phi| with max|phi''| / max|phi| at
    most b^2 (Kaiser-Bessel, b = pi (2 - 1/sigma)) or 4 m^2 / b_G^2 + 2 / b_G (Gaussian,
    b_G = 2 sigma m / ((2 sigma - 1) pi)).  (The measured interpolation error of the factors
    is about 5e-9 of their peak, 30 times below the bound.)"""
    sigma = min(nt / Nt for nt, Nt in zip(n, N))
    if window == "gaussian":
        bg = 2 * sigma * m / ((2 * sigma - 1) * np.pi)
        c2 = 4 * m * m / bg ** 2 + 2 / bg
    else:
        c2 = (np.pi * (2 - 1 / sigma)) ** 2
    return 4 * d * H * H * c2 / 8


@pytest.mark.parametrize("window", ["kaiser-bessel", "gaussian"])
@pytest.mark.parametrize("d,N,M,m", [(1, (256,), 1500, 8), (2, (64, 48), 3000, 6), (3, (16, 20, 12), 2000, 4)])
def test_tables_within_interpolation_bound(window, d, N, M, m):
    announce("lin psi", window, d, N, M, m)
    c = W.small_case(d, N, M, seed=700 + d + m)
    p = Plan(N, M, m=m, dtype=C128, flags=NFFT_PRE_LIN_PSI, window=window)
    n = tuple(int(v) for v in p.n)
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], C128)))
    h = host(p.adjoint(dev(c["f"], C128)))
    ref_f = O.nfft_trafo(c["x"], c["fhat"], n, m) if window == "kaiser-bessel" else None
    q = Plan(N, M, m=m, dtype=C128, window=window)
    q.set_nodes(dev(c["x"], torch.float64))
    f0 = host(q.trafo(dev(c["fhat"], C128)))
    h0 = host(q.adjoint(dev(c["f"], C128)))
    bar = _bar(d, N, n, m, window)
    assert parity_err(f0, f) < bar and parity_err(h0, h) < bar, (parity_err(f0, f), parity_err(h0, h), bar)
    assert rel_l2(f0, f) > 1e-13  # the tables are in use
    if ref_f is not None:
        assert parity_err(ref_f, f) < bar + 1e-12
    # complex64 with the tables stays within the complex64 bar
    r = Plan(N, M, m=m, dtype=C64, flags=NFFT_PRE_LIN_PSI, window=window)
    r.set_nodes(dev(c["x"], torch.float64))
    f32 = host(r.trafo(dev(c["fhat"], C64)))
    assert parity_err(f0, f32) < 5e-6


@pytest.mark.parametrize("d,N,M,m", [(1, (64,), 300, 6), (2, (32, 16), 700, 5)])
def test_gradient_from_tables(d, N, M, m):
    """nfft_grad_x with the derivative table against the oracle's derivative of the
    interpolation step."""
    announce("lin psi grad", d, N, M, m)
    n = tuple(2 * v for v in N)
    c = W.small_case(d, N, M, seed=720 + d)
    p = Plan(N, M, n=n, m=m, dtype=C128, flags=NFFT_KEEP_GRID | NFFT_PRE_LIN_PSI)
    p.set_nodes(dev(c["x"], torch.float64))
    p.trafo(dev(c["fhat"], C128))
    g = p.grad_x(dev(c["f"], C128))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], n, m), N, m)
    ref = np.real(np.conj(c["f"])[:, None] * dfdx)
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    # the derivative table's error: h^2/8 max|phi'''| relative to max|phi'|, about b^2 h^2 / 8
    assert 1e-13 < err < 4 * d * H * H * (np.pi * 1.5) ** 2 / 8 * 4, err
