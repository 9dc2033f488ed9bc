"""Gradients of the differentiable NFFT (through the C ABI) against the FP64 oracle.

* nfft_grad_x against the oracle's derivative of the interpolation step (complex128, 1e-12);
* torch.autograd.gradcheck of nfft(x, fhat) in complex128;
* the loss ||A(x) fhat - y||^2 on 65536 nodes on radial spokes with N(0, 1e-3^2) jitter,
  complex64, m = 6: gradients with respect to fhat and x against the FP64 oracle gradient
  (adjoint NFFT and the closed-form derivative of the direct sum) and against central
  finite differences of the direct-sum loss.
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, dev, host, parity_err
from oracle import oracle as O
from paper_1810_09891_amd import NFFT_KEEP_GRID, Plan, differentiable_plan, nfft, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,N,M,m", [(1, (64,), 300, 6), (2, (32, 16), 700, 5), (3, (8, 16, 16), 400, 4)])
def test_grad_x_kernel_matches_oracle(d, N, M, m):
    """Re(conj(v_j) d f_j/d x_{j,t}) through the window, against the oracle's derivative of
    the interpolation step on the oracle grid."""
    announce("grad_x kernel", d, N, M, m)
    n = tuple(2 * v for v in N)
    c = W.small_case(d, N, M, seed=60 + d)
    p = Plan(N, M, n=n, m=m, dtype=torch.complex128, flags=NFFT_KEEP_GRID)
    p.set_nodes(dev(c["x"], torch.float64))
    p.trafo(dev(c["fhat"], torch.complex128))
    v = c["f"]
    g = p.grad_x(dev(v, torch.complex128))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], n, m), N, m)
    ref = np.real(np.conj(v)[:, None] * dfdx)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-12


def test_gradcheck_complex128():
    announce("gradcheck")
    N, M = (16, 16), 24
    c = W.small_case(2, N, M, seed=70)
    plan = differentiable_plan(N, M, m=8, dtype=torch.complex128)
    x = torch.tensor(c["x"], device="cuda", dtype=torch.float64, requires_grad=True)
    fh = torch.tensor(c["fhat"], device="cuda", dtype=torch.complex128, requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: nfft(a, b, plan), (x, fh), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_keep_grid_required():
    plan = Plan((16, 16), 10, m=4, dtype=torch.complex64)
    with pytest.raises(ValueError):
        nfft(torch.zeros(10, 2, device="cuda", dtype=torch.float64),
             torch.zeros(16, 16, device="cuda", dtype=torch.complex64), plan)


def test_radial_spokes_loss_gradients():
    """Full differentiable workload: d=2, N=(256,256), 256 spokes x 256 points + jitter,
    complex64, m=6; loss = ||A(x) fhat - y||^2 with y = A(x) fhat_star (FP64 oracle)."""
    announce("radial spokes gradients")
    w = W.workload("grad")
    N, M, x = w["N"], w["M"], w["x"]
    r = W.rng("grad", 1)
    fhat_star = W.cgauss(r, N)
    fhat = W.cgauss(r, N)
    y = O.nfft_trafo(x, fhat_star, None, 8)

    plan = differentiable_plan(N, M, m=6, dtype=torch.complex64)
    xt = torch.tensor(x, device="cuda", dtype=torch.float64, requires_grad=True)
    ft = torch.tensor(fhat, device="cuda", dtype=torch.complex64, requires_grad=True)
    yt = torch.tensor(y, device="cuda", dtype=torch.complex64)
    f = nfft(xt, ft, plan)
    loss = torch.sum(torch.abs(f - yt) ** 2)
    loss.backward()
    gx = xt.grad.detach().cpu().numpy()
    gf = ft.grad.detach().cpu().numpy().astype(np.complex128)

    # FP64 oracle gradient: residual of the m=8 NFFT, 2 A^H r for fhat
    res = O.nfft_trafo(x, fhat, None, 8) - y
    gf_ref = 2.0 * O.nfft_adjoint(x, res, N, None, 8)
    assert parity_err(gf_ref, gf) < 1e-5
    # closed-form derivative of the direct sum on sampled nodes
    sel = np.sort(np.random.default_rng(5).choice(M, 256, replace=False))
    gx_ref = O.ndft_grad_x(x[sel], fhat, res[sel])
    assert np.linalg.norm(gx[sel] - gx_ref) / np.linalg.norm(gx_ref) < 1e-5
    # central differences of the direct-sum loss (only node j's term depends on x_j)
    h = 1e-7
    for j in sel[:6]:
        for t in range(2):
            xp = x[j:j + 1].copy()
            xm = x[j:j + 1].copy()
            xp[0, t] += h
            xm[0, t] -= h
            lp = abs(O.ndft_trafo(xp, fhat)[0] - y[j]) ** 2
            lm = abs(O.ndft_trafo(xm, fhat)[0] - y[j]) ** 2
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gx[j, t]) <= 1e-5 * max(1.0, np.abs(gx_ref).max()), (j, t, fd, gx[j, t])


@pytest.mark.parametrize("need_x", [False, True])
def test_plan_reused_before_backward(need_x):
    """One plan runs nfft at nodes x1, then at x2, then both backwards run: each gradient
    must use its own call's nodes (and grid), also when only fhat requires a gradient."""
    announce("plan reused before backward", need_x)
    N, M, m = (16, 12), 90, 8
    plan = differentiable_plan(N, M, m=m, dtype=torch.complex128)
    cases = [W.small_case(2, N, M, seed=80 + i) for i in range(2)]
    xs, fhs, outs = [], [], []
    for c in cases:
        x = torch.tensor(c["x"], device="cuda", dtype=torch.float64, requires_grad=need_x)
        fh = torch.tensor(c["fhat"], device="cuda", dtype=torch.complex128, requires_grad=True)
        xs.append(x)
        fhs.append(fh)
        outs.append(nfft(x, fh, plan))
    for i in (0, 1):
        v = cases[i]["f"]
        outs[i].backward(torch.tensor(v, device="cuda", dtype=torch.complex128))
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        ref = O.nfft_adjoint(c["x"], c["f"], N, plan.n, m)
        assert parity_err(ref, host(fhs[i].grad)) < 1e-12
        if need_x:
            dfdx = O.nfft_interp_dx(c["x"], O.nfft_grid(c["fhat"], plan.n, m), N, m)
            refx = np.real(np.conj(c["f"])[:, None] * dfdx)
            gx = xs[i].grad.cpu().numpy()
            assert np.linalg.norm(gx - refx) / np.linalg.norm(refx) < 1e-12
