"""Transforms under conditions the parity sweep does not reach: a side stream, node sets
replaced on a live plan, the smallest and largest plans the library accepts, non-finite
coordinates and coordinates far outside the unit torus.

Tolerances as for the other parity tests: 1e-12 (complex128), 5e-6 (complex64) against
the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, host, parity_err, rel_l2
from oracle import oracle as O
from paper_1810_09891_amd import NFFT_KEEP_GRID, Batch, Plan, workloads as W
from paper_1810_09891_amd._lib import NfftError

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def _check(p, c, N, n, m, dtype):
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    assert parity_err(O.nfft_trafo(c["x"], c["fhat"], n, m), f) < TOL[dtype]
    assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, n, m), h) < TOL[dtype]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_side_stream(dtype):
    """Every call enqueued on a non-default stream (plan, nodes, transforms, batch)."""
    announce("side stream", dtype)
    N, M, m = (64, 48), 3000, 6
    c = W.small_case(2, N, M, seed=600)
    xs, fh, fv = dev(c["x"], torch.float64), dev(c["fhat"], dtype), dev(c["f"], dtype)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        p = Plan(N, M, m=m, dtype=dtype).set_nodes(xs)
        f = p.trafo(fh)
        h = p.adjoint(fv)
        b = Batch([p])
        fb, = b.trafo([fh])
        hb, = b.adjoint([fv])
    side.synchronize()
    f, h, fb, hb = host(f), host(h), host(fb), host(hb)
    assert parity_err(O.nfft_trafo(c["x"], c["fhat"], p.n, m), f) < TOL[dtype]
    assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, p.n, m), h) < TOL[dtype]
    assert parity_err(f, fb) < TOL[dtype]
    assert parity_err(h, hb) < TOL[dtype]


def test_nodes_replaced_on_live_plan():
    """Three node sets in turn on one plan (uniform, clustered, wide): each transform
    matches the oracle for the nodes set last, and a kept grid is dropped by set_nodes."""
    announce("replace nodes")
    N, M, m = (48, 64), 2500, 6
    p = Plan(N, M, m=m, dtype=C128, flags=NFFT_KEEP_GRID)
    for i, kind in enumerate(("uniform", "clustered", "wide")):
        c = W.small_case(2, N, M, seed=610 + i, kind=kind)
        p.set_nodes(dev(c["x"], torch.float64))
        with pytest.raises(NfftError):
            p.grad_x(dev(c["f"], C128))  # the grid kept from the previous nodes is gone
        _check(p, c, N, p.n, m, C128)


@pytest.mark.parametrize("N,n,m,M", [((2,), (4,), 1, 1), ((2,), (4,), 1, 5), ((2, 2), (4, 4), 1, 1),
                                     ((2, 4), (4, 8), 1, 7), ((2, 2, 2), (4, 4, 4), 1, 3)],
                         ids=["d1M1", "d1M5", "d2M1", "d2M7", "d3M3"])
@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_smallest_plans(N, n, m, M, dtype):
    """N = 2 per axis on a 4-point grid with the 4-point stencil (m = 1): every tile wraps
    around the grid, every FFT line is a single radix-4 stage."""
    announce("smallest", N, n, m, M, dtype)
    c = W.small_case(len(N), N, M, seed=620 + M)
    p = Plan(N, M, n=n, m=m, dtype=dtype).set_nodes(dev(c["x"], torch.float64))
    _check(p, c, N, n, m, dtype)


@pytest.mark.parametrize("N,n,m,M,dtype", [((2048,), (4096,), 12, 3000, C128),
                                           ((2048,), (4096,), 12, 3000, C64),
                                           ((2048, 8), (4096, 32), 12, 2000, C64),
                                           ((8, 2048), (32, 4096), 12, 2000, C128),
                                           ((16, 16, 16), (32, 32, 32), 8, 700, C128)],
                         ids=["d1c128", "d1c64", "d2col4096", "d2row4096", "d3onetile"])
def test_largest_plans(N, n, m, M, dtype):
    """FFT lines of 4096 points (the longest held in one workgroup) with the widest
    stencil (m = 12), and a 3-D complex128 plan whose single spreading tile fills most of
    the LDS."""
    announce("largest", N, n, m, M, dtype)
    c = W.small_case(len(N), N, M, seed=630 + len(N))
    p = Plan(N, M, n=n, m=m, dtype=dtype).set_nodes(dev(c["x"], torch.float64))
    _check(p, c, N, n, m, dtype)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_nonfinite_nodes(dtype):
    """NaN and infinite coordinates are reported by nodes_finite and give NaN at those
    nodes only in the forward transform and the gradient (the other nodes keep their
    values) and NaN throughout the adjoint; finite nodes set afterwards give clean results
    in both directions."""
    announce("non-finite nodes", dtype)
    N, M, m = (32, 32), 1500, 6
    n = (64, 64)
    c = W.small_case(2, N, M, seed=640)
    bad = np.array([5, 77, 1000])
    x = c["x"].copy()
    x[bad[0], 0] = np.nan
    x[bad[1], 1] = np.inf
    x[bad[2], :] = -np.inf
    p = Plan(N, M, n=n, m=m, dtype=dtype, flags=NFFT_KEEP_GRID).set_nodes(dev(x, torch.float64))
    assert not p.nodes_finite()
    f = host(p.trafo(dev(c["fhat"], dtype)))
    assert np.isnan(f[bad]).all()
    good = np.setdiff1d(np.arange(M), bad)
    assert np.isfinite(f[good]).all()
    assert parity_err(O.nfft_trafo(c["x"][good], c["fhat"], n, m), f[good]) < TOL[dtype]
    gx = p.grad_x(dev(c["f"], dtype)).cpu().numpy()
    assert np.isnan(gx[bad]).all()
    assert np.isfinite(gx[good]).all()
    h = host(p.adjoint(dev(c["f"], dtype)))
    assert np.isnan(h).all()
    p.set_nodes(dev(c["x"], torch.float64))
    assert p.nodes_finite()
    _check(p, c, N, n, m, dtype)


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
def test_far_periodic_images(dtype):
    """Coordinates shifted by large integers (up to 2^40) give exactly the results of the
    shifted-back coordinates: n x is exact for power-of-two n, so the grid index and the
    offset do not change."""
    announce("far images", dtype)
    N, M, m = (32, 64), 2000, 6
    c = W.small_case(2, N, M, seed=650)
    shifts = np.random.default_rng(651).choice([-(2.0 ** 40), -12345.0, 3.0, 7e6, 2.0 ** 33], size=(M, 2))
    x_far = c["x"] + shifts
    x_back = x_far - shifts  # exact: the rounding happened in the addition
    p = Plan(N, M, m=m, dtype=dtype)
    p.set_nodes(dev(x_far, torch.float64))
    f_far = host(p.trafo(dev(c["fhat"], dtype)))
    h_far = host(p.adjoint(dev(c["f"], dtype)))
    p.set_nodes(dev(x_back, torch.float64))
    f_back = host(p.trafo(dev(c["fhat"], dtype)))
    h_back = host(p.adjoint(dev(c["f"], dtype)))
    assert np.array_equal(f_far, f_back)
    assert parity_err(h_back, h_far) < TOL[dtype]
    assert parity_err(O.nfft_trafo(x_back, c["fhat"], p.n, m), f_back) < TOL[dtype]


@pytest.mark.parametrize("n", [(1024, 1024, 1024), (1008, 1008, 1008)], ids=["pow2", "mixed"])
def test_grid_beyond_2_28_cells(n):
    """A 3-D grid of about 2^30 cells (8 GB in complex64): 64-bit grid indices in the window
    kernels, the fold and the FFT passes, and the interpolation's loading waves on their
    64-bit path (which keeps half as many tile entries in registers).  Checked against the
    direct sums on 500 nodes (sigma = 16 or 15.75, m = 4: the window error is far below the
    complex64 bar)."""
    N, M, m = (64, 64, 64), 500, 4
    announce("large grid", n)
    c = W.small_case(3, N, M, seed=900)
    p = Plan(N, M, n=n, m=m, dtype=torch.complex64)
    assert p.n[0] * p.n[1] * p.n[2] >= 1 << 29
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], torch.complex64)))
    h = host(p.adjoint(dev(c["f"], torch.complex64)))
    assert rel_l2(O.ndft_trafo(c["x"], c["fhat"]), f) < 5e-6
    assert rel_l2(O.ndft_adjoint(c["x"], c["f"], N), h) < 5e-6
    p.close()
    torch.cuda.empty_cache()
