"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative l2 against the oracle): 1e-12 for complex128 plans, 5e-6 for
complex64 plans.  Small cases span several bins, tiles and FFT line groups with ragged
node counts; the full-size workloads are checked on sampled outputs (forward) and on
all or sampled coefficients (adjoint).
"""
import numpy as np
import pytest
import torch

from error_scale import adjoint_errors
from gpu_util import TOL, announce, dev, host, parity_err
from oracle import oracle as O
from paper_1810_09891_amd import Plan, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64

SMALL = [
    # d, N, M, kind
    (1, (512,), 2001, "uniform"),
    (2, (64, 48), 3001, "uniform"),
    (2, (32, 64), 2500, "clustered"),
    (3, (16, 12, 20), 2003, "uniform"),
    (3, (16, 16, 16), 1500, "wide"),
]


def make_plan(N, M, m, dtype, n=None, flags=0):
    return Plan(N, M, n=n, m=m, dtype=dtype, flags=flags)


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "d%d_%s_%d_%s" % (c[0], "x".join(map(str, c[1])), c[2], c[3]))
@pytest.mark.parametrize("dtype,m", [(C128, 2), (C128, 5), (C128, 8), (C64, 4), (C64, 8)],
                         ids=["c128m2", "c128m5", "c128m8", "c64m4", "c64m8"])
def test_trafo_adjoint_small(case, dtype, m):
    d, N, M, kind = case
    n = tuple(2 * v if (2 * v) & (2 * v - 1) == 0 else 1 << int(np.ceil(np.log2(v)) + 1) for v in N)
    if 2 * m + 2 > min(n):
        pytest.skip("stencil wider than the grid")
    c = W.small_case(d, N, M, seed=d * 10 + m, kind=kind)
    announce("trafo/adjoint small", d, N, M, kind, dtype, m)
    p = make_plan(N, M, m, dtype, n=n)
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    f_ref = O.nfft_trafo(c["x"], c["fhat"], n, m)
    h_ref = O.nfft_adjoint(c["x"], c["f"], N, n, m)
    assert parity_err(f_ref, f) < TOL[dtype]
    assert parity_err(h_ref, h) < TOL[dtype]


@pytest.mark.parametrize("d,N,M", [(1, (256,), 1024), (2, (32, 32), 700), (3, (16, 16, 16), 500)])
def test_against_direct_sums_m8(d, N, M):
    """With m = 8 the NFFT reaches the direct sums eq. (1.2)/(1.3) (window error ~1e-14)."""
    c = W.small_case(d, N, M, seed=77 + d)
    announce("vs ndft", d, N, M)
    p = make_plan(N, M, 8, C128)
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], C128)))
    h = host(p.adjoint(dev(c["f"], C128)))
    assert parity_err(O.ndft_trafo(c["x"], c["fhat"]), f) < 1e-12
    assert parity_err(O.ndft_adjoint(c["x"], c["f"], N), h) < 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("d,N,M", [(1, (128,), 999), (2, (24, 40), 1777), (3, (12, 8, 16), 1234)])
def test_device_ndft(dtype, d, N, M):
    c = W.small_case(d, N, M, seed=5 + d)
    announce("device ndft", d, N, M, dtype)
    p = make_plan(N, M, 4, dtype)
    p.set_nodes(dev(c["x"], torch.float64))
    f = host(p.ndft_trafo(dev(c["fhat"], dtype)))
    h = host(p.ndft_adjoint(dev(c["f"], dtype)))
    tol = 1e-13 if dtype == C128 else 2e-6
    assert parity_err(O.ndft_trafo(c["x"], c["fhat"]), f) < tol
    assert parity_err(O.ndft_adjoint(c["x"], c["f"], N), h) < tol


@pytest.mark.parametrize("dtype,m", [(C128, 3), (C128, 6), (C64, 6)])
@pytest.mark.parametrize("d,N,M", [(1, (512,), 1500), (2, (64, 32), 2222), (3, (16, 8, 16), 999)])
def test_single_steps(dtype, m, d, N, M):
    """Each step of Algorithm 2.1 / 2.2 against the oracle's step on identical inputs."""
    n = tuple(2 * v for v in N)
    c = W.small_case(d, N, M, seed=300 + m + d)
    announce("steps", d, N, M, dtype, m)
    p = make_plan(N, M, m, dtype, n=n)
    p.set_nodes(dev(c["x"], torch.float64))
    tol = TOL[dtype]
    # the step grids carry S = prod_t e^{b_t m}, b_t = pi (2 - N_t / n_t)
    S = float(np.prod([np.exp(np.pi * (2.0 - Nt / nt) * m) for Nt, nt in zip(N, n)]))
    assert abs(p.info.grid_scale / S - 1.0) < 1e-13
    # D + F
    g_ref = O.nfft_grid(c["fhat"], n, m)
    g = host(p.step_grid(dev(c["fhat"], dtype)))
    assert parity_err(g_ref * S, g) < tol
    # B on the oracle's grid
    f = host(p.step_interp(dev(g_ref * S, dtype)))
    assert parity_err(O.nfft_interp(c["x"], g_ref, N, m), f) < tol
    # B^T
    gs_ref = O.nfft_spread(c["x"], c["f"], N, n, m)
    gs = host(p.step_spread(dev(c["f"], dtype)))
    assert parity_err(gs_ref / S, gs) < tol
    # F^H + D^H on the oracle's spread grid
    h = host(p.step_coeffs(dev(gs_ref / S, dtype)))
    assert parity_err(O.nfft_adjoint_from_grid(gs_ref, N, m), h) < tol


OWNER = [
    # N, M, kind: grids n = (64, 64, 128) / 32^3 / 64^3, nodes uniform, clustered (dense
    # tiles split over several work items), outside [-1/2, 1/2), and a tiny grid where a
    # tile's neighbourhood covers every bin of a dimension
    ((32, 24, 40), 20000, "uniform"),
    ((32, 24, 40), 30000, "clustered"),
    ((16, 16, 16), 6000, "wide"),
    ((32, 32, 32), 50000, "clustered"),
]


def _owner_expected(n, m, dtype):
    T = (16, 16, 16)
    return all(nt % Tt == 0 and nt >= Tt + 2 * m + 1 for nt, Tt in zip(n, T))


@pytest.mark.parametrize("case", OWNER, ids=lambda c: "%s_%d_%s" % ("x".join(map(str, c[0])), c[1], c[2]))
@pytest.mark.parametrize("dtype,m", [(C64, 6), (C128, 6), (C64, 4), (C128, 8), (C64, 8), (C128, 2)],
                         ids=["c64m6", "c128m6", "c64m4", "c128m8", "c64m8", "c128m2"])
def test_spread_by_output_tiles_3d(case, dtype, m):
    """3-D spreading by output tiles (every grid cell written once by its owner, split tiles
    folded in item order): the spread grid and the adjoint against the oracle, bitwise
    repeatable."""
    N, M, kind = case
    if dtype == C64 and kind == "clustered":
        # complex64 sums in FP32: the rounding error grows with the number of nodes that
        # reach one cell (here tens of thousands within a few cells)
        M = min(M, 30000 if m <= 6 else 15000)
    c = W.small_case(3, N, M, seed=500 + M % 97 + m, kind=kind)
    announce("owner tiles", N, M, kind, dtype, m)
    p = make_plan(N, M, m, dtype)
    n = p.n
    assert (p.info.own_tiles > 0) == _owner_expected(n, m, dtype)
    p.set_nodes(dev(c["x"], torch.float64))
    S = float(np.prod([np.exp(np.pi * (2.0 - Nt / nt) * m) for Nt, nt in zip(N, n)]))
    gs = host(p.step_spread(dev(c["f"], dtype)))
    assert parity_err(O.nfft_spread(c["x"], c["f"], N, n, m) / S, gs) < TOL[dtype]
    fv = dev(c["f"], dtype)
    h1 = host(p.adjoint(fv))
    h2 = host(p.adjoint(fv))
    assert np.array_equal(h1, h2)
    ref = O.nfft_adjoint(c["x"], c["f"], N, n, m)
    if dtype == C128:
        assert parity_err(ref, h1) < TOL[dtype]
    else:
        # the deconvolution weights w_k = 1 / (n phi_hat(k)) of a 3-D grid at n = 2N span
        # up to 750x (m = 8) between the centre and the corners of I_N, so the plain relative
        # error of complex64 results is set by the FP32 rounding of a few corner frequencies
        # and changes several-fold with the summation order; the relative error of
        # y = F^H B^T f and its element-wise form (error_scale) are the measures in which the
        # last step is well-conditioned
        e2, emax = adjoint_errors(c["x"], c["f"], N, n, m, h1, ref=ref)
        assert e2 < TOL[dtype] and emax < 2e-5, (e2, emax)


@pytest.mark.parametrize("dtype,m", [(C128, 8), (C64, 10)], ids=["c128m8", "c64m10"])
def test_spread_by_output_tiles_widest_stencils(dtype, m):
    """The output-tile spreading at the widest stencils a 3-D plan accepts (2m + 2 = 18
    points per dimension in complex128, 22 in complex64: the largest factor records in
    LDS), uniform and clustered nodes, against the oracle: the spread grid, the adjoint and
    the forward transform."""
    N, n = (32, 24, 32), (64, 48, 64)
    for kind, M in (("uniform", 2500), ("clustered", 2500)):
        announce("owner tiles wide", N, M, kind, dtype, m)
        c = W.small_case(3, N, M, seed=560 + m, kind=kind)
        p = make_plan(N, M, m, dtype, n=n)
        assert p.info.own_tiles > 0
        p.set_nodes(dev(c["x"], torch.float64))
        S = float(np.prod([np.exp(np.pi * (2.0 - Nt / nt) * m) for Nt, nt in zip(N, n)]))
        gs = host(p.step_spread(dev(c["f"], dtype)))
        assert parity_err(O.nfft_spread(c["x"], c["f"], N, n, m) / S, gs) < TOL[dtype]
        h = host(p.adjoint(dev(c["f"], dtype)))
        ref = O.nfft_adjoint(c["x"], c["f"], N, n, m)
        if dtype == C128:
            assert parity_err(ref, h) < TOL[dtype]
        else:
            e2, emax = adjoint_errors(c["x"], c["f"], N, n, m, h, ref=ref)
            assert e2 < TOL[dtype] and emax < 2e-5, (e2, emax)
        f = host(p.trafo(dev(c["fhat"], dtype)))
        assert parity_err(O.nfft_trafo(c["x"], c["fhat"], n, m), f) < TOL[dtype]


def test_edge_nodes_and_tiny_grids():
    """Nodes on the torus edges and outside [-1/2,1/2); grids where the padded tile wraps
    around the grid more than once (n = 16 with m = 6); a single node."""
    announce("edge nodes")
    cases = [
        ((8, 8), 40, 6, (16, 16)),
        ((4,), 1, 1, (8,)),
        ((6, 4, 8), 33, 2, (8, 8, 16)),
    ]
    for N, M, m, n in cases:
        c = W.small_case(len(N), N, M, seed=9)
        x = c["x"].copy()
        x[0, :] = -0.5
        if M > 2:
            x[1, :] = 0.5 - 2.0 ** -52
            x[2, :] = x[2, :] + 2.0
        for dtype in (C128, C64):
            p = make_plan(N, M, m, dtype, n=n)
            p.set_nodes(dev(x, torch.float64))
            f = host(p.trafo(dev(c["fhat"], dtype)))
            h = host(p.adjoint(dev(c["f"], dtype)))
            assert parity_err(O.nfft_trafo(x, c["fhat"], n, m), f) < TOL[dtype], (N, dtype)
            assert parity_err(O.nfft_adjoint(x, c["f"], N, n, m), h) < TOL[dtype], (N, dtype)


def test_adjoint_identity_gpu():
    """<A fhat, f> = <fhat, A^H f> for the HIP transforms (complex128)."""
    N, M = (64, 64), 5000
    c = W.small_case(2, N, M, seed=12)
    announce("adjoint identity")
    p = make_plan(N, M, 6, C128)
    p.set_nodes(dev(c["x"], torch.float64))
    Af = host(p.trafo(dev(c["fhat"], C128)))
    Ah = host(p.adjoint(dev(c["f"], C128)))
    lhs = np.vdot(c["f"], Af)
    rhs = np.vdot(Ah, c["fhat"])
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


@pytest.mark.parametrize("d,N,M", [(2, (128, 128), 20000), (3, (32, 32, 32), 30000)], ids=["d2", "d3"])
@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_repeatable_results(d, N, M, dtype):
    """Bitwise run-to-run repeatability of the forward and the adjoint transform, also when
    the node precomputation runs again: clustered nodes, so that bins hold many more nodes
    than a work item (their split into work items must not depend on the order in which
    the bin counters were incremented)."""
    c = W.small_case(d, N, M, seed=13, kind="clustered")
    announce("repeatability", d, N, M, dtype)
    p = make_plan(N, M, 6, dtype)
    assert p.info.chunk_cap * 4 < M  # several work items per dense bin
    fh = dev(c["fhat"], dtype)
    fv = dev(c["f"], dtype)
    x = dev(c["x"], torch.float64)
    res = []
    for _ in range(2):
        p.set_nodes(x)
        res.append((host(p.trafo(fh)), host(p.adjoint(fv)), host(p.adjoint(fv))))
    (a1, h1, h1b), (a2, h2, h2b) = res
    assert np.array_equal(a1, a2)
    assert np.array_equal(h1, h1b)
    assert np.array_equal(h1, h2)
    assert np.array_equal(h2, h2b)
    assert parity_err(O.nfft_adjoint(c["x"], c["f"], N, p.n, 6), h1) < TOL[dtype]


# ----------------------------------------------------------------------------- full sizes


def _sample(M, count, seed):
    return np.sort(np.random.default_rng(seed).choice(M, size=count, replace=False))


@pytest.mark.parametrize("dtype,m", [(C128, 8), (C128, 4), (C64, 8), (C64, 4)],
                         ids=["c128m8", "c128m4", "c64m8", "c64m4"])
def test_full_d2_512(dtype, m):
    """d=2, N=(512,512), M=262144 uniform nodes: forward on 2048 sampled nodes against the
    oracle NFFT, adjoint on every coefficient against the oracle adjoint NFFT."""
    w = W.workload("d2", m=m)
    announce("full d2", dtype, m)
    p = make_plan(w["N"], w["M"], m, dtype)
    p.set_nodes(dev(w["x"], torch.float64))
    f = host(p.trafo(dev(w["fhat"], dtype)))
    h = host(p.adjoint(dev(w["f"], dtype)))
    sel = _sample(w["M"], 2048, 1)
    f_ref = O.nfft_trafo(w["x"][sel], w["fhat"], w["n"], m)
    assert parity_err(f_ref, f[sel]) < TOL[dtype]
    h_ref = O.nfft_adjoint(w["x"], w["f"], w["N"], w["n"], m)
    assert parity_err(h_ref, h) < TOL[dtype]
    if m == 8:
        # against the direct sums on the sampled nodes / coefficients
        assert parity_err(O.ndft_trafo(w["x"][sel], w["fhat"]), f[sel]) < TOL[dtype]
        ks = _sample(int(np.prod(w["N"])), 64, 2)
        hk = O.ndft_adjoint_at(w["x"], w["f"], w["N"], ks)
        assert parity_err(hk, h.reshape(-1)[ks]) < TOL[dtype]


def test_full_d1_256():
    w = W.workload("d1")
    announce("full d1")
    p = make_plan(w["N"], w["M"], 8, C128)
    p.set_nodes(dev(w["x"], torch.float64))
    f = host(p.trafo(dev(w["fhat"], C128)))
    h = host(p.adjoint(dev(w["f"], C128)))
    assert parity_err(O.ndft_trafo(w["x"], w["fhat"]), f) < 1e-12
    assert parity_err(O.ndft_adjoint(w["x"], w["f"], w["N"]), h) < 1e-12


_D3R_ADJ = {}


def _d3r_adjoint_ref(w):
    """Oracle adjoint NFFT (Algorithm 2.2 in FP64) of the whole 3-D radial workload, computed
    once per session (about half a minute on 16 host threads)."""
    if "h" not in _D3R_ADJ:
        _D3R_ADJ["h"] = O.nfft_adjoint(w["x"], w["f"], w["N"], w["n"], 6)
    return _D3R_ADJ["h"]


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_full_d3_radial(dtype):
    """d=3, N=128^3, 2,097,152 nodes on 4096 radial spokes, m=6: forward on 16384 sampled
    nodes against the oracle NFFT, adjoint on every coefficient against the oracle adjoint
    NFFT; complex64 also against the direct sums on 48 sampled coefficients."""
    w = W.workload("d3r")
    announce("full d3 radial", dtype)
    p = make_plan(w["N"], w["M"], 6, dtype)
    p.set_nodes(dev(w["x"], torch.float64))
    f = host(p.trafo(dev(w["fhat"], dtype)))
    h = host(p.adjoint(dev(w["f"], dtype)))
    del p
    torch.cuda.empty_cache()
    sel = _sample(w["M"], 16384, 3)
    f_ref = O.nfft_trafo(w["x"][sel], w["fhat"], w["n"], 6)
    assert parity_err(f_ref, f[sel]) < TOL[dtype]
    assert parity_err(_d3r_adjoint_ref(w), h) < TOL[dtype]
    if dtype == C64:
        ks = _sample(int(np.prod(w["N"])), 48, 4)
        hk = O.ndft_adjoint_at(w["x"], w["f"], w["N"], ks)
        assert parity_err(hk, h.reshape(-1)[ks]) < TOL[C64]
