"""NNFFT (nonequispaced nodes in both domains, the generalisation named in Sec. 1) against
the oracle's direct sums.

The HIP path spreads the frequencies with one inner plan, runs an NFFT of the frequency
grid at scaled nodes with a second plan and divides by the window's Fourier transform at
each node.  The oracle is the definition itself (oracle.nndft_*), so the comparison
includes the method's approximation error, which is that of the two inner NFFTs.  Bars:
Kaiser-Bessel with m = 8 keeps the transforms' own bars (1e-12 complex128, 5e-6
complex64); for the other windows and smaller m the bar is 20 times the approximation
error of the oracle's own NFFT (Algorithm 2.1, same window, m and grid as the inner NFFT)
against its direct sum, or the transforms' bar when that is larger -- a bound taken from
the oracle alone.
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, e_inf, host, parity_err, rel_l2
from oracle import oracle as O
from paper_1810_09891_amd import NNPlan, Plan, workloads as W
from paper_1810_09891_amd._lib import NfftError

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def _case(N, K, M, seed):
    r = np.random.default_rng(seed)
    d = len(N)
    return {"x": r.random((M, d)) - 0.5,
            "v": (r.random((K, d)) - 0.5) * np.asarray(N, dtype=np.float64),
            "fhat": W.cgauss(r, (K,)), "f": W.cgauss(r, (M,))}


def _bar(p, dtype, window, m):
    if window == "kaiser-bessel" and m == 8:
        return TOL[dtype]
    # the inner NFFT's approximation error, from the oracle: N2 coefficients at nodes in
    # [-1/(2 sigma1), 1/(2 sigma1)), the window and m of the plan
    r = np.random.default_rng(5)
    d = len(p.N2)
    z = (r.random((300, d)) - 0.5) / np.asarray(p.sigma1)
    c = W.cgauss(r, p.N2)
    with O.window(window):
        e = rel_l2(O.ndft_trafo(z, c), O.nfft_trafo(z, c, m=m))
    return max(TOL[dtype], 20.0 * e)


def _run(N, K, M, dtype, m, window="kaiser-bessel", seed=0, sigma=None):
    announce("nnfft", N, K, M, dtype, m, window, sigma)
    c = _case(N, K, M, seed)
    p = NNPlan(N, K, M, sigma=sigma, m=m, dtype=dtype, window=window)
    p.set_nodes(dev(c["x"], torch.float64), dev(c["v"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], dtype)))
    h = host(p.adjoint(dev(c["f"], dtype)))
    # the direct sums differ from the fast transform by its approximation error: E_2 and
    # the E_inf of eq. (2.16) against the bar
    fr = O.nndft_trafo(c["v"], c["x"], c["fhat"])
    hr = O.nndft_adjoint(c["v"], c["x"], c["f"])
    ef = max(rel_l2(fr, f), e_inf(fr, f, c["fhat"]))
    eh = max(rel_l2(hr, h), e_inf(hr, h, c["f"]))
    return p, ef, eh


@pytest.mark.parametrize("N,K,M", [((64,), 611, 733), ((32, 24), 1511, 1303), ((12, 16, 10), 907, 811)],
                         ids=["d1", "d2", "d3"])
@pytest.mark.parametrize("dtype,m", [(C128, 8), (C64, 8), (C64, 4), (C128, 4)],
                         ids=["c128m8", "c64m8", "c64m4", "c128m4"])
def test_nnfft_matches_direct_sums(N, K, M, dtype, m):
    p, ef, eh = _run(N, K, M, dtype, m, seed=11 + len(N))
    bar = _bar(p, dtype, "kaiser-bessel", m)
    assert ef < bar and eh < bar, (ef, eh, bar)


@pytest.mark.parametrize("window", ["gaussian", "bspline", "sinc"])
@pytest.mark.parametrize("dtype,m", [(C128, 8), (C64, 6)], ids=["c128m8", "c64m6"])
def test_nnfft_windows(window, dtype, m):
    p, ef, eh = _run((32, 24), 1201, 1103, dtype, m, window=window, seed=23)
    bar = _bar(p, dtype, window, m)
    assert ef < bar and eh < bar, (ef, eh, bar)


@pytest.mark.parametrize("sigma", [1.5, 3.0])
def test_nnfft_other_frequency_oversampling(sigma):
    # explicit sigma: N2 >= sigma N + 2m + 4 (here sigma1 > 2 in both dimensions)
    p, ef, eh = _run((40, 18), 997, 1009, C128, 8, seed=29, sigma=sigma)
    assert min(p.sigma1) > 2.0
    assert ef < TOL[C128] and eh < TOL[C128], (ef, eh)


def test_nnfft_integer_frequencies_agree_with_the_nfft():
    # v running over I_N makes the NNFFT an NFFT: compare with the plan's own transform
    N = (16, 12)
    announce("nnfft integer frequencies", N)
    r = np.random.default_rng(31)
    M = 700
    x = r.random((M, 2)) - 0.5
    axes = [np.arange(n) - n // 2 for n in N]
    v = np.stack([g.reshape(-1) for g in np.meshgrid(*axes, indexing="ij")], axis=1).astype(np.float64)
    fhat = W.cgauss(r, N)
    f = W.cgauss(r, (M,))
    nn = NNPlan(N, v.shape[0], M, m=8, dtype=C128).set_nodes(dev(x, torch.float64), dev(v, torch.float64))
    pl = Plan(N, M, m=8, dtype=C128).set_nodes(dev(x, torch.float64))
    a = host(nn.trafo(dev(fhat.reshape(-1), C128)))
    b = host(pl.trafo(dev(fhat, C128)))
    assert parity_err(b, a) < 1e-12
    ha = host(nn.adjoint(dev(f, C128)))
    hb = host(pl.adjoint(dev(f, C128))).reshape(-1)
    assert parity_err(hb, ha) < 1e-12


def test_nnfft_edge_cases():
    # one frequency and one node; frequencies at -N/2 and just below N/2; nodes at -1/2
    N = (20, 14)
    announce("nnfft edge cases", N)
    for K, M in [(1, 1), (1, 5), (7, 1)]:
        c = _case(N, K, M, 37 + K + M)
        p = NNPlan(N, K, M, m=8, dtype=C128).set_nodes(dev(c["x"], torch.float64), dev(c["v"], torch.float64))
        f = host(p.trafo(dev(c["fhat"], C128)))
        h = host(p.adjoint(dev(c["f"], C128)))
        assert parity_err(O.nndft_trafo(c["v"], c["x"], c["fhat"]), f) < 1e-12
        assert parity_err(O.nndft_adjoint(c["v"], c["x"], c["f"]), h) < 1e-12
    r = np.random.default_rng(41)
    K, M = 301, 257
    v = (r.random((K, 2)) - 0.5) * np.asarray(N, dtype=np.float64)
    v[:40, 0] = -N[0] / 2
    v[40:80, 1] = -N[1] / 2
    v[80:120, 0] = np.nextafter(N[0] / 2, 0)
    v[120:160, 1] = np.nextafter(N[1] / 2, 0)
    x = r.random((M, 2)) - 0.5
    x[:30, 0] = -0.5
    x[30:60, 1] = -0.5
    fh = W.cgauss(r, (K,))
    fv = W.cgauss(r, (M,))
    p = NNPlan(N, K, M, m=8, dtype=C128).set_nodes(dev(x, torch.float64), dev(v, torch.float64))
    assert parity_err(O.nndft_trafo(v, x, fh), host(p.trafo(dev(fh, C128)))) < 1e-12
    assert parity_err(O.nndft_adjoint(v, x, fv), host(p.adjoint(dev(fv, C128)))) < 1e-12


def test_nnfft_new_nodes_on_the_same_plan():
    N, K, M = (24, 24), 500, 400
    announce("nnfft set_nodes twice", N, K, M)
    p = NNPlan(N, K, M, m=8, dtype=C64)
    for seed in (43, 44):
        c = _case(N, K, M, seed)
        p.set_nodes(dev(c["x"], torch.float64), dev(c["v"], torch.float64))
        f = host(p.trafo(dev(c["fhat"], C64)))
        assert parity_err(O.nndft_trafo(c["v"], c["x"], c["fhat"]), f) < TOL[C64]


def test_nnfft_nonfinite_node_stays_local():
    N, K, M = (16, 16), 200, 150
    announce("nnfft nonfinite node", N, K, M)
    c = _case(N, K, M, 47)
    x = c["x"].copy()
    x[17, 1] = np.nan
    p = NNPlan(N, K, M, m=8, dtype=C128).set_nodes(dev(x, torch.float64), dev(c["v"], torch.float64))
    f = host(p.trafo(dev(c["fhat"], C128)))
    assert np.isnan(f[17])
    keep = np.arange(M) != 17
    ref = O.nndft_trafo(c["v"], c["x"], c["fhat"])
    assert parity_err(ref[keep], f[keep]) < 1e-12


def test_nnfft_trafo_before_nodes_raises():
    announce("nnfft state error")
    p = NNPlan((16,), 10, 10, m=4, dtype=C64).allocate()
    with pytest.raises(NfftError):
        p.trafo(torch.zeros(10, dtype=C64, device="cuda"))


def test_nnfft_bench_size_sampled():
    # the benchmark's NNFFT workload, checked on sampled outputs the oracle sums one by one
    w = W.workload("nnfft_d2")
    N, K, M = w["N"], w["K"], w["M"]
    announce("nnfft bench size", N, K, M)
    p = NNPlan(N, K, M, m=w["m"], dtype=C64).set_nodes(dev(w["x"], torch.float64), dev(w["v"], torch.float64))
    f = host(p.trafo(dev(w["fhat"], C64)))
    h = host(p.adjoint(dev(w["f"], C64)))
    r = np.random.default_rng(53)
    js = r.choice(M, 48, replace=False)
    ks = r.choice(K, 48, replace=False)
    ref_f = O.nndft_trafo(w["v"], w["x"][js], w["fhat"])
    ref_h = O.nndft_adjoint(w["v"][ks], w["x"], w["f"])
    assert parity_err(ref_f, f[js]) < TOL[C64]
    assert parity_err(ref_h, h[ks]) < TOL[C64]
