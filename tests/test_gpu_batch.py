"""Batched launches (nfft_batch_*) against per-plan launches and the FP64 oracle.

A batch launches each step kind once for all of its plans; every plan's result must
equal the per-plan call (the same arithmetic in the same order, so equal up to at most
the last bit: relative l2 <= 1e-6 in complex64, 1e-14 in complex128) and agree with the
oracle to the usual tolerances.  Covers mixed launch groups (dimensions, stencil
widths), more than 64 plans, every candidate launch shape of the autotuner, the tuning
cache round trip, and the full 64-plan workload.
"""
import numpy as np
import pytest
import torch

from gpu_util import TOL, announce, dev, host, parity_err
from oracle import oracle as O
from paper_1810_09891_amd import Batch, NfftError, Plan, workloads as W

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
SAME = {C64: 1e-6, C128: 1e-14}


def setup_plans(specs, dtype, seed0=0):
    """specs: (N, M, m, kind); returns plans with nodes set and their cases."""
    plans, cases = [], []
    for i, (N, M, m, kind) in enumerate(specs):
        c = W.small_case(len(N), N, M, seed=300 + seed0 + i, kind=kind)
        p = Plan(N, M, m=m, dtype=dtype)
        p.set_nodes(dev(c["x"], torch.float64))
        plans.append(p)
        cases.append(c)
    return plans, cases


def per_plan(plans, cases, dtype):
    fs = [host(p.trafo(dev(c["fhat"], dtype))) for p, c in zip(plans, cases)]
    hs = [host(p.adjoint(dev(c["f"], dtype))) for p, c in zip(plans, cases)]
    return fs, hs


def batched(batch, cases, dtype):
    fs = batch.trafo([dev(c["fhat"], dtype) for c in cases])
    fs = [host(f) for f in fs]
    hs = batch.adjoint([dev(c["f"], dtype) for c in cases])
    hs = [host(h) for h in hs]
    return fs, hs


MIXED = [
    ((64, 128), 3001, 6, "uniform"),
    ((128, 64), 1200, 6, "clustered"),
    ((32, 32), 5000, 6, "uniform"),
    ((256, 64), 700, 6, "wide"),
    ((64, 64), 2000, 4, "uniform"),   # another stencil width: second launch group
    ((512,), 4000, 6, "uniform"),     # d = 1
    ((16, 16, 16), 1500, 4, "uniform"),  # d = 3
]


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_batch_mixed_matches_per_plan_and_oracle(dtype):
    announce("batch mixed", dtype)
    plans, cases = setup_plans(MIXED, dtype)
    b = Batch(plans)
    assert b.info.groups == 4
    fb, hb = batched(b, cases, dtype)
    fp, hp = per_plan(plans, cases, dtype)
    for i, (p, c) in enumerate(zip(plans, cases)):
        assert parity_err(fp[i], fb[i]) <= SAME[dtype], i
        assert parity_err(hp[i], hb[i]) <= SAME[dtype], i
        f_ref = O.nfft_trafo(c["x"], c["fhat"], p.n, p.m)
        h_ref = O.nfft_adjoint(c["x"], c["f"], p.N, p.n, p.m)
        assert parity_err(f_ref, fb[i]) < TOL[dtype], i
        assert parity_err(h_ref, hb[i]) < TOL[dtype], i


def test_batch_c128_m8_reaches_direct_sums():
    announce("batch c128 m8 vs ndft")
    specs = [((32, 32), 700, 8, "uniform"), ((64, 32), 400, 8, "clustered"), ((32, 64), 900, 8, "uniform")]
    plans, cases = setup_plans(specs, C128, seed0=20)
    fb, hb = batched(Batch(plans), cases, C128)
    for i, c in enumerate(cases):
        assert parity_err(O.ndft_trafo(c["x"], c["fhat"]), fb[i]) < 1e-12
        assert parity_err(O.ndft_adjoint(c["x"], c["f"], specs[i][0]), hb[i]) < 1e-12


# every candidate of the autotuner for one step kind at a time, the rest at defaults
CANDIDATES = ([dict(pack_fwd=p, k_fwd=k) for p in (1, 2, 4, 8) for k in (0, 1, 2, 4, 8)]
              + [dict(pack_adj=p, k_adj=k) for p in (1, 2, 4, 8) for k in (0, 1, 2, 4, 8)]
              + [dict(k_interp=k, k_spread=k, k_fold=k) for k in (0, 1, 2, 4, 8, 16)])


def test_batch_every_launch_shape_gives_the_same_result():
    announce("batch launch shapes")
    specs = MIXED[:4]
    plans, cases = setup_plans(specs, C64, seed0=40)
    b = Batch(plans)
    fp, hp = per_plan(plans, cases, C64)
    for cand in CANDIDATES:
        b.set_params(0, **cand)
        fb, hb = batched(b, cases, C64)
        for i in range(len(plans)):
            assert parity_err(fp[i], fb[i]) <= SAME[C64], (cand, i)
            assert parity_err(hp[i], hb[i]) <= SAME[C64], (cand, i)


def test_batch_group_mixing_spreading_kernels():
    """Plans of one kind (d = 2, m = 4, complex64): one with 32-cell bins, which the
    spreading kernel that keeps tile columns in registers takes, and two with 16-cell bins
    (N = 8^2, 8 x 32), which it does not: the batch puts them in separate launch groups, so
    the first keeps the register kernel, and every plan matches its own transforms and the
    oracle."""
    announce("batch mixed spreading kernels")
    specs = [((64, 64), 3000, 4, "uniform"), ((8, 8), 300, 4, "uniform"), ((8, 32), 500, 4, "clustered")]
    plans, cases = setup_plans(specs, C64, seed0=140)
    b = Batch(plans)
    assert b.info.groups == 2
    fb, hb = batched(b, cases, C64)
    fp, hp = per_plan(plans, cases, C64)
    for i, (p, c) in enumerate(zip(plans, cases)):
        assert parity_err(fp[i], fb[i]) <= SAME[C64], i
        assert parity_err(hp[i], hb[i]) <= SAME[C64], i
        assert parity_err(O.nfft_adjoint(c["x"], c["f"], p.N, p.n, p.m), hb[i]) < TOL[C64], i


def test_batch_more_than_64_plans():
    announce("batch 70 plans")
    r = np.random.default_rng(11)
    specs = [((int(r.choice([16, 32, 64])), int(r.choice([16, 32]))), int(r.integers(50, 600)), 4, "uniform")
             for _ in range(70)]
    plans, cases = setup_plans(specs, C64, seed0=100)
    b = Batch(plans)
    assert b.info.groups == 2
    assert sorted(b.params(g)["plans"] for g in range(2)) == [6, 64]
    fb, hb = batched(b, cases, C64)
    fp, hp = per_plan(plans, cases, C64)
    for i in range(70):
        assert parity_err(fp[i], fb[i]) <= SAME[C64], i
        assert parity_err(hp[i], hb[i]) <= SAME[C64], i


def test_autotune_and_cache_round_trip(tmp_path):
    announce("batch autotune")
    cache = tmp_path / "tune.txt"
    plans, cases = setup_plans(MIXED[:5], C64, seed0=60)
    b = Batch(plans, tune_cache=cache)
    assert b.info.tuned == 0
    tuned = b.autotune()
    assert b.info.tuned == 1
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln and not ln.startswith("#")]
    assert len(lines) == b.info.groups
    assert all(len(ln) == 9 for ln in lines)
    # a new batch over the same plan shapes finds the tuned parameters in the cache
    b2 = Batch(plans, tune_cache=cache)
    assert b2.info.tuned == 1
    assert [b2.params(g) for g in range(b2.info.groups)] == tuned
    fb, hb = batched(b2, cases, C64)
    fp, hp = per_plan(plans, cases, C64)
    for i in range(len(plans)):
        assert parity_err(fp[i], fb[i]) <= SAME[C64]
        assert parity_err(hp[i], hb[i]) <= SAME[C64]


def test_batch_state_errors():
    plans, cases = setup_plans(MIXED[:2], C64, seed0=80)
    b = Batch(plans)
    fh = [dev(c["fhat"], C64) for c in cases]
    b.trafo(fh)
    plans[1].allocate()  # new workspace: the batch's descriptors are stale
    with pytest.raises(NfftError) as e:
        b.trafo(fh)
    assert e.value.status == -2
    torch.cuda.synchronize()


def test_batch_full_64_plan_workload():
    """64 plans, N_i from {64,...,512}^2, M_i log-uniform in [1e3, 2e5], complex64, m = 6:
    batched results against per-plan launches for every plan, and every plan's batched
    result against the FP64 oracle: the forward on up to 1024 sampled nodes, the adjoint on
    all coefficients; the largest plan also against the direct sums on sampled nodes."""
    announce("batch full 64 plans")
    specs = W.batch_plans()
    plans = []
    for s in specs:
        p = Plan(s["N"], s["M"], m=6, dtype=C64)
        p.set_nodes(dev(s["x"], torch.float64))
        plans.append(p)
    b = Batch(plans)
    assert b.info.groups == 1
    fb, hb = batched(b, specs, C64)
    fp, hp = per_plan(plans, specs, C64)
    for i in range(64):
        assert parity_err(fp[i], fb[i]) <= SAME[C64], i
        assert parity_err(hp[i], hb[i]) <= SAME[C64], i
    for i, s in enumerate(specs):
        sel = np.sort(np.random.default_rng(100 + i).choice(s["M"], min(1024, s["M"]), replace=False))
        assert parity_err(O.nfft_trafo(s["x"][sel], s["fhat"], None, 6), fb[i][sel]) < TOL[C64], i
        assert parity_err(O.nfft_adjoint(s["x"], s["f"], s["N"], None, 6), hb[i]) < TOL[C64], i
    order = np.argsort([s["M"] for s in specs])
    big = int(order[-1])
    s = specs[big]
    sel = np.sort(np.random.default_rng(3).choice(s["M"], 512, replace=False))
    f_ref = O.ndft_trafo(s["x"][sel], s["fhat"])
    assert parity_err(f_ref, fb[big][sel]) < TOL[C64]


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_batch_3d_output_tile_plans(dtype):
    """3-D plans whose spreading runs by output tiles, mixed with one that does not, in one
    batch: every plan's batched result equals its per-plan result and the oracle."""
    announce("batch 3-D output tiles", dtype)
    specs = [((32, 24, 40), 9000, 6, "clustered"), ((32, 32, 32), 4000, 6, "uniform"),
             ((16, 12, 20), 2000, 6, "wide")]
    plans, cases = setup_plans(specs, dtype, seed0=90)
    assert plans[0].info.own_tiles > 0 and plans[1].info.own_tiles > 0
    b = Batch(plans)
    fb, hb = batched(b, cases, dtype)
    fp, hp = per_plan(plans, cases, dtype)
    for i, (p, c) in enumerate(zip(plans, cases)):
        assert parity_err(fp[i], fb[i]) <= SAME[dtype], i
        assert parity_err(hp[i], hb[i]) <= SAME[dtype], i
        assert parity_err(O.nfft_adjoint(c["x"], c["f"], p.N, p.n, 6), hb[i]) < TOL[dtype], i
        assert parity_err(O.nfft_trafo(c["x"], c["fhat"], p.n, 6), fb[i]) < TOL[dtype], i
