"""Throughput of the NFFT forward + adjoint on one MI355X.

Headline workload: d = 3, N = (128, 128, 128), n = (256, 256, 256) (sigma = 2),
M = 2,097,152 nodes on 4096 radial spokes of 512 points (density clustered at the origin),
complex Gaussian data, Kaiser-Bessel window, m = 6, complex128 (FP64 throughout, the
paper's arithmetic): the plan shape of the paper's largest timing (Sec. 4, Fig. 4.6).
Reported beside it: the same workload in complex64; the d = 2 workload (N = 512^2,
M = 262144 uniform nodes) in complex64 and complex128 with m = 8 and m = 4 and with the
Gaussian window; d = 1 (N = 256, M = 1024, complex128, m = 8); 64 uneven d = 2 plans in one
batch (complex64, m = 6, autotuned, against per-plan launches); the differentiable d = 2
radial workload (forward + backward); a Gaussian-kernel fast summation; an NNFFT.

A step is one nfft_trafo plus one nfft_adjoint of the whole node set, inputs resident in
device memory (the node precomputation is timed separately, as Sec. 4 of the paper does).
value = M / (time of one step) in nonuniform points per second.  The K timed steps run as
R = min(10, K) back-to-back groups, each bracketed by HIP events on the stream; ms_per_step
is the whole window divided by K, ms_per_step_median the median over the groups.  A cold
figure repeats single steps after overwriting 1 GiB of device memory (more than the 256 MB
Infinity Cache) before each.

Kernel durations are measured live with HIP events: after the timed steps, the same number
of steps runs again with the library recording a HIP event pair around every launch on the
stream it launches on.  The dominant kernel's algorithmic bytes per launch (the byte model
below) over its average duration give the HBM roofline fraction; the binding fraction is
max(t_HBM, t_VALU) / t with t_VALU the multiply-add issue time of the window step.  The CPU
baseline is the FP64 oracle on the host's cores (a bounded sample, extrapolated: see
cpu_baseline); the E_2 errors are against the oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--graph] [--no-cpu]
                    [--primary-only] [--copy-calibration-mib MIB]
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NFFT fwd+adj nonuniform points/s at stated rel-ℓ2 error; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# VALU issue rate of one MI355X: 256 CUs x 64 lanes x 2.4 GHz lane-slots per second.  A
# (node, cell) pair of the window steps is one complex x real multiply-add: two FP64 FMAs
# (complex128) or two FP32 FMAs (complex64; one packed FMA if packed FP32 were used, which
# the library's code does not emit).
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9
# dense matrix-core peaks of one MI355X (FP64 and FP32 MFMA)
MFMA_F64_FLOPS = 78.6e12
MFMA_F32_FLOPS = 157.3e12
# LDS read ceiling of one MI355X measured with _build/lds_bw (conflict-free
# 8-byte reads issued as separate ds_read_b64, all 256 CUs; the highest 8-byte read rate it
# measures): the bound of the interpolation kernel (an 8-byte LDS read per stencil point)
LDS_READ8_PEAK_GBS = 128000.0
# Published FP32 vector peak of the MI355X (256 CUs, 2.4 GHz, packed FP32 counted) and the
# FP64 vector peak.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
PROFILES = os.path.join(ROOT, "profiles")
# HBM traffic of the headline kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated)
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_d3_radial_128_c128_m6.json")
# Context only: the paper's own timing of the same plan shape (Sec. 4, Fig. 4.6): forward
# NFFT, d = 3, N = 128^3, n = 256^3, m = 6, M = 2 * 128^3 uniform nodes, FP64, 10 threads of
# a 4 x Intel Xeon E7-4880 v2 (2.5 GHz) machine, 4.05 s per transform.
PAPER_CONTEXT = {
    "value": 4194304 / 4.05,
    "unit": "points/s",
    "what": "forward NFFT only (the paper times no adjoint), d=3 N=128^3 n=256^3 m=6, M=4,194,304 uniform "
            "nodes, FP64, 10 threads of 4x Intel Xeon E7-4880 v2 @ 2.5 GHz: 4.05 s (Sec. 4, Fig. 4.6)",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(name, d, N, n, M, cbytes):
    """Bytes a step must move at least once (per launch) for this plan.

    Window steps (interpolation, spreading, node gradient): the FP64 nodes (8 d bytes), the
    value (cbytes) per node and the grid once, M (8 d + cbytes) + |I_n| cbytes.  FFT pass
    over dimension t: its nonzero input and its output once; a forward pass reads lines of
    N_t entries (coefficients for the first pass) and writes n_t, an adjoint pass reads n_t
    and writes N_t (coefficients for the last), with earlier dimensions already pruned to
    N and later ones full.  The fold of split output tiles is overhead (no algorithmic
    bytes of its own)."""
    import numpy as np

    window = M * (8 * d + cbytes) + int(np.prod(n)) * cbytes
    if name in ("interp", "grad_x", "spread_tiles", "spread_own"):
        return window

    def fft_pass(t, forward):
        before = int(np.prod(N[:t])) if t > 0 else 1
        after = int(np.prod(n[t + 1:])) if t + 1 < d else 1
        return cbytes * before * after * (N[t] + n[t])

    fwd_order = list(range(d - 1, -1, -1))  # first forward pass: last dimension
    adj_order = list(range(d))               # last adjoint pass: last dimension
    if name == "fft_fwd_deconv":
        return fft_pass(fwd_order[0], True)
    if name == "fft_adj_deconv":
        return fft_pass(adj_order[-1], False)
    if name == "fft_fwd":  # average of the remaining forward passes
        return sum(fft_pass(t, True) for t in fwd_order[1:]) // max(1, d - 1)
    if name == "fft_adj":
        return sum(fft_pass(t, False) for t in adj_order[:-1]) // max(1, d - 1)
    return None


def valu_seconds(d, M, m, dbl):
    """Multiply-add issue time of one window step: (2m+2)^d (node, cell) pairs, one complex x
    real multiply-add each (two FMA slots)."""
    return M * (2 * m + 2) ** d * 2 / VALU_SLOTS_PER_S


def mfma_seconds(d, M, m, dbl):
    """The same multiply-adds on the matrix cores at their dense peak (FP64 78.6 TFLOP/s,
    FP32 157.3 TFLOP/s): the floor of the 3-D spreading by output tiles."""
    return M * (2 * m + 2) ** d * 4 / (MFMA_F64_FLOPS if dbl else MFMA_F32_FLOPS)


# rocprofv3 kernel names of the library's launch labels, in order of preference
ROCPROF_NAME = {"interp": ("k_interp3", "k_interp_nodes"),
                "spread_tiles": ("k_spread_cols", "k_spread_tiles"), "spread_own": ("k_spread_own_mx",),
                "spread_fold": ("k_fold",), "grad_x": ("k_grad_x",)}


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


class Case:
    def __init__(self, w, m, dtype, torch, window="kaiser-bessel"):
        from paper_1810_09891_amd import Plan

        self.w = w
        self.m = m
        self.dtype = dtype
        self.torch = torch
        dev = torch.device("cuda:0")
        self.plan = Plan(w["N"], w["M"], n=w["n"], m=m, dtype=dtype, device=dev, window=window)
        self.x = torch.as_tensor(w["x"]).to(dev)
        self.fhat = torch.as_tensor(w["fhat"]).to(dev, dtype)
        self.f = torch.as_tensor(w["f"]).to(dev, dtype)
        self.out_f = torch.empty(w["M"], dtype=dtype, device=dev)
        self.out_h = torch.empty(w["N"], dtype=dtype, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        self.graph = None

    def set_nodes_ms(self, reps=5):
        torch = self.torch
        self.plan.set_nodes(self.x)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            self.plan.set_nodes(self.x)
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def step(self):
        self.plan.trafo(self.fhat, out=self.out_f)
        self.plan.adjoint(self.f, out=self.out_h)

    def capture(self):
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(self.stream)
        with torch.cuda.stream(s):
            self.step()  # tables uploaded, kernels attributed before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        torch.cuda.synchronize()
        self.graph = g

    def run(self, steps):
        if self.graph is not None:
            for _ in range(steps):
                self.graph.replay()
        else:
            for _ in range(steps):
                self.step()

    def time_steps(self, steps, warmup, events):
        """Time exactly `steps` steps after `warmup` untimed ones, as R = min(10, steps)
        back-to-back groups bracketed by HIP events on the stream (synchronised before and
        after).  Returns (window / steps, median over the groups of ms per step, per-launch
        kernel averages when `events`)."""
        torch = self.torch
        self.run(warmup)
        torch.cuda.synchronize()
        if events:
            self.plan.profile(True)
            self.plan.profile_read()
        stream = torch.cuda.current_stream()
        R = max(1, min(10, steps))
        per = [steps // R + (1 if i < steps % R else 0) for i in range(R)]
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(R + 1)]
        evs[0].record(stream)
        for i in range(R):
            self.run(per[i])
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        total = evs[0].elapsed_time(evs[R])
        groups = sorted(evs[i].elapsed_time(evs[i + 1]) / per[i] for i in range(R))
        median = groups[R // 2] if R % 2 else 0.5 * (groups[R // 2 - 1] + groups[R // 2])
        kt = None
        if events:
            res = self.plan.profile_read()
            self.plan.profile(False)
            kt = {k: (v[0] / v[1], v[1]) for k, v in res.items()}
        return total / steps, median, kt

    def time_cold(self, reps):
        """Median ms of single steps, each after overwriting 1 GiB of device memory (more
        than the 256 MB Infinity Cache), so that grid, nodes and values come from HBM."""
        torch = self.torch
        flush = torch.empty(1 << 28, dtype=torch.float32, device=self.x.device)
        stream = torch.cuda.current_stream()
        times = []
        for _ in range(reps):
            flush.fill_(1.0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            self.step()
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        del flush
        times.sort()
        return times[len(times) // 2]

    def outputs(self):
        torch = self.torch
        self.step()
        torch.cuda.synchronize()
        return self.out_f.cpu().numpy(), self.out_h.cpu().numpy()


def cpu_baseline(w, m, reps, window="kaiser-bessel"):
    """Serial FP64 oracle NFFT + adjoint on the full workload (one core)."""
    import numpy as np

    from oracle import oracle as O

    times = []
    f_ref = h_ref = None
    for _ in range(reps):
        t0 = time.perf_counter()
        with O.window(window):
            f_ref = O.nfft_trafo(w["x"], w["fhat"], w["n"], m)
            h_ref = O.nfft_adjoint(w["x"], w["f"], w["N"], w["n"], m)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"seconds_per_step": t, "f": f_ref, "h": h_ref, "runs": reps}


def e2(ref, approx):
    import numpy as np

    ref = np.ravel(ref).astype(np.complex128)
    approx = np.ravel(approx).astype(np.complex128)
    return float(np.linalg.norm(ref - approx) / np.linalg.norm(ref))


def sample(n, k, seed):
    import numpy as np

    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False))


def cuda_time(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(steps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


# ------------------------------------------------------------------ other workloads

def bench_d1(torch, steps, warmup, check):
    """d = 1, N = 256, M = 1024, complex128, m = 8 against the direct sums."""
    from oracle import oracle as O
    from paper_1810_09891_amd import workloads as W

    w = W.workload("d1")
    case = Case(w, 8, torch.complex128, torch)
    case.set_nodes_ms()
    ms, _, _ = case.time_steps(steps, warmup, False)
    f, h = case.outputs()
    r = {"workload": "d=1 N=256 n=512 M=1024 uniform, complex128, m=8", "ms_per_step": ms,
         "points_per_s": w["M"] / (ms * 1e-3)}
    if check:
        r["e2_trafo_vs_ndft"] = e2(O.ndft_trafo(w["x"], w["fhat"]), f)
        r["e2_adjoint_vs_ndft"] = e2(O.ndft_adjoint(w["x"], w["f"], w["N"]), h)
    return r


# Fig. 4.5 (d = 3) of the paper: its forward transform times in ms (and precomputation
# times) for the test polynomial f_3, N = 32^3, M = 65536, n = 2N, against the window size m
PAPER_FIG45_D3 = {"trafo_ms": {2: 39.57, 3: 80.42, 4: 191.90, 5: 311.19, 6: 468.07, 7: 657.49, 8: 896.82,
                               9: 1182.30, 10: 1529.24},
                  "precompute_ms": {2: 60.00, 3: 76.88, 4: 93.51, 5: 109.09, 6: 114.44, 7: 124.89, 8: 138.31,
                                    9: 153.43, 10: 163.47}}


def bench_window_sweep_d3(torch, steps, warmup, check):
    """The paper's d = 3 window-size sweep (Fig. 4.4(a) errors, Fig. 4.5 times): test
    polynomial f_3, N = 32^3, M = 65536 uniform nodes, n = 2N, complex128, m = 2 .. 10.  m >= 9
    stage the interpolation tile in slabs.  Per m: forward-only and forward+adjoint time, node
    precomputation, and E_2 against the GPU's direct sums."""
    import numpy as np

    from paper_1810_09891_amd import workloads as W

    w = dict(W.paper_workload(3))
    w["n"] = tuple(2 * v for v in w["N"])
    r = np.random.default_rng(4545)
    w["f"] = r.standard_normal(w["M"]) + 1j * r.standard_normal(w["M"])
    per_m = {}
    ref = None
    for m in range(2, 11):
        case = Case(w, m, torch.complex128, torch)
        t_nodes = case.set_nodes_ms()
        ms, _, _ = case.time_steps(steps, warmup, False)
        p = case.plan
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(case.stream)
        for _ in range(steps):
            p.trafo(case.fhat, out=case.out_f)
        b.record(case.stream)
        torch.cuda.synchronize()
        e = {"trafo_ms": a.elapsed_time(b) / steps, "trafo_adjoint_ms": ms, "set_nodes_ms": t_nodes}
        if check:
            if ref is None:
                ref = p.ndft_trafo(case.fhat).cpu().numpy()
            e["e2_trafo_vs_ndft"] = e2(ref, case.out_f.cpu().numpy())
        e["paper_trafo_ms"] = PAPER_FIG45_D3["trafo_ms"][m]
        per_m[str(m)] = e
        del case, p
        torch.cuda.empty_cache()
    return {"workload": "paper test polynomial f_3: d=3 N=(32,32,32) n=(64,64,64) M=65536 uniform, complex128, "
                        "m=2..10 (m >= 9: interpolation in slabs)",
            "per_m": per_m, "ms_per_step": per_m["8"]["trafo_adjoint_ms"],
            "points_per_s": w["M"] / (per_m["8"]["trafo_adjoint_ms"] * 1e-3),
            "paper_context": "Fig. 4.5 (d = 3): forward transform times of the paper's CPU runs, per m"}


D3_WORKLOAD = ("d=3 N=(128,128,128) n=(256,256,256) M=2097152 on 4096 radial spokes of 512 points "
               "(density clustered at the origin), Kaiser-Bessel m=6, %s, trafo+adjoint")


class D3Refs:
    """Oracle references for the 3-D radial workload, computed once: the oversampled grid
    (Algorithm 2.1 steps 1-2) at full size, the forward transform at 16384 sampled nodes
    (step 3 on that grid) and the adjoint at 64 sampled coefficients (direct sums, eq. (1.3)).
    The timings of these oracle steps give the CPU baseline (see cpu_baseline_3d)."""

    def __init__(self, w, m):
        import numpy as np

        from oracle import oracle as O

        O.set_threads(os.cpu_count() or 1)
        self.threads = O.get_threads()
        self.sel = sample(w["M"], 16384, 3)
        self.ks = sample(int(np.prod(w["N"])), 64, 4)
        t0 = time.perf_counter()
        g = O.nfft_grid(w["fhat"], w["n"], m)
        self.t_grid = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.f_sel = O.nfft_interp(w["x"][self.sel], g, w["N"], m)
        self.t_interp = time.perf_counter() - t0
        t0 = time.perf_counter()
        gs = O.nfft_spread(w["x"][self.sel], w["f"][self.sel], w["N"], w["n"], m)
        self.t_spread = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.nfft_adjoint_from_grid(gs, w["N"], m)
        self.t_coef = time.perf_counter() - t0
        del g, gs
        t0 = time.perf_counter()
        self.h_ks = O.ndft_adjoint_at(w["x"], w["f"], w["N"], self.ks)
        self.t_ndft = time.perf_counter() - t0
        self.M = w["M"]
        self.Ms = len(self.sel)

    def cpu_seconds_per_step(self):
        """Oracle NFFT + adjoint NFFT of the whole workload, extrapolated: deconvolution and
        FFT steps timed at full size, the window steps on the 16384-node sample scaled by
        M / 16384 (their cost is proportional to the number of nodes)."""
        return self.t_grid + self.t_coef + (self.t_interp + self.t_spread) * self.M / self.Ms


def run_d3(torch, w, dtype, steps, warmup, refs, cold_reps=5):
    """The 3-D radial workload at one precision: timed steps, kernel averages, cold steps,
    node precomputation, errors against the oracle references."""
    case = Case(w, 6, dtype, torch)
    t_nodes = case.set_nodes_ms(reps=3)
    ms, med, _ = case.time_steps(steps, warmup, False)
    ms_ev, _, kt = case.time_steps(steps, warmup, True)
    cold = case.time_cold(cold_reps)
    f, h = case.outputs()
    r = {"workload": D3_WORKLOAD % ("complex128" if dtype == torch.complex128 else "complex64"),
         "dtype": "c128" if dtype == torch.complex128 else "c64", "m": 6,
         "ms_per_step": ms, "ms_per_step_median": med, "ms_per_step_cold": cold,
         "ms_per_step_with_events": ms_ev, "steps": steps,
         "points_per_s": w["M"] / (ms * 1e-3), "set_nodes_ms": t_nodes,
         "kernels_ms": {k: round(v[0], 5) for k, v in sorted(kt.items())}, "_kernel_avg": kt,
         "_w": (w["N"], w["n"], w["M"])}
    if refs is not None:
        r["e2_trafo_vs_oracle_16384_nodes"] = e2(refs.f_sel, f[refs.sel])
        r["e2_adjoint_vs_ndft_64_coefficients"] = e2(refs.h_ks, h.reshape(-1)[refs.ks])
    del case
    torch.cuda.empty_cache()
    return r


def bench_batch(torch, steps, warmup, check):
    """64 d = 2 plans, N_i in {64,...,512}^2, M_i log-uniform in [1e3, 2e5], complex64,
    m = 6: one batch (autotuned) against the same plans launched one by one."""
    import numpy as np

    from oracle import oracle as O
    from paper_1810_09891_amd import Batch, Plan, workloads as W

    specs = W.batch_plans()
    C64 = torch.complex64
    plans, fh, fv = [], [], []
    for s in specs:
        p = Plan(s["N"], s["M"], m=6, dtype=C64)
        p.set_nodes(torch.as_tensor(s["x"]).cuda())
        plans.append(p)
        fh.append(torch.as_tensor(s["fhat"]).to("cuda", C64))
        fv.append(torch.as_tensor(s["f"]).to("cuda", C64))
    outs_f = [torch.empty(s["M"], dtype=C64, device="cuda") for s in specs]
    outs_h = [torch.empty(s["N"], dtype=C64, device="cuda") for s in specs]
    with tempfile.TemporaryDirectory() as td:
        b = Batch(plans, tune_cache=os.path.join(td, "tune.txt"))
        t0 = time.perf_counter()
        params = b.autotune()
        tune_s = time.perf_counter() - t0

    def batched():
        b.trafo(fh, outs_f)
        b.adjoint(fv, outs_h)

    def sequential():
        for p, a, o in zip(plans, fh, outs_f):
            p.trafo(a, out=o)
        for p, a, o in zip(plans, fv, outs_h):
            p.adjoint(a, out=o)

    ms_b = cuda_time(torch, batched, steps, warmup)
    ms_s = cuda_time(torch, sequential, steps, warmup)
    Mtot = int(sum(s["M"] for s in specs))

    # the same plans with measured bin edges and work-item caps (nfft_plan_tune per plan
    # shape, one cache for all), batched and autotuned again
    from paper_1810_09891_amd import tune_plan_params
    with tempfile.TemporaryDirectory() as td:
        t0 = time.perf_counter()
        tplans, chosen = [], []
        for s in specs:
            x = torch.as_tensor(s["x"]).cuda()
            prm, _ = tune_plan_params(s["N"], s["M"], x, m=6, dtype=C64, cache=os.path.join(td, "plans.txt"))
            p = Plan(s["N"], s["M"], m=6, dtype=C64, params=prm)
            p.set_nodes(x)
            tplans.append(p)
            chosen.append(prm)
        plan_tune_s = time.perf_counter() - t0
        bt = Batch(tplans, tune_cache=os.path.join(td, "tune.txt"))
        bt.autotune()
    outs_ft = [torch.empty(s["M"], dtype=C64, device="cuda") for s in specs]
    outs_ht = [torch.empty(s["N"], dtype=C64, device="cuda") for s in specs]

    def batched_tuned():
        bt.trafo(fh, outs_ft)
        bt.adjoint(fv, outs_ht)

    ms_t = cuda_time(torch, batched_tuned, steps, warmup)
    defaults = [{"bin": tuple(int(p.info.bin[t]) for t in range(2)), "chunk_cap": int(p.info.chunk_cap)}
                for p in plans]
    r = {"workload": "64 plans d=2, N_i from {64,128,256,512}^2, M_i log-uniform in [1e3,2e5] "
                     "(total M=%d, total grid points=%d), complex64, m=6" %
                     (Mtot, int(sum(4 * np.prod(s["N"]) for s in specs))),
         "ms_per_step": ms_b, "points_per_s": Mtot / (ms_b * 1e-3),
         "sequential_ms_per_step": ms_s, "sequential_points_per_s": Mtot / (ms_s * 1e-3),
         "speedup_vs_sequential": ms_s / ms_b, "autotune_s": tune_s, "params": params,
         "tuned_plan_params": {
             "what": "bin edges and work-item cap measured per plan shape (nfft_plan_tune), then batched",
             "ms_per_step": ms_t, "points_per_s": Mtot / (ms_t * 1e-3), "plan_tune_s": plan_tune_s,
             "speedup_vs_default_params": ms_b / ms_t,
             "plans_changed": int(sum(c != dflt for c, dflt in zip(chosen, defaults))),
             "chosen": sorted({(c["bin"], c["chunk_cap"]) for c in chosen})}}
    if check:
        batched_tuned()
        ft = [o.cpu().numpy() for o in outs_ft]
        ht = [o.cpu().numpy() for o in outs_ht]
        batched()
        fb = [o.cpu().numpy() for o in outs_f]
        hb = [o.cpu().numpy() for o in outs_h]
        sequential()
        fs = [o.cpu().numpy() for o in outs_f]
        hs = [o.cpu().numpy() for o in outs_h]
        r["max_e2_batched_vs_per_plan"] = max(max(e2(a, c) for a, c in zip(fs, fb)),
                                             max(e2(a, c) for a, c in zip(hs, hb)))
        r["tuned_plan_params"]["max_e2_vs_default_params"] = max(max(e2(a, c) for a, c in zip(fb, ft)),
                                                                 max(e2(a, c) for a, c in zip(hb, ht)))
        order = np.argsort([s["M"] for s in specs])
        worst = 0.0
        for i in order[:3]:
            s = specs[i]
            worst = max(worst, e2(O.nfft_trafo(s["x"], s["fhat"], None, 6), fb[i]),
                        e2(O.nfft_adjoint(s["x"], s["f"], s["N"], None, 6), hb[i]))
        r["max_e2_vs_oracle_3_smallest_plans"] = worst
    b.close()
    bt.close()
    return r


def bench_grad(torch, steps, warmup, check):
    """d = 2, N = (256,256), 256 spokes x 256 points + N(0, 1e-3^2) jitter, complex64,
    m = 6: loss ||A(x) fhat - y||^2, forward and backward for fhat and x."""
    import numpy as np

    from oracle import oracle as O
    from paper_1810_09891_amd import differentiable_plan, nfft, workloads as W

    w = W.workload("grad")
    N, M, x = w["N"], w["M"], w["x"]
    r0 = W.rng("grad", 1)
    fhat_star = W.cgauss(r0, N)
    fhat = W.cgauss(r0, N)
    y = O.nfft_trafo(x, fhat_star, None, 8)
    plan = differentiable_plan(N, M, m=6, dtype=torch.complex64)
    xt = torch.tensor(x, device="cuda", dtype=torch.float64, requires_grad=True)
    ft = torch.tensor(fhat, device="cuda", dtype=torch.complex64, requires_grad=True)
    yt = torch.tensor(y, device="cuda", dtype=torch.complex64)

    def step():
        xt.grad = None
        ft.grad = None
        f = nfft(xt, ft, plan)
        loss = torch.sum(torch.abs(f - yt) ** 2)
        loss.backward()

    ms = cuda_time(torch, step, steps, warmup)
    r = {"workload": "d=2 N=(256,256) M=65536 on 256 radial spokes + N(0,1e-3^2) jitter, complex64, m=6; "
                     "loss ||A(x)fhat - y||^2, forward + backward (set_nodes, trafo, grad_x, adjoint)",
         "ms_per_step": ms, "points_per_s": M / (ms * 1e-3)}
    if check:
        step()
        gx = xt.grad.detach().cpu().numpy()
        gf = ft.grad.detach().cpu().numpy()
        res = O.nfft_trafo(x, fhat, None, 8) - y
        r["e2_grad_fhat_vs_oracle"] = e2(2.0 * O.nfft_adjoint(x, res, N, None, 8), gf)
        sel = sample(M, 256, 5)
        gref = O.ndft_grad_x(x[sel], fhat, res[sel])
        r["e2_grad_x_vs_ndft_256_nodes"] = float(np.linalg.norm(gx[sel] - gref) / np.linalg.norm(gref))
    return r


def bench_fastsum(torch, steps, warmup, check):
    """Fast summation with a Gaussian kernel: d = 2, N = (128, 128), 32768 source and
    32768 target nodes uniform on [-1/2, 1/2)^2, complex64, m = 6, c = 0.05."""
    import numpy as np

    from oracle import oracle as O
    from paper_1810_09891_amd import Plan, fastsum, gaussian_coefficients, workloads as W

    r = W.rng("fastsum", 0)
    N, M, cw = (128, 128), 32768, 0.05
    x = W.uniform_nodes(r, M, 2)
    y = W.uniform_nodes(r, M, 2)
    alpha = W.cgauss(r, (M,))
    C64 = torch.complex64
    px = Plan(N, M, m=6, dtype=C64).set_nodes(torch.as_tensor(x).cuda())
    py = Plan(N, M, m=6, dtype=C64).set_nodes(torch.as_tensor(y).cuda())
    bhat = gaussian_coefficients(N, cw, dtype=C64)
    a = torch.as_tensor(alpha).to("cuda", C64)
    out = torch.empty(M, dtype=C64, device="cuda")
    ms = cuda_time(torch, lambda: fastsum(px, py, bhat, a, out=out), steps, warmup)
    r_ = {"workload": "fast summation, Gaussian kernel c=0.05: d=2 N=(128,128), 32768 sources and 32768 targets "
                      "uniform, complex64, m=6 (adjoint NFFT with the kernel product fused, then NFFT)",
          "ms_per_step": ms, "points_per_s": 2 * M / (ms * 1e-3)}
    if check:
        fastsum(px, py, bhat, a, out=out)
        g = out.cpu().numpy()
        sel = sample(M, 512, 6)
        ref = O.fastsum(x, y[sel], gaussian_coefficients(N, cw, device="cpu").numpy(), alpha)
        r_["e2_vs_oracle_512_targets"] = e2(ref, g[sel])
    return r_


def bench_nnfft(torch, steps, warmup, check):
    """NNFFT (nonequispaced in both domains): d = 2, N = (256, 256), 131072 frequencies and
    131072 nodes uniform, complex64, m = 8; one step is a transform and its adjoint."""
    from oracle import oracle as O
    from paper_1810_09891_amd import NNPlan, workloads as W

    w = W.workload("nnfft_d2")
    C64 = torch.complex64
    p = NNPlan(w["N"], w["K"], w["M"], m=w["m"], dtype=C64)
    p.set_nodes(torch.as_tensor(w["x"]).cuda(), torch.as_tensor(w["v"]).cuda())
    fh = torch.as_tensor(w["fhat"]).to("cuda", C64)
    fv = torch.as_tensor(w["f"]).to("cuda", C64)
    f = torch.empty(w["M"], dtype=C64, device="cuda")
    h = torch.empty(w["K"], dtype=C64, device="cuda")

    def step():
        p.trafo(fh, out=f)
        p.adjoint(fv, out=h)

    ms = cuda_time(torch, step, steps, warmup)
    r_ = {"workload": "NNFFT d=2 N=(256,256) (frequency grid %s, sigma1 %.3f), K=131072 frequencies and "
                      "M=131072 nodes uniform, complex64, m=8, trafo+adjoint" % (list(p.N2), p.sigma1[0]),
          "ms_per_step": ms, "points_per_s": (w["K"] + w["M"]) / (ms * 1e-3)}
    if check:
        step()
        fo = f.cpu().numpy()
        ho = h.cpu().numpy()
        js = sample(w["M"], 256, 7)
        ks = sample(w["K"], 256, 8)
        r_["e2_trafo_vs_nndft_256"] = e2(O.nndft_trafo(w["v"], w["x"][js], w["fhat"]), fo[js])
        r_["e2_adjoint_vs_nndft_256"] = e2(O.nndft_adjoint(w["v"][ks], w["x"], w["f"]), ho[ks])
    return r_


def roofline_entry(name, avg_ms, d, N, n, M, m, cbytes, dbl):
    """HBM fraction of a kernel under the byte model, and for the window kernels the
    binding fraction max(t_HBM, t_VALU) / t."""
    bts = algorithmic_bytes(name, d, N, n, M, cbytes)
    e = {"avg_ms": round(avg_ms, 5), "algorithmic_bytes": bts}
    if bts is not None:
        e["hbm_GBs"] = round(bts / (avg_ms * 1e-3) / 1e9, 1)
        e["hbm_frac"] = round(bts / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        if name in ("interp", "spread_own", "spread_tiles", "grad_x"):
            t_hbm = bts / (HBM_PEAK_GBS * 1e9)
            e["t_hbm_us"] = round(t_hbm * 1e6, 2)
            if name == "spread_own":  # runs on the matrix cores
                t_ar, unit = mfma_seconds(d, M, m, dbl), "mfma"
            else:
                t_ar, unit = valu_seconds(d, M, m, dbl), "valu"
            e["t_%s_us" % unit] = round(t_ar * 1e6, 2)
            e["binding"] = unit if t_ar > t_hbm else "hbm"
            e["binding_frac"] = round(max(t_hbm, t_ar) / (avg_ms * 1e-3), 4)
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--graph", action="store_true", help="replay the d=2 steps as captured HIP graphs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the E_2 checks")
    ap.add_argument("--primary-only", action="store_true", help="only the headline plan")
    ap.add_argument("--d2-only", action="store_true",
                    help="only the d=2 N=512^2 complex64 m=8 workload, K steps (for profiling; prints its own line)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the design notes "
              "describe how the transform would shard); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1810_09891_amd import workloads as W
    from paper_1810_09891_amd.profiling import source_hash

    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read, %d MiB written" % (args.copy_calibration_mib, args.copy_calibration_mib))
        del src, dst

    C64, C128 = torch.complex64, torch.complex128
    KB, GAUSS = "kaiser-bessel", "gaussian"
    check = not args.no_cpu

    if args.d2_only:
        w = W.workload("d2", m=8)
        case = Case(w, 8, C64, torch, KB)
        t_nodes = case.set_nodes_ms()
        ms, med, _ = case.time_steps(args.steps, 1, events=False)
        print(json.dumps({"workload": "d=2 N=(512,512) n=(1024,1024) M=262144 uniform nodes, kaiser-bessel m=8, "
                                      "complex64, trafo+adjoint", "steps": args.steps, "ms_per_step": ms,
                          "points_per_s": w["M"] / (ms * 1e-3), "set_nodes_ms": t_nodes}), flush=True)
        return

    # ---------------------------------------------------------------- headline: 3-D radial, c128
    w3 = W.workload("d3r")
    refs = None
    if check:
        t0 = time.perf_counter()
        refs = D3Refs(w3, 6)
        log("oracle references for d=3 radial: %.1f s (%d threads)" % (time.perf_counter() - t0, refs.threads))
    head = run_d3(torch, w3, C128, args.steps, args.warmup, refs)
    log("headline d=3 radial c128 m=6: %.4f ms/step (median %.4f, cold %.4f), %.3e points/s, set_nodes %.3f ms" %
        (head["ms_per_step"], head["ms_per_step_median"], head["ms_per_step_cold"], head["points_per_s"],
         head["set_nodes_ms"]))
    variants = []
    if not args.primary_only:
        v = run_d3(torch, w3, C64, args.steps, args.warmup, refs)
        log("d=3 radial c64 m=6: %.4f ms/step, %.3e points/s" % (v["ms_per_step"], v["points_per_s"]))
        variants.append(v)

    # ---------------------------------------------------------------- d = 2 variants
    cpu2 = {}
    if not args.primary_only:
        for m, dtype, window in ((8, C64, KB), (8, C128, KB), (4, C64, KB), (4, C128, KB), (8, C64, GAUSS)):
            w = W.workload("d2", m=m)
            case = Case(w, m, dtype, torch, window)
            t_nodes = case.set_nodes_ms()
            if args.graph:
                case.capture()
            steps = 1000  # >= 10 ms per repeat group at about 0.1 ms per step
            ms, med, _ = case.time_steps(steps, 20, events=False)
            ms_events, _, kt = case.time_steps(steps // 4, 20, events=not args.graph)
            f_gpu, h_gpu = case.outputs()
            r = {"workload": "d=2 N=(512,512) n=(1024,1024) M=262144 uniform nodes, %s m=%d, %s, trafo+adjoint" %
                             (window, m, "complex64" if dtype == C64 else "complex128"),
                 "m": m, "window": window, "dtype": "c64" if dtype == C64 else "c128",
                 "ms_per_step": ms, "ms_per_step_median": med, "ms_per_step_with_events": ms_events,
                 "points_per_s": w["M"] / (ms * 1e-3), "set_nodes_ms": t_nodes, "steps": steps,
                 "kernels_ms": None if kt is None else {k: round(v[0], 5) for k, v in sorted(kt.items())}}
            if kt is not None:
                r["kernels"] = {k: roofline_entry(k, a, 2, w["N"], w["n"], w["M"], m, 8 if dtype == C64 else 16,
                                                  dtype == C128) for k, (a, _) in sorted(kt.items())}
            if check:
                if (m, window) not in cpu2:
                    cpu2[(m, window)] = cpu_baseline(w, m, reps=1, window=window)
                r["e2_trafo_vs_oracle"] = e2(cpu2[(m, window)]["f"], f_gpu)
                r["e2_adjoint_vs_oracle"] = e2(cpu2[(m, window)]["h"], h_gpu)
                if (m, window) == (8, KB) and dtype == C64:
                    r["cpu_oracle_points_per_s_1_thread"] = w["M"] / cpu2[(m, window)]["seconds_per_step"]
            variants.append(r)
            log("d=2 %s m=%d %s: %.4f ms/step, %.3e points/s" % (r["dtype"], m, window, ms, r["points_per_s"]))
            del case
            torch.cuda.empty_cache()

    extra = {}
    if not args.primary_only:
        for name, fn, st in (("d1_256_c128_m8", bench_d1, 200), ("batch64_c64_m6", bench_batch, 20),
                             ("grad_radial_256_c64_m6", bench_grad, 20),
                             ("fastsum_gauss_128_c64_m6", bench_fastsum, 50),
                             ("nnfft_d2_256_c64_m8", bench_nnfft, 50),
                             ("window_sweep_d3_32_c128", bench_window_sweep_d3, 20)):
            t0 = time.perf_counter()
            extra[name] = fn(torch, st, 3, check)
            log("%s: %.4f ms/step, %.3e points/s (%.1f s)" %
                (name, extra[name]["ms_per_step"], extra[name]["points_per_s"], time.perf_counter() - t0))
            torch.cuda.empty_cache()

    # ---------------------------------------------------------------- roofline of the headline
    N, n, M = head["_w"]
    kt = head["_kernel_avg"]
    per_kernel = {k: roofline_entry(k, a, 3, N, n, M, 6, 16, True) for k, (a, _) in sorted(kt.items())}
    for k, (a, c) in kt.items():
        per_kernel[k]["launches"] = c
    dom = max((k for k in kt if not k.startswith("nodes")), key=lambda k: kt[k][0])
    e = per_kernel[dom]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_hash") == source_hash():
            for kname in ROCPROF_NAME.get(dom, ()):
                entry = tr.get("kernels", {}).get(kname)
                if entry is not None and "bytes_per_launch" in entry:
                    traffic = entry["bytes_per_launch"]
                    break
    if e.get("binding") == "mfma":
        # a matrix-core contraction: algorithmic flops per launch against the FP64 MFMA peak
        flops = M * (2 * 6 + 2) ** 3 * 4
        achieved = flops / (e["avg_ms"] * 1e-3) / 1e12
        bound = {"bound": "mfma", "achieved": round(achieved, 2), "peak": MFMA_F64_FLOPS / 1e12,
                 "unit": "TFLOP/s", "frac": round(achieved * 1e12 / MFMA_F64_FLOPS, 4), "algorithmic_flops": flops,
                 "hbm_GBs": e.get("hbm_GBs"), "hbm_frac": e.get("hbm_frac")}
    else:
        bound = {"bound": "hbm", "achieved": e.get("hbm_GBs"), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": e.get("hbm_frac")}
    roofline = {
        **bound,
        "kernel": dom,
        "traffic": traffic,
        "algorithmic_bytes": e.get("algorithmic_bytes"),
        "avg_launch_ms": e["avg_ms"],
        "binding": e.get("binding"),
        "binding_frac": e.get("binding_frac"),
        "t_hbm_us": e.get("t_hbm_us"),
        "t_valu_us": e.get("t_valu_us"),
        "t_mfma_us": e.get("t_mfma_us"),
        "byte_model": "window steps: M (8 d + c) + |I_n| c bytes per launch (FP64 nodes, values, grid once); "
                      "FFT passes: nonzero input + output of the pass",
        "valu_model": "(2m+2)^d (node, cell) pairs x 2 FMA slots / (256 CUs x 64 lanes x 2.4 GHz)",
        "mfma_model": "(2m+2)^d (node, cell) pairs x 4 flops / dense MFMA peak (FP64 78.6, FP32 157.3 TFLOP/s)",
    }
    out = {
        "metric": METRIC,
        "value": head["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "ms_per_step_cold": head["ms_per_step_cold"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": head["workload"],
            "d": 3, "N": list(N), "n": list(n), "M": M, "m": 6,
            "nodes": "4096 spokes x 512 points through the origin, directions uniform on the sphere",
            "precision": "complex128: FP64 data, window, accumulation, FFT and deconvolution",
        },
        "roofline": roofline,
        "kernels": per_kernel,
        "set_nodes_ms": head["set_nodes_ms"],
        "ms_per_step_with_events": head["ms_per_step_with_events"],
        "paper_context": PAPER_CONTEXT,
    }
    if check:
        t_cpu = refs.cpu_seconds_per_step()
        out["cpu_baseline"] = {
            "value": M / t_cpu,
            "unit": "points/s",
            "cores": refs.threads,
            "kind": "oracle",
            "sample": "headline workload: FP64 oracle NFFT + adjoint NFFT on %d host threads, deconvolution and FFT "
                      "steps at full size (%.2f s + %.2f s), interpolation and spreading on a 16384-node sample "
                      "(%.2f s + %.2f s) scaled by M/16384: %.1f s per step" %
                      (refs.threads, refs.t_grid, refs.t_coef, refs.t_interp, refs.t_spread, t_cpu),
            "host_cpu": host_cpu(),
        }
        out["e2_vs_oracle"] = {"trafo_16384_nodes_vs_oracle_nfft": head["e2_trafo_vs_oracle_16384_nodes"],
                               "adjoint_64_coefficients_vs_direct_sums": head["e2_adjoint_vs_ndft_64_coefficients"]}
    out["variants"] = [{k: v for k, v in r.items() if not k.startswith("_")} for r in variants]
    out["workloads"] = extra
    print(json.dumps(out))


if __name__ == "__main__":
    main()
