"""Throughput of the NFFT forward + adjoint on one MI355X.

Workload: d = 2, N = (512, 512), n = (1024, 1024) (sigma = 2), M = 262144 nodes uniform on
[-1/2, 1/2)^2, complex Gaussian data, Kaiser-Bessel window.  The headline line is the
complex64 plan with m = 8; complex128 and m = 4 variants are reported beside it.

A step is one nfft_trafo plus one nfft_adjoint of the whole node set (inputs resident in
device memory; the node precomputation is timed separately, as Sec. 4 of the paper does).
value = M / (time of one step) in nonuniform points per second.

The dominant kernel is timed with HIP events recorded around every kernel launch on the
stream the library launches on (a second, event-bracketed pass of the same steps).  Its
algorithmic bytes per launch (nodes, values and grid read or written once) over that time
give the HBM roofline fraction.  The CPU baseline is the FP64 oracle (serial NFFT, one
core) on the same workload; it also provides the reference for the E_2 errors.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--graph] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NFFT fwd+adj nonuniform points/s at stated rel-ℓ2 error; % HBM roofline"
HBM_PEAK_GBS = 8000.0
FETCH_WRITE_FILE = os.path.join(ROOT, "profiles", "traffic_d2_512.json")


def algorithmic_bytes(name, d, N, n, M, cbytes):
    """Bytes a kernel must move at least once (per launch) for this plan.

    Per node: the grid index and offset (8 bytes per dimension: int32 index + float32
    offset, or int32 + float64 in complex128 where this counts 12), the permutation entry
    (4 bytes) and the value (cbytes).  Grid, coefficient and line data: cbytes per entry."""
    import numpy as np

    per_node = d * (4 + cbytes // 2) + 4 + cbytes
    grid = int(np.prod(n)) * cbytes
    coef = int(np.prod(N)) * cbytes
    rows_after_pass1 = int(np.prod(N[:-1])) * n[-1] * cbytes
    if name == "interp" or name == "grad_x":
        return M * per_node + grid
    if name == "spread_tiles":
        return M * per_node
    if name == "spread_fold":
        return grid
    if name == "fft_fwd_deconv":
        return coef + rows_after_pass1
    if name == "fft_fwd":
        return rows_after_pass1 + grid
    if name == "fft_adj":
        return grid + rows_after_pass1
    if name == "fft_adj_deconv":
        return rows_after_pass1 + coef
    return None


class Case:
    def __init__(self, w, m, dtype, torch):
        from paper_1810_09891_amd import Plan

        self.w = w
        self.m = m
        self.dtype = dtype
        self.torch = torch
        dev = torch.device("cuda:0")
        self.plan = Plan(w["N"], w["M"], m=m, dtype=dtype, device=dev)
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

    def time_steps(self, steps, warmup):
        torch = self.torch
        self.run(warmup)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        self.run(steps)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def kernel_times(self, steps):
        """Average duration per launch of every kernel, from HIP events the library
        records around each launch on its stream."""
        torch = self.torch
        self.plan.profile(True)
        self.plan.profile_read()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        res = self.plan.profile_read()
        self.plan.profile(False)
        return {k: (v[0] / v[1], v[1]) for k, v in res.items()}

    def outputs(self):
        torch = self.torch
        self.step()
        torch.cuda.synchronize()
        return self.out_f.cpu().numpy(), self.out_h.cpu().numpy()


def cpu_baseline(w, m, reps):
    """Serial FP64 oracle NFFT + adjoint on the full workload (one core)."""
    import numpy as np

    from oracle import oracle as O

    times = []
    f_ref = h_ref = None
    for _ in range(reps):
        t0 = time.perf_counter()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--graph", action="store_true", help="replay the step as a captured HIP graph")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and E_2")
    ap.add_argument("--primary-only", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md for how "
              "the transform would shard); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1810_09891_amd import workloads as W

    C64, C128 = torch.complex64, torch.complex128
    variants = [(8, C64)] + ([] if args.primary_only else [(8, C128), (4, C64), (4, C128)])
    results = []
    cpu = {}
    for i, (m, dtype) in enumerate(variants):
        w = W.workload("d2", m=m)
        case = Case(w, m, dtype, torch)
        t_nodes = case.set_nodes_ms()
        if args.graph:
            case.capture()
        steps = args.steps if i == 0 else max(10, args.steps // 4)
        ms = case.time_steps(steps, args.warmup)
        kt = case.kernel_times(steps)
        f_gpu, h_gpu = case.outputs()
        r = {
            "m": m,
            "dtype": "c64" if dtype == C64 else "c128",
            "ms_per_step": ms,
            "points_per_s": w["M"] / (ms * 1e-3),
            "set_nodes_ms": t_nodes,
            "kernels_ms": {k: round(v[0], 5) for k, v in sorted(kt.items())},
            "steps": steps,
        }
        if not args.no_cpu:
            if m not in cpu:
                cpu[m] = cpu_baseline(w, m, reps=1 if cpu else 3)
            r["e2_trafo_vs_oracle"] = e2(cpu[m]["f"], f_gpu)
            r["e2_adjoint_vs_oracle"] = e2(cpu[m]["h"], h_gpu)
        r["_kernel_avg"] = kt
        r["_w"] = (w["N"], w["n"], w["M"])
        results.append(r)
        print("[bench] %s m=%d: %.4f ms/step, %.3e points/s, set_nodes %.3f ms" %
              (r["dtype"], m, ms, r["points_per_s"], t_nodes), file=sys.stderr, flush=True)
        del case
        torch.cuda.empty_cache()

    prim = results[0]
    N, n, M = prim["_w"]
    cb = 8
    # dominant kernel of the primary plan
    kt = prim["_kernel_avg"]
    dom = max((k for k in kt if not k.startswith("nodes")), key=lambda k: kt[k][0])
    dom_ms = kt[dom][0]
    alg = algorithmic_bytes(dom, 2, N, n, M, cb)
    achieved = alg / (dom_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(FETCH_WRITE_FILE):
        try:
            tr = json.load(open(FETCH_WRITE_FILE))
            if tr.get("kernel") == dom and tr.get("source_hash") == tr.get("source_hash"):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes": alg,
        "avg_launch_ms": round(dom_ms, 5),
    }
    per_kernel = {}
    for k, (avg, cnt) in sorted(kt.items()):
        b = algorithmic_bytes(k, 2, N, n, M, cb)
        per_kernel[k] = {"avg_ms": round(avg, 5), "launches": cnt,
                         "algorithmic_bytes": b,
                         "hbm_frac": None if b is None else round(b / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC,
        "value": prim["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": prim["steps"],
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "d=2 N=(512,512) n=(1024,1024) M=262144 uniform nodes, Kaiser-Bessel m=8, complex64, fwd+adj",
            "d": 2, "N": list(N), "n": list(n), "M": M, "m": 8, "precision": "complex64 data, FP32 window and "
            "accumulation, FP64 node index and deconvolution table",
            "graph": bool(args.graph),
        },
        "roofline": roofline,
        "kernels": per_kernel,
        "set_nodes_ms": prim["set_nodes_ms"],
    }
    if not args.no_cpu:
        c = cpu[8]
        import multiprocessing

        out["cpu_baseline"] = {
            "value": M / c["seconds_per_step"],
            "unit": "points/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "full workload (d=2, N=512^2, M=262144, m=8), serial FP64 NFFT + adjoint NFFT of the "
                      "oracle, median of %d runs, %.2f s per step; host has %d cores" %
                      (c["runs"], c["seconds_per_step"], multiprocessing.cpu_count()),
        }
        out["e2_vs_oracle"] = {"trafo": prim["e2_trafo_vs_oracle"], "adjoint": prim["e2_adjoint_vs_oracle"]}
    out["variants"] = [{k: v for k, v in r.items() if not k.startswith("_")} for r in results[1:]]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
