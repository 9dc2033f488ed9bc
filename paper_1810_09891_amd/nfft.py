"""Python front end of the HIP NFFT library (argument marshalling only).

``Plan`` mirrors the plan interface of arXiv:1810.09891 Sec. 3 (Table 3.1, the
constructors ``Plan(N, M)`` / ``Plan(N, M, n, m, ...)``, ``p.x = ...``,
``NFFT.trafo(p)``): create a plan, set its nodes (which runs the node
precomputation), then call ``trafo`` / ``adjoint`` as often as needed.  PyTorch only
provides device memory (tensors, including the plan's workspace) and the stream the
library enqueues on.
"""
import ctypes
import os

import torch

from . import _lib
from ._lib import NFFT_C64, NFFT_C128, NFFT_KEEP_GRID, NFFT_SORT_NODES, check

_CDTYPE = {torch.complex64: NFFT_C64, torch.complex128: NFFT_C128}
_RDTYPE = {torch.complex64: torch.float32, torch.complex128: torch.float64}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def default_n(N):
    """n_t = 2^(ceil(log2 N_t) + 1), the default FFT length (Sec. 2 and Sec. 3.1)."""
    out = []
    for v in N:
        e = 0
        while (1 << e) < v:
            e += 1
        out.append(1 << (e + 1))
    return tuple(out)


def _plan_params(params):
    """nfft_plan_params from a dict {"bin": (B0[, B1[, B2]]), "chunk_cap": C} (missing: 0)."""
    pp = _lib.PlanParams()
    b = tuple(params.get("bin", ())) + (0, 0, 0)
    for t in range(3):
        pp.bin[t] = int(b[t]) if b[0] else 0
    pp.chunk_cap = int(params.get("chunk_cap", 0))
    return pp


def tune_plan_params(N, M, x, n=None, m=8, dtype=torch.complex64, flags=0, window="kaiser-bessel", cache=None):
    """Measured bin edges and work-item cap for this plan shape and node set (nfft_plan_tune).

    x: (M, d) float64 device tensor.  Returns ({"bin": (...), "chunk_cap": C}, ms) where ms is
    the measured time of one trafo + adjoint pair with them (0.0 when read from `cache`).
    Allocates temporary device memory; synchronises the current stream."""
    lib = _lib.load()
    if window not in _lib.WINDOW_FLAGS:
        raise ValueError("window must be one of %s" % sorted(_lib.WINDOW_FLAGS))
    N = tuple(int(v) for v in N)
    d = len(N)
    if x.dtype != torch.float64 or not x.is_cuda or tuple(x.shape) != (int(M), d):
        raise ValueError("x must be a (M, d) float64 device tensor")
    x = x.contiguous()
    Na = (ctypes.c_int64 * d)(*N)
    na = None if n is None else (ctypes.c_int64 * d)(*[int(v) for v in n])
    out = _lib.PlanParams()
    ms = ctypes.c_double(0.0)
    check(lib.nfft_plan_tune(d, Na, int(M), na, int(m), _CDTYPE[dtype], int(flags) | _lib.WINDOW_FLAGS[window],
                             _ptr(x), None if cache is None else os.fsencode(cache), _stream(x.device),
                             ctypes.byref(out), ctypes.byref(ms)), "nfft_plan_tune")
    return {"bin": tuple(int(out.bin[t]) for t in range(d)), "chunk_cap": int(out.chunk_cap)}, float(ms.value)


class Plan:
    """NFFT plan for d-variate transforms with bandwidths N, M nodes, FFT lengths n and
    window size m, computing in complex64 or complex128, with the Kaiser-Bessel window
    (default) or the Gaussian window.

    Arrays: coefficients have shape N (centred: index i holds k = i - N/2), nodes are
    (M, d) float64, values are (M,).  All tensors live on ``device``.
    """

    def __init__(self, N, M, n=None, m=8, dtype=torch.complex64, flags=0, device="cuda", window="kaiser-bessel",
                 params=None):
        lib = _lib.load()
        if window not in _lib.WINDOW_FLAGS:
            raise ValueError("window must be one of %s" % sorted(_lib.WINDOW_FLAGS))
        flags = int(flags) | _lib.WINDOW_FLAGS[window]
        self.N = tuple(int(v) for v in N)
        self.d = len(self.N)
        self.M = int(M)
        self.dtype = dtype
        if dtype not in _CDTYPE:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.device = torch.device(device)
        Na = (ctypes.c_int64 * self.d)(*self.N)
        na = None if n is None else (ctypes.c_int64 * self.d)(*[int(v) for v in n])
        h = ctypes.c_void_p()
        if params is None:
            check(lib.nfft_plan_create(ctypes.byref(h), self.d, Na, self.M, na, int(m), _CDTYPE[dtype], int(flags)),
                  "nfft_plan_create")
        else:
            pp = _plan_params(params)
            check(lib.nfft_plan_create_params(ctypes.byref(h), self.d, Na, self.M, na, int(m), _CDTYPE[dtype],
                                              int(flags), ctypes.byref(pp)), "nfft_plan_create_params")
        self._h = h
        self._lib = lib
        info = _lib.PlanInfo()
        check(lib.nfft_plan_get_info(h, ctypes.byref(info)), "nfft_plan_get_info")
        self.info = info
        self.n = tuple(int(info.n[t]) for t in range(self.d))
        self.m = int(info.m)
        self.flags = int(info.flags)
        self.window = window
        self.workspace = None
        self._x = None
        self.nodes_set = False
        self.nodes_version = None
        self.generation = 0  # counts calls that rewrite the plan's forward grid
        self.node_generation = 0  # counts node sets

    # ---------------------------------------------------------------- set-up

    def allocate(self):
        """Allocate and attach the workspace (a uint8 tensor on the plan's device)."""
        nbytes = ctypes.c_size_t()
        check(self._lib.nfft_workspace_bytes(self._h, ctypes.byref(nbytes)), "nfft_workspace_bytes")
        ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        check(self._lib.nfft_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr() + off), nbytes.value),
              "nfft_set_workspace")
        return self

    @property
    def workspace_bytes(self):
        return int(self.info.workspace_bytes)

    def set_nodes(self, x):
        """Set the nodes x, an (M, d) float64 tensor, and run the node precomputation."""
        if self.workspace is None:
            self.allocate()
        x = self._as(x, torch.float64, (self.M, self.d), "x")
        check(self._lib.nfft_set_nodes(self._h, _ptr(x), _stream(self.device)), "nfft_set_nodes")
        self._x = x  # kept alive until the enqueued work has read it
        self.nodes_set = True
        self.nodes_version = x._version
        self.generation += 1
        self.node_generation += 1
        return self

    def nodes_finite(self):
        """True if every coordinate of the last set_nodes was finite (waits for the stream)."""
        flag = ctypes.c_int(0)
        check(self._lib.nfft_nodes_finite(self._h, ctypes.byref(flag), _stream(self.device)), "nfft_nodes_finite")
        return bool(flag.value)

    # ---------------------------------------------------------------- transforms

    def _as(self, t, dtype, shape, name):
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype)
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t.contiguous()

    def _out(self, out, shape, dtype=None):
        dtype = self.dtype if dtype is None else dtype
        if out is None:
            return torch.empty(shape, dtype=dtype, device=self.device)
        if out.dtype != dtype or tuple(out.shape) != tuple(shape) or not out.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (dtype, shape))
        return out

    def trafo(self, fhat, out=None):
        """NFFT (Algorithm 2.1): f_j ~ sum_k fhat_k exp(-2 pi i k.x_j)."""
        fhat = self._as(fhat, self.dtype, self.N, "fhat")
        f = self._out(out, (self.M,))
        check(self._lib.nfft_trafo(self._h, _ptr(fhat), _ptr(f), _stream(self.device)), "nfft_trafo")
        self.generation += 1
        return f

    def adjoint(self, f, out=None):
        """Adjoint NFFT (Algorithm 2.2): hhat_k ~ sum_j f_j exp(+2 pi i k.x_j)."""
        f = self._as(f, self.dtype, (self.M,), "f")
        h = self._out(out, self.N)
        check(self._lib.nfft_adjoint(self._h, _ptr(f), _ptr(h), _stream(self.device)), "nfft_adjoint")
        return h

    def ndft_trafo(self, fhat, out=None):
        """Direct sum eq. (1.2) on the device."""
        fhat = self._as(fhat, self.dtype, self.N, "fhat")
        f = self._out(out, (self.M,))
        check(self._lib.ndft_trafo(self._h, _ptr(fhat), _ptr(f), _stream(self.device)), "ndft_trafo")
        return f

    def ndft_adjoint(self, f, out=None):
        """Direct sum eq. (1.3) on the device."""
        f = self._as(f, self.dtype, (self.M,), "f")
        h = self._out(out, self.N)
        check(self._lib.ndft_adjoint(self._h, _ptr(f), _ptr(h), _stream(self.device)), "ndft_adjoint")
        return h

    def grad_x(self, v, out=None):
        """Re(conj(v_j) d f_j / d x_{j,t}) for the last trafo (needs NFFT_KEEP_GRID)."""
        v = self._as(v, self.dtype, (self.M,), "v")
        g = self._out(out, (self.M, self.d), _RDTYPE[self.dtype])
        check(self._lib.nfft_grad_x(self._h, _ptr(v), _ptr(g), _stream(self.device)), "nfft_grad_x")
        return g

    # ---------------------------------------------------------------- single steps

    def step_grid(self, fhat, out=None):
        fhat = self._as(fhat, self.dtype, self.N, "fhat")
        g = self._out(out, self.n)
        if self.workspace is None:
            self.allocate()
        check(self._lib.nfft_step_grid(self._h, _ptr(fhat), _ptr(g), _stream(self.device)), "nfft_step_grid")
        return g

    def step_interp(self, g, out=None):
        g = self._as(g, self.dtype, self.n, "g")
        f = self._out(out, (self.M,))
        check(self._lib.nfft_step_interp(self._h, _ptr(g), _ptr(f), _stream(self.device)), "nfft_step_interp")
        return f

    def step_spread(self, f, out=None):
        f = self._as(f, self.dtype, (self.M,), "f")
        g = self._out(out, self.n)
        check(self._lib.nfft_step_spread(self._h, _ptr(f), _ptr(g), _stream(self.device)), "nfft_step_spread")
        return g

    def step_coeffs(self, g, out=None):
        g = self._as(g, self.dtype, self.n, "g")
        h = self._out(out, self.N)
        if self.workspace is None:
            self.allocate()
        check(self._lib.nfft_step_coeffs(self._h, _ptr(g), _ptr(h), _stream(self.device)), "nfft_step_coeffs")
        return h

    # ---------------------------------------------------------------- timing

    def profile(self, on=True):
        check(self._lib.nfft_profile_enable(self._h, 1 if on else 0), "nfft_profile_enable")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last read (synchronise first)."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        count = ctypes.c_int()
        check(self._lib.nfft_profile_read(self._h, names, ms, cnt, cap, ctypes.byref(count)), "nfft_profile_read")
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(cap, count.value))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nfft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NNPlan:
    """NNFFT plan: nonequispaced nodes in both domains (the generalisation named in Sec. 1).

    ``trafo`` computes f_j = sum_k fhat_k exp(-2 pi i v_k.x_j) for K frequencies v (K, d)
    with v_{k,t} in [-N_t/2, N_t/2) and M nodes x (M, d) in [-1/2, 1/2)^d; ``adjoint``
    computes hhat_k = sum_j f_j exp(+2 pi i v_k.x_j).  ``sigma`` is the oversampling of the
    frequency grid the frequencies are spread onto (None: chosen by the library), ``m`` the
    window size of both inner NFFT plans.  All tensors live on ``device``.
    """

    def __init__(self, N, K, M, sigma=None, m=8, dtype=torch.complex64, device="cuda", window="kaiser-bessel"):
        lib = _lib.load()
        if window not in _lib.WINDOW_FLAGS:
            raise ValueError("window must be one of %s" % sorted(_lib.WINDOW_FLAGS))
        if dtype not in _CDTYPE:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.N = tuple(int(v) for v in N)
        self.d = len(self.N)
        self.K = int(K)
        self.M = int(M)
        self.dtype = dtype
        self.window = window
        self.device = torch.device(device)
        Na = (ctypes.c_int64 * self.d)(*self.N)
        h = ctypes.c_void_p()
        check(lib.nnfft_plan_create(ctypes.byref(h), self.d, Na, self.K, self.M, float(sigma or 0.0), int(m),
                                    _CDTYPE[dtype], int(_lib.WINDOW_FLAGS[window])), "nnfft_plan_create")
        self._h = h
        self._lib = lib
        info = _lib.NNPlanInfo()
        check(lib.nnfft_plan_get_info(h, ctypes.byref(info)), "nnfft_plan_get_info")
        self.info = info
        self.m = int(info.m)
        self.N2 = tuple(int(info.N2[t]) for t in range(self.d))
        self.NA = tuple(int(info.NA[t]) for t in range(self.d))
        self.sigma1 = tuple(float(info.sigma1[t]) for t in range(self.d))
        self.workspace = None
        self._keep = None

    def allocate(self):
        nbytes = ctypes.c_size_t()
        check(self._lib.nnfft_workspace_bytes(self._h, ctypes.byref(nbytes)), "nnfft_workspace_bytes")
        ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        check(self._lib.nnfft_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr() + off), nbytes.value),
              "nnfft_set_workspace")
        return self

    def _as(self, t, dtype, shape):
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype)
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t.contiguous()

    def set_nodes(self, x, v):
        """Nodes x (M, d) and frequencies v (K, d), float64."""
        if self.workspace is None:
            self.allocate()
        x = self._as(x, torch.float64, (self.M, self.d))
        v = self._as(v, torch.float64, (self.K, self.d))
        check(self._lib.nnfft_set_nodes(self._h, _ptr(x), _ptr(v), _stream(self.device)), "nnfft_set_nodes")
        self._keep = (x, v)  # alive until the enqueued work has read them
        return self

    def trafo(self, fhat, out=None):
        fhat = self._as(fhat, self.dtype, (self.K,))
        f = out if out is not None else torch.empty(self.M, dtype=self.dtype, device=self.device)
        check(self._lib.nnfft_trafo(self._h, _ptr(fhat), _ptr(f), _stream(self.device)), "nnfft_trafo")
        return f

    def adjoint(self, f, out=None):
        f = self._as(f, self.dtype, (self.M,))
        h = out if out is not None else torch.empty(self.K, dtype=self.dtype, device=self.device)
        check(self._lib.nnfft_adjoint(self._h, _ptr(f), _ptr(h), _stream(self.device)), "nnfft_adjoint")
        return h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nnfft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many plans run together: ``trafo`` / ``adjoint`` take and return lists in the order of
    ``plans`` and launch each step kind once for all of them.  Every plan needs its nodes
    set (``Plan.set_nodes``) before the first call; ``autotune`` picks the launch shapes
    (cached in ``tune_cache`` when given)."""

    def __init__(self, plans, tune_cache=None):
        lib = _lib.load()
        self._lib = lib
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("a batch needs at least one plan")
        self.device = self.plans[0].device
        for p in self.plans:
            if p.workspace is None:
                p.allocate()
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        cache = None if tune_cache is None else str(tune_cache).encode()
        check(lib.nfft_batch_create(ctypes.byref(h), len(self.plans), arr, cache), "nfft_batch_create")
        self._h = h
        info = _lib.BatchInfo()
        check(lib.nfft_batch_get_info(h, ctypes.byref(info)), "nfft_batch_get_info")
        nbytes = int(info.workspace_bytes)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        check(lib.nfft_batch_set_workspace(h, ctypes.c_void_p(ws.data_ptr() + off), nbytes),
              "nfft_batch_set_workspace")

    @property
    def info(self):
        info = _lib.BatchInfo()
        check(self._lib.nfft_batch_get_info(self._h, ctypes.byref(info)), "nfft_batch_get_info")
        return info

    def params(self, group):
        """Launch parameters of launch group ``group`` as a dict (see the C header)."""
        v = (ctypes.c_int * _lib.NFFT_BATCH_NPARAMS)()
        cnt = ctypes.c_int()
        check(self._lib.nfft_batch_get_params(self._h, int(group), v, ctypes.byref(cnt)), "nfft_batch_get_params")
        out = dict(zip(_lib.BATCH_PARAM_NAMES, list(v)))
        out["plans"] = cnt.value
        return out

    def set_params(self, group, **kw):
        cur = self.params(group)
        v = (ctypes.c_int * _lib.NFFT_BATCH_NPARAMS)(*[int(kw.get(k, cur[k])) for k in _lib.BATCH_PARAM_NAMES])
        check(self._lib.nfft_batch_set_params(self._h, int(group), v), "nfft_batch_set_params")

    def autotune(self):
        check(self._lib.nfft_batch_autotune(self._h, _stream(self.device)), "nfft_batch_autotune")
        return [self.params(g) for g in range(self.info.groups)]

    def _io(self, ins, outs, in_shape, out_shape):
        if len(ins) != len(self.plans):
            raise ValueError("expected %d arrays" % len(self.plans))
        ins = [p._as(a, p.dtype, in_shape(p), "in") for p, a in zip(self.plans, ins)]
        if outs is None:
            outs = [p._out(None, out_shape(p)) for p in self.plans]
        else:
            outs = [p._out(o, out_shape(p)) for p, o in zip(self.plans, outs)]
        n = len(self.plans)
        ip = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ins])
        op = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
        return ins, outs, ip, op

    def trafo(self, fhats, outs=None):
        fhats, outs, ip, op = self._io(fhats, outs, lambda p: p.N, lambda p: (p.M,))
        check(self._lib.nfft_batch_trafo(self._h, ip, op, _stream(self.device)), "nfft_batch_trafo")
        for p in self.plans:
            p.generation += 1
        self._keep = fhats  # alive until the enqueued work has read them
        return outs

    def trafo_noalloc(self, fhats, outs):
        """``trafo`` through nfft_batch_trafo_noalloc: no batch workspace and no allocation in
        the call (the outputs are given)."""
        fhats, outs, ip, op = self._io(fhats, outs, lambda p: p.N, lambda p: (p.M,))
        check(self._lib.nfft_batch_trafo_noalloc(self._h, ip, op, _stream(self.device)),
              "nfft_batch_trafo_noalloc")
        for p in self.plans:
            p.generation += 1
        self._keep = fhats
        return outs

    def adjoint(self, fs, outs=None):
        fs, outs, ip, op = self._io(fs, outs, lambda p: (p.M,), lambda p: p.N)
        check(self._lib.nfft_batch_adjoint(self._h, ip, op, _stream(self.device)), "nfft_batch_adjoint")
        self._keep = fs
        return outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.nfft_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fastsum(px, py, bhat, alpha, out=None):
    """Kernel sums g_j = sum_l alpha_l K(y_j - x_l) for K(z) = sum_k bhat_k e^{-2 pi i k.z}
    (nfft_fastsum): x are the nodes of plan px, y those of plan py (px may be py)."""
    if px.N != py.N or px.dtype != py.dtype:
        raise ValueError("plans must have equal N and dtype")
    bhat = px._as(bhat, px.dtype, px.N, "bhat")
    alpha = px._as(alpha, px.dtype, (px.M,), "alpha")
    g = py._out(out, (py.M,))
    work = torch.empty(px.N, dtype=px.dtype, device=px.device)
    check(px._lib.nfft_fastsum(px._h, py._h, _ptr(bhat), _ptr(alpha), _ptr(g), _ptr(work), _stream(px.device)),
          "nfft_fastsum")
    if px is not py:
        px.generation += 1
    py.generation += 1
    px._keep = (bhat, alpha, work)  # alive until the enqueued work has read them
    return g


def gaussian_coefficients(N, c, dtype=torch.complex128, device="cuda"):
    """Fourier coefficients on I_N of the 1-periodised Gaussian exp(-|z|^2 / c^2):
    bhat_k = (c sqrt(pi))^d exp(-pi^2 c^2 |k|^2) (centred row-major), a kernel for
    ``fastsum``; for c well below 1/2 the periodisation is the Gaussian itself near 0."""
    import math

    grids = torch.meshgrid(*[torch.arange(-n // 2, n // 2, dtype=torch.float64) for n in N], indexing="ij")
    k2 = sum(g * g for g in grids)
    b = (c * math.sqrt(math.pi)) ** len(N) * torch.exp(-(math.pi ** 2) * c * c * k2)
    return b.to(device=device, dtype=dtype)
