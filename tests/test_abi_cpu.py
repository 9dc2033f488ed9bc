"""Host-side checks of the C ABI: the library loads, exports every declared entry point,
and validates arguments and call order before enqueueing anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1810_09891_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nfft_mi355x.h")

OK, ARG, STATE, WS, HIP, UNSUP = 0, -1, -2, -3, -4, -5


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|char)\s*\**\s*(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def create(lib, N, M, n=None, m=8, dtype=1, flags=0):
    h = ctypes.c_void_p()
    d = len(N)
    Na = (ctypes.c_int64 * d)(*N)
    na = None if n is None else (ctypes.c_int64 * d)(*n)
    st = lib.nfft_plan_create(ctypes.byref(h), d, Na, M, na, m, dtype, flags)
    return st, h


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 20
    assert set(names) == set(_lib.ABI_SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in (OK, ARG, STATE, WS, HIP, UNSUP):
        assert lib.nfft_status_string(st)


@pytest.mark.parametrize(
    "N,M,n,m,expect",
    [
        ((8,), 10, None, 8, ARG),  # default n = 16 < 2m+2 = 18
        ((8,), 10, (16,), 7, OK),
        ((7,), 10, None, 2, ARG),  # odd N (Sec. 3.1: N in 2N^d)
        ((8,), 0, None, 2, ARG),  # M < 1
        ((8,), 10, (8,), 2, ARG),  # n <= N
        ((8,), 10, (11,), 2, ARG),  # odd n
        ((8,), 10, (12,), 2, OK),  # even, > N, not a power of two (mixed-radix passes)
        ((512,), 1024, (514,), 8, OK),  # n = 2 * 257 (Fig. 4.1's shortest grid)
        ((128, 128), 100, (130, 154), 8, OK),
        ((2000,), 10, (4094,), 6, OK),  # longest line with an odd factor
        ((8,), 10, (4098,), 2, UNSUP),  # longer than one workgroup line
        ((8,), 10, (8192,), 2, UNSUP),
        ((8,), 10, (64,), 13, UNSUP),  # m beyond the compiled stencils
        ((8,), 10, (16,), -1, ARG),
        ((8, 8, 8, 8), 10, None, 2, ARG),  # d > 3
        ((512, 512), 262144, None, 8, OK),
        ((128, 128, 128), 2097152, None, 6, OK),
    ],
)
def test_plan_validation(lib, N, M, n, m, expect):
    st, h = create(lib, N, M, n, m)
    assert st == expect
    if st == OK:
        assert lib.nfft_plan_destroy(h) == OK


@pytest.mark.parametrize(
    "N,n,m,dtype,expect",
    [
        ((16, 16, 16), (32, 32, 32), 8, 2, OK),  # one 21^3 complex128 tile (141 KiB) per workgroup
        ((16, 16, 16), (32, 32, 32), 12, 1, UNSUP),  # 29^3 complex64 tile exceeds the LDS
        ((2048,), (4096,), 12, 2, OK),  # longest line and widest stencil
        ((2048, 8), (4096, 32), 12, 1, OK),
        # 3-D: past complex128 m = 8 and complex64 m = 10 the smallest padded interpolation
        # tile no longer fits; grids that spread by output tiles (n_t multiples of 16) stage
        # it in slabs and take every m up to 12, other grids refuse
        ((32, 24, 32), (64, 48, 64), 9, 2, OK),
        ((32, 24, 32), (64, 48, 64), 12, 2, OK),
        ((32, 24, 32), (64, 48, 64), 12, 1, OK),
        ((20, 20, 20), (40, 40, 40), 8, 2, OK),
        ((20, 20, 20), (40, 40, 40), 9, 2, UNSUP),
        ((20, 20, 20), (40, 40, 40), 10, 1, OK),
        ((20, 20, 20), (40, 40, 40), 11, 1, UNSUP),
    ],
)
def test_lds_limits(lib, N, n, m, dtype, expect):
    """Plans whose smallest spreading tile does not fit the 160 KiB of LDS are refused."""
    st, h = create(lib, N, 100, n, m, dtype)
    assert st == expect
    if st == OK:
        assert lib.nfft_plan_destroy(h) == OK


def test_window_flags(lib):
    """One window flag at most; each selects its window (reported in the plan info)."""
    for flags, code in ((0, 0), (1 << 2, 1), (1 << 3, 2), (1 << 4, 3)):
        st, h = create(lib, (16, 16), 100, None, 4, 1, flags)
        assert st == OK
        info = _lib.PlanInfo()
        assert lib.nfft_plan_get_info(h, ctypes.byref(info)) == OK
        assert info.window == code
        assert lib.nfft_plan_destroy(h) == OK
    for flags in ((1 << 2) | (1 << 3), (1 << 3) | (1 << 4), (1 << 2) | (1 << 4)):
        st, h = create(lib, (16, 16), 100, None, 4, 1, flags)
        assert st == ARG


def test_defaults(lib):
    st, h = create(lib, (100, 64), 5, None, 0)
    assert st == OK
    info = _lib.PlanInfo()
    assert lib.nfft_plan_get_info(h, ctypes.byref(info)) == OK
    assert info.m == 8  # m = 0 selects the default 8 (Sec. 3.1)
    assert (info.n[0], info.n[1]) == (256, 128)  # 2^(ceil(log2 N)+1)
    lib.nfft_plan_destroy(h)


def test_call_order_and_workspace(lib):
    st, h = create(lib, (16, 16), 100, None, 4)
    assert st == OK
    nbytes = ctypes.c_size_t()
    assert lib.nfft_workspace_bytes(h, ctypes.byref(nbytes)) == OK
    assert nbytes.value > 0
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced on the host
    # no workspace yet
    flag = ctypes.c_int(-7)
    assert lib.nfft_set_nodes(h, fake, None) == WS
    assert lib.nfft_nodes_finite(h, ctypes.byref(flag), None) == WS
    assert lib.nfft_trafo(h, fake, fake, None) == WS
    # workspace too small / misaligned
    assert lib.nfft_set_workspace(h, fake, nbytes.value - 1) == WS
    assert lib.nfft_set_workspace(h, ctypes.c_void_p((1 << 20) + 8), nbytes.value) == WS
    assert lib.nfft_set_workspace(h, None, nbytes.value) == WS
    assert lib.nfft_set_workspace(h, fake, nbytes.value) == OK
    # nodes not set yet
    assert lib.nfft_trafo(h, fake, fake, None) == STATE
    assert lib.nfft_adjoint(h, fake, fake, None) == STATE
    assert lib.ndft_trafo(h, fake, fake, None) == STATE
    assert lib.nfft_step_interp(h, fake, fake, None) == STATE
    assert lib.nfft_step_spread(h, fake, fake, None) == STATE
    assert lib.nfft_grad_x(h, fake, fake, None) == STATE
    assert lib.nfft_nodes_finite(h, ctypes.byref(flag), None) == STATE
    assert flag.value == -7
    # null arguments
    assert lib.nfft_set_nodes(h, None, None) == ARG
    assert lib.nfft_nodes_finite(h, None, None) == ARG
    assert lib.nfft_nodes_finite(None, ctypes.byref(flag), None) == ARG
    assert lib.nfft_workspace_bytes(None, ctypes.byref(nbytes)) == ARG
    assert lib.nfft_plan_destroy(h) == OK


def test_null_plan_arguments(lib):
    fake = ctypes.c_void_p(1 << 20)
    for fn in ("nfft_trafo", "nfft_adjoint", "ndft_trafo", "ndft_adjoint", "nfft_grad_x"):
        assert getattr(lib, fn)(None, fake, fake, None) == ARG, fn
    st = lib.nfft_plan_create(None, 1, (ctypes.c_int64 * 1)(8), 4, None, 2, 1, 0)
    assert st == ARG
    assert lib.nfft_plan_create(ctypes.byref(ctypes.c_void_p()), 1, (ctypes.c_int64 * 1)(8), 4, None, 2, 3, 0) == ARG


def test_workspace_sizes_scale(lib):
    """Workspace grows with M and with the grid; complex128 needs more than complex64."""
    sizes = {}
    for dt in (1, 2):
        for M in (1000, 100000):
            st, h = create(lib, (64, 64), M, None, 4, dt)
            nb = ctypes.c_size_t()
            lib.nfft_workspace_bytes(h, ctypes.byref(nb))
            sizes[(dt, M)] = nb.value
            lib.nfft_plan_destroy(h)
    assert sizes[(1, 100000)] > sizes[(1, 1000)]
    assert sizes[(2, 1000)] > sizes[(1, 1000)]


def test_batch_create_validation(lib):
    """Batch creation is host-only: it checks its plans and lays out its own memory."""
    fake = ctypes.c_void_p(1 << 20)
    hs = []
    for N, m, dt in (((64, 64), 6, 1), ((32, 128), 6, 1), ((64, 64), 4, 1), ((128,), 6, 1), ((64, 64), 6, 2)):
        st, h = create(lib, N, 1000, None, m, dt)
        assert st == OK
        hs.append(h)
    P = ctypes.c_void_p
    arr = lambda *h: (P * len(h))(*[x.value for x in h])  # noqa: E731
    out = P()
    assert lib.nfft_batch_create(None, 1, arr(hs[0]), None) == ARG
    assert lib.nfft_batch_create(ctypes.byref(out), 0, arr(hs[0]), None) == ARG
    assert lib.nfft_batch_create(ctypes.byref(out), 1, None, None) == ARG
    # no workspace attached yet
    assert lib.nfft_batch_create(ctypes.byref(out), 2, arr(hs[0], hs[1]), None) == WS
    for h in hs:
        nb = ctypes.c_size_t()
        lib.nfft_workspace_bytes(h, ctypes.byref(nb))
        assert lib.nfft_set_workspace(h, fake, nb.value) == OK
    # mixed precision, repeated plan
    assert lib.nfft_batch_create(ctypes.byref(out), 2, arr(hs[0], hs[4]), None) == ARG
    assert lib.nfft_batch_create(ctypes.byref(out), 2, arr(hs[0], hs[0]), None) == ARG
    # four complex64 plans: d=2 width 14 (two plans), d=2 width 10, d=1 -> three launch groups
    assert lib.nfft_batch_create(ctypes.byref(out), 4, arr(*hs[:4]), None) == OK
    info = _lib.BatchInfo()
    assert lib.nfft_batch_get_info(out, ctypes.byref(info)) == OK
    assert (info.count, info.groups, info.tuned) == (4, 3, 0)
    assert info.workspace_bytes > 0
    params = (ctypes.c_int * 8)()
    cnt = ctypes.c_int()
    counts = []
    for g in range(3):
        assert lib.nfft_batch_get_params(out, g, params, ctypes.byref(cnt)) == OK
        counts.append(cnt.value)
        assert list(params)[:7] == [1, 0, 1, 0, 8, 8, 0]
    assert sorted(counts) == [1, 1, 2]
    assert lib.nfft_batch_get_params(out, 3, params, None) == ARG
    bad = (ctypes.c_int * 8)(3, 0, 1, 0, 8, 8, 0, 0)  # packing must be a power of two
    assert lib.nfft_batch_set_params(out, 0, bad) == ARG
    good = (ctypes.c_int * 8)(2, 4, 1, 0, 2, 2, 1, 0)
    assert lib.nfft_batch_set_params(out, 0, good) == OK  # no batch workspace yet: host only
    assert lib.nfft_batch_get_params(out, 0, params, None) == OK
    assert list(params) == list(good)
    # calls before the batch workspace is attached
    ptrs = (P * 4)(*([fake.value] * 4))
    assert lib.nfft_batch_trafo(out, ptrs, ptrs, None) == WS
    assert lib.nfft_batch_adjoint(out, ptrs, ptrs, None) == WS
    assert lib.nfft_batch_autotune(out, None) == WS
    assert lib.nfft_batch_set_workspace(out, fake, 0) == WS
    assert lib.nfft_batch_destroy(out) == OK
    assert lib.nfft_batch_destroy(None) == ARG
    for h in hs:
        lib.nfft_plan_destroy(h)


def test_fastsum_argument_checks(lib):
    fake = ctypes.c_void_p(1 << 20)
    assert lib.nfft_fastsum(None, None, fake, fake, fake, fake, None) == ARG
    st, h = create(lib, (16, 16), 100, None, 4)
    assert st == OK
    # no workspace / no nodes
    assert lib.nfft_fastsum(h, h, fake, fake, fake, fake, None) == WS
    nb = ctypes.c_size_t()
    lib.nfft_workspace_bytes(h, ctypes.byref(nb))
    assert lib.nfft_set_workspace(h, fake, nb.value) == OK
    assert lib.nfft_fastsum(h, h, fake, fake, fake, fake, None) == STATE
    assert lib.nfft_plan_destroy(h) == OK


def nn_create(lib, N, K, M, sigma=2.0, m=8, dtype=1, flags=0):
    h = ctypes.c_void_p()
    d = len(N)
    Na = (ctypes.c_int64 * d)(*N)
    st = lib.nnfft_plan_create(ctypes.byref(h), d, Na, K, M, sigma, m, dtype, flags)
    return st, h


@pytest.mark.parametrize("N,sigma,m", [((64,), 2.0, 8), ((30, 48), 2.0, 4), ((16, 10, 8), 1.5, 6), ((200,), 3.0, 2)])
def test_nnfft_plan_geometry(lib, N, sigma, m):
    # frequency grid N2: a power of two with sigma N + 2m + 4 points; N_A the smallest even
    # count for which sigma1 = N2 / N_A puts sigma1 [-N/2, N/2) and the stencils inside it
    st, h = nn_create(lib, N, 100, 120, sigma, m)
    assert st == OK
    info = _lib.NNPlanInfo()
    assert lib.nnfft_plan_get_info(h, ctypes.byref(info)) == OK
    assert (info.d, info.m, info.K, info.M) == (len(N), m, 100, 120)
    for t, Nt in enumerate(N):
        n2, na = info.N2[t], info.NA[t]
        assert n2 & (n2 - 1) == 0 and n2 >= -(-sigma * Nt // 1) + 2 * m + 4
        assert n2 // 2 < -(-sigma * Nt // 1) + 2 * m + 4  # smallest such power of two
        assert na % 2 == 0 and Nt < na < n2
        assert Nt * n2 <= na * (n2 - 2 * m - 4)
        assert (na - 2) * (n2 - 2 * m - 4) < Nt * n2
        assert info.sigma1[t] == pytest.approx(n2 / na)
    nbytes = ctypes.c_size_t()
    assert lib.nnfft_workspace_bytes(h, ctypes.byref(nbytes)) == OK
    assert nbytes.value == info.workspace_bytes > 0
    assert lib.nnfft_plan_destroy(h) == OK


@pytest.mark.parametrize("args,expect", [
    (((63,), 10, 10, 2.0, 8, 1, 0), ARG),            # odd bandwidth
    (((64,), 0, 10, 2.0, 8, 1, 0), ARG),             # no frequencies
    (((64,), 10, 0, 2.0, 8, 1, 0), ARG),             # no nodes
    (((64,), 10, 10, 1.0, 8, 1, 0), ARG),            # sigma must exceed 1
    (((64,), 10, 10, 2.0, -1, 1, 0), ARG),           # window size
    (((64,), 10, 10, 2.0, 8, 3, 0), ARG),            # dtype
    (((64,), 10, 10, 2.0, 8, 1, 1 << 1), ARG),       # NFFT_KEEP_GRID is not an NNFFT flag
    (((64,), 10, 10, 2.0, 8, 1, (1 << 2) | (1 << 3)), ARG),  # two windows
    (((1024,), 10, 10, 2.0, 8, 1, 0), UNSUP),        # N2 = 4096: plan B's FFT length 8192
])
def test_nnfft_plan_validation(lib, args, expect):
    st, h = nn_create(lib, *args)
    assert st == expect
    if st == OK:
        lib.nnfft_plan_destroy(h)


def test_nnfft_call_order(lib):
    st, h = nn_create(lib, (32, 32), 50, 60, 2.0, 4)
    assert st == OK
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced on the host
    nbytes = ctypes.c_size_t()
    assert lib.nnfft_workspace_bytes(h, ctypes.byref(nbytes)) == OK
    assert lib.nnfft_set_nodes(h, fake, fake, None) == WS
    assert lib.nnfft_trafo(h, fake, fake, None) == WS
    assert lib.nnfft_set_workspace(h, fake, nbytes.value - 1) == WS
    assert lib.nnfft_set_workspace(h, ctypes.c_void_p((1 << 20) + 8), nbytes.value) == WS
    assert lib.nnfft_set_workspace(h, fake, nbytes.value) == OK
    assert lib.nnfft_trafo(h, fake, fake, None) == STATE
    assert lib.nnfft_adjoint(h, fake, fake, None) == STATE
    assert lib.nnfft_set_nodes(h, None, fake, None) == ARG
    assert lib.nnfft_set_nodes(h, fake, None, None) == ARG
    assert lib.nnfft_trafo(h, None, fake, None) == ARG
    assert lib.nnfft_plan_get_info(h, None) == ARG
    assert lib.nnfft_plan_destroy(None) == ARG
    assert lib.nnfft_plan_destroy(h) == OK


@pytest.mark.parametrize("N,m", [((256,), 8), ((64, 16), 8), ((16,), 8), ((512, 100), 4)])
def test_nnfft_automatic_frequency_grid(lib, N, m):
    # sigma = 0: N2 the smallest power of two >= 2N, doubled while sigma1 < 1.5
    st, h = nn_create(lib, N, 10, 10, 0.0, m)
    assert st == OK
    info = _lib.NNPlanInfo()
    assert lib.nnfft_plan_get_info(h, ctypes.byref(info)) == OK
    for t, Nt in enumerate(N):
        n2, na = info.N2[t], info.NA[t]
        assert n2 & (n2 - 1) == 0 and n2 >= 2 * Nt
        assert n2 / na >= 1.5
        assert Nt * n2 <= na * (n2 - 2 * m - 4) and (na - 2) * (n2 - 2 * m - 4) < Nt * n2
        half = n2 // 2
        if half >= 2 * Nt and half > 2 * m + 4:
            a = -(-Nt * half // (half - 2 * m - 4))
            a += a & 1
            assert half / a < 1.5  # the smaller grid would not do
    lib.nnfft_plan_destroy(h)


def test_deterministic_flag_accepted(lib):
    """NFFT_DETERMINISTIC (always on) is accepted and reported back; the header states
    that only the tuning calls allocate device memory."""
    st, h = create(lib, (64, 64), 1000, None, 6, 1, _lib.NFFT_DETERMINISTIC | _lib.NFFT_KEEP_GRID)
    assert st == OK
    info = _lib.PlanInfo()
    assert lib.nfft_plan_get_info(h, ctypes.byref(info)) == OK
    assert info.flags & _lib.NFFT_DETERMINISTIC
    assert lib.nfft_plan_destroy(h) == OK
    txt = open(HEADER).read()
    assert "NFFT_DETERMINISTIC = 1u << 5" in txt
    assert "exceptions are the tuning calls nfft_batch_autotune and nfft_plan_tune" in txt.replace("\n *    ", " ")


def test_noalloc_batch_rejects_tables_beyond_the_static_scratch(lib):
    """nfft_batch_trafo_noalloc refuses, before any device work, a batch whose descriptor
    tables exceed its 1 MiB static array (here 1200 tiny plans)."""
    plans = []
    for _ in range(1200):
        st, h = create(lib, (8,), 10, (16,), 2)
        assert st == OK
        nbytes = ctypes.c_size_t()
        assert lib.nfft_workspace_bytes(h, ctypes.byref(nbytes)) == OK
        # a nominal 256-byte aligned address: nothing reads it before the size check
        assert lib.nfft_set_workspace(h, ctypes.c_void_p(1 << 20), nbytes.value) == OK
        plans.append(h)
    b = ctypes.c_void_p()
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    assert lib.nfft_batch_create(ctypes.byref(b), len(plans), arr, None) == OK
    info = _lib.BatchInfo()
    assert lib.nfft_batch_get_info(b, ctypes.byref(info)) == OK
    assert info.workspace_bytes > (1 << 20)
    ptrs = (ctypes.c_void_p * len(plans))(*([1] * len(plans)))
    assert lib.nfft_batch_trafo_noalloc(b, ptrs, ptrs, None) == WS
    assert lib.nfft_batch_destroy(b) == OK
    for h in plans:
        assert lib.nfft_plan_destroy(h) == OK


def create_params(lib, N, M, n, m, dtype, bins, cap):
    d = len(N)
    h = ctypes.c_void_p()
    Na = (ctypes.c_int64 * d)(*N)
    na = None if n is None else (ctypes.c_int64 * d)(*n)
    pp = _lib.PlanParams()
    for t in range(3):
        pp.bin[t] = bins[t] if t < len(bins) else 0
    pp.chunk_cap = cap
    st = lib.nfft_plan_create_params(ctypes.byref(h), d, Na, M, na, m, dtype, 0, ctypes.byref(pp))
    return st, h


@pytest.mark.parametrize(
    "N,n,m,dtype,bins,cap,expect",
    [
        ((64, 64), (128, 128), 6, 1, (16, 32), 256, OK),
        ((64, 64), (128, 128), 6, 1, (0,), 0, OK),  # defaults
        ((64, 64), (128, 128), 6, 1, (16, 24), 256, ARG),  # not a power of two
        ((64, 64), (128, 128), 6, 1, (256, 32), 256, ARG),  # longer than the grid
        ((64, 64), (128, 128), 6, 1, (16, 32), 48, ARG),  # cap not a power of two
        ((64, 64), (128, 128), 6, 1, (16, 32), 2048, ARG),  # cap past 1024
        ((64, 64), (128, 128), 6, 1, (128, 128), 256, UNSUP),  # tiles beyond the LDS
        ((32, 32, 32), (64, 64, 64), 6, 2, (4, 8, 8), 512, OK),
        ((256,), (514,), 8, 2, (256,), 128, OK),
    ],
)
def test_plan_params_validation(lib, N, n, m, dtype, bins, cap, expect):
    """nfft_plan_create_params takes the requested bin edges and work-item cap, reports them
    in the plan info, and refuses edges and caps outside the documented ranges."""
    st, h = create_params(lib, N, 1000, n, m, dtype, bins, cap)
    assert st == expect
    if st == OK:
        info = _lib.PlanInfo()
        assert lib.nfft_plan_get_info(h, ctypes.byref(info)) == OK
        if bins[0]:
            assert tuple(info.bin[t] for t in range(len(N))) == tuple(bins)
        if cap:
            assert info.chunk_cap == cap
        assert lib.nfft_plan_destroy(h) == OK


def test_plan_tune_rejects_missing_arguments(lib):
    """nfft_plan_tune needs nodes and an output (checked before any device work)."""
    Na = (ctypes.c_int64 * 2)(64, 64)
    out = _lib.PlanParams()
    assert lib.nfft_plan_tune(2, Na, 100, None, 6, 1, 0, None, None, None, ctypes.byref(out), None) == ARG
    assert lib.nfft_plan_tune(2, Na, 100, None, 6, 1, 0, ctypes.c_void_p(256), None, None, None, None) == ARG



def test_lin_psi_flag_reserves_its_tables(lib):
    """NFFT_PRE_LIN_PSI is accepted, reported, and its tables (2 (2m+2) 4097 reals per
    dimension) are part of the workspace."""
    sizes = []
    for flags in (0, _lib.NFFT_PRE_LIN_PSI):
        st, h = create(lib, (32, 32), 500, None, 6, 2, flags)
        assert st == OK
        info = _lib.PlanInfo()
        assert lib.nfft_plan_get_info(h, ctypes.byref(info)) == OK
        assert (info.flags & _lib.NFFT_PRE_LIN_PSI) == flags
        sizes.append(info.workspace_bytes)
        assert lib.nfft_plan_destroy(h) == OK
    assert sizes[1] - sizes[0] >= 2 * 2 * 14 * 4097 * 8
