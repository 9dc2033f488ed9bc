"""ctypes front end of the C oracle in ``nfft_oracle.c`` (test infrastructure only).

Every routine takes and returns numpy arrays:

* nodes ``x``: float64, shape (M, d), row-major;
* coefficients ``fhat``: complex128, shape ``N`` (centred: position i holds k = i - N/2);
* node values ``f``: complex128, shape (M,);
* oversampled grid ``g``: complex128, shape ``n`` (position l holds index l mod n).

The functions follow Algorithm 2.1 / 2.2 and eq. (1.2) / (1.3) of arXiv:1810.09891;
the C source documents each step and the readings of the paper it takes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "nfft_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force=False):
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L = ctypes.c_long
        Ii = ctypes.c_int
        D = ctypes.c_double
        sig = {
            "or_bessel_i0": (D, [D]),
            "or_kb_b": (D, [L, L]),
            "or_kb_phi": (D, [D, Ii, D]),
            "or_kb_dphi": (D, [D, Ii, D]),
            "or_kb_phihat": (D, [L, L, Ii, D]),
            "or_gauss_b": (D, [L, L, Ii]),
            "or_gauss_phi": (D, [D, D]),
            "or_gauss_dphi": (D, [D, D]),
            "or_gauss_phihat": (D, [L, L, D]),
            "or_bspline_n": (D, [Ii, D]),
            "or_bspline_phi": (D, [D, Ii]),
            "or_bspline_dphi": (D, [D, Ii]),
            "or_bspline_phihat": (D, [L, L, Ii]),
            "or_sinc_a": (D, [L, L, Ii]),
            "or_sinc_phi": (D, [D, Ii, D]),
            "or_sinc_dphi": (D, [D, Ii, D]),
            "or_sinc_phihat": (D, [L, L, Ii, D]),
            "or_set_window": (None, [Ii]),
            "or_get_window": (Ii, []),
            "or_dft_naive": (None, [P, P, L, Ii]),
            "or_fft_1d": (None, [P, L, Ii]),
            "or_fft_d": (None, [Ii, P, P, Ii]),
            "or_ndft_trafo": (None, [Ii, P, L, P, P, P]),
            "or_ndft_adjoint": (None, [Ii, P, L, P, P, P]),
            "or_ndft_grad_x": (None, [Ii, P, L, P, P, P, P]),
            "or_nndft_trafo": (None, [Ii, L, L, P, P, P, P]),
            "or_nndft_adjoint": (None, [Ii, L, L, P, P, P, P]),
            "or_ndft_adjoint_at": (None, [Ii, P, L, P, P, L, P, P]),
            "or_nfft_deconv": (None, [Ii, P, P, Ii, P, P]),
            "or_nfft_deconv_adj": (None, [Ii, P, P, Ii, P, P]),
            "or_nfft_interp": (None, [Ii, P, P, Ii, L, P, P, P]),
            "or_nfft_spread": (None, [Ii, P, P, Ii, L, P, P, P]),
            "or_nfft_interp_dx": (None, [Ii, P, P, Ii, L, P, P, P]),
            "or_nfft_trafo": (None, [Ii, P, P, Ii, L, P, P, P]),
            "or_nfft_adjoint": (None, [Ii, P, P, Ii, L, P, P, P]),
            "or_nfft_grid": (None, [Ii, P, P, Ii, P, P]),
            "or_nfft_adjoint_from_grid": (None, [Ii, P, P, Ii, P, P]),
            "or_err_l2": (D, [P, P, L]),
            "or_err_inf": (D, [P, P, L, D]),
            "or_set_threads": (None, [Ii]),
            "or_get_threads": (Ii, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(-1))
    assert v.dtype.itemsize == ctypes.sizeof(ctypes.c_long)
    return v


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(nt):
    _load().or_set_threads(int(nt))


def get_threads():
    return int(_load().or_get_threads())


def bessel_i0(x):
    return _load().or_bessel_i0(float(x))


def kb_b(N, n):
    return _load().or_kb_b(int(N), int(n))


def kb_phi(z, m, b):
    return _load().or_kb_phi(float(z), int(m), float(b))


def kb_dphi(z, m, b):
    return _load().or_kb_dphi(float(z), int(m), float(b))


def kb_phihat(k, n, m, b):
    return _load().or_kb_phihat(int(k), int(n), int(m), float(b))


def gauss_b(N, n, m):
    return _load().or_gauss_b(int(N), int(n), int(m))


def gauss_phi(z, b):
    return _load().or_gauss_phi(float(z), float(b))


def gauss_dphi(z, b):
    return _load().or_gauss_dphi(float(z), float(b))


def gauss_phihat(k, n, b):
    return _load().or_gauss_phihat(int(k), int(n), float(b))


def bspline_n(k, x):
    return _load().or_bspline_n(int(k), float(x))


def bspline_phi(z, m):
    return _load().or_bspline_phi(float(z), int(m))


def bspline_dphi(z, m):
    return _load().or_bspline_dphi(float(z), int(m))


def bspline_phihat(k, n, m):
    return _load().or_bspline_phihat(int(k), int(n), int(m))


def sinc_a(N, n, m):
    return _load().or_sinc_a(int(N), int(n), int(m))


def sinc_phi(z, m, a):
    return _load().or_sinc_phi(float(z), int(m), float(a))


def sinc_dphi(z, m, a):
    return _load().or_sinc_dphi(float(z), int(m), float(a))


def sinc_phihat(k, n, m, a):
    return _load().or_sinc_phihat(int(k), int(n), int(m), float(a))


WINDOWS = {"kaiser-bessel": 0, "gaussian": 1, "bspline": 2, "sinc": 3}


class window:
    """Context manager selecting the window of the oracle's NFFT functions
    (``with window("gaussian"): ...``; also "bspline", "sinc"); Kaiser-Bessel otherwise."""

    def __init__(self, name):
        self.code = WINDOWS[name]

    def __enter__(self):
        self.prev = _load().or_get_window()
        _load().or_set_window(self.code)
        return self

    def __exit__(self, *exc):
        _load().or_set_window(self.prev)
        return False


def dft_naive(a, sign):
    a = _c128(a)
    out = np.empty_like(a)
    _load().or_dft_naive(_p(a), _p(out), a.size, int(sign))
    return out


def fft_1d(a, sign):
    a = _c128(a).copy()
    _load().or_fft_1d(_p(a), a.size, int(sign))
    return a


def fft_d(a, sign):
    a = _c128(a).copy()
    n = _dims(a.shape)
    _load().or_fft_d(a.ndim, _p(n), _p(a), int(sign))
    return a


def ndft_trafo(x, fhat):
    x = _f64(x)
    fhat = _c128(fhat)
    N = _dims(fhat.shape)
    M, d = x.shape
    assert d == fhat.ndim
    f = np.empty(M, dtype=np.complex128)
    _load().or_ndft_trafo(d, _p(N), M, _p(x), _p(fhat), _p(f))
    return f


def ndft_adjoint(x, f, N):
    x = _f64(x)
    f = _c128(f)
    N = _dims(N)
    M, d = x.shape
    out = np.empty(tuple(N), dtype=np.complex128)
    _load().or_ndft_adjoint(d, _p(N), M, _p(x), _p(f), _p(out))
    return out


def nndft_trafo(v, x, fhat):
    """NNDFT (Sec. 1's generalisation with nonequispaced frequencies), by its definition:
    f_j = sum_k fhat_k exp(-2 pi i v_k.x_j) for frequencies v (K, d) and nodes x (M, d)."""
    v = _f64(v)
    x = _f64(x)
    fhat = _c128(fhat).reshape(-1)
    K, d = v.shape
    M, d2 = x.shape
    assert d == d2 and fhat.shape[0] == K
    f = np.empty(M, dtype=np.complex128)
    _load().or_nndft_trafo(d, K, M, _p(v), _p(x), _p(fhat), _p(f))
    return f


def nndft_adjoint(v, x, f):
    """hhat_k = sum_j f_j exp(+2 pi i v_k.x_j)."""
    v = _f64(v)
    x = _f64(x)
    f = _c128(f).reshape(-1)
    K, d = v.shape
    M, d2 = x.shape
    assert d == d2 and f.shape[0] == M
    h = np.empty(K, dtype=np.complex128)
    _load().or_nndft_adjoint(d, K, M, _p(v), _p(x), _p(f), _p(h))
    return h


def fastsum(x, y, bhat, alpha):
    """Kernel sums g_j = sum_l alpha_l K(y_j - x_l) for the trigonometric polynomial
    K(z) = sum_k bhat_k e^{-2 pi i k.z} (the sign of eq. (1.2)) -- the fast summation
    application named in Sec. 1 -- written out through the direct sums:
    g_j = sum_k (bhat_k sum_l alpha_l e^{2 pi i k.x_l}) e^{-2 pi i k.y_j}."""
    c = _c128(bhat) * ndft_adjoint(x, alpha, np.shape(bhat))
    return ndft_trafo(y, c)


def ndft_adjoint_at(x, f, N, flat_idx):
    """hhat at the given flat (centred, row-major) coefficient positions."""
    x = _f64(x)
    f = _c128(f)
    N = _dims(N)
    sel = _dims(flat_idx)
    M, d = x.shape
    out = np.empty(sel.size, dtype=np.complex128)
    _load().or_ndft_adjoint_at(d, _p(N), M, _p(x), _p(f), sel.size, _p(sel), _p(out))
    return out


def ndft_grad_x(x, fhat, r):
    """dL/dx for L = ||A(x) fhat - y||^2 given the residual r = A(x) fhat - y."""
    x = _f64(x)
    fhat = _c128(fhat)
    r = _c128(r)
    N = _dims(fhat.shape)
    M, d = x.shape
    g = np.empty((M, d), dtype=np.float64)
    _load().or_ndft_grad_x(d, _p(N), M, _p(x), _p(fhat), _p(r), _p(g))
    return g


def default_n(N):
    """n_t = 2^(ceil(log2 N_t) + 1), the default FFT length (Sec. 3.1)."""
    return tuple(1 << (int(np.ceil(np.log2(v))) + 1) for v in N)


def nfft_deconv(fhat, n, m):
    fhat = _c128(fhat)
    N = _dims(fhat.shape)
    n = _dims(n)
    g = np.empty(tuple(n), dtype=np.complex128)
    _load().or_nfft_deconv(fhat.ndim, _p(N), _p(n), int(m), _p(fhat), _p(g))
    return g


def nfft_deconv_adj(g, N, m):
    g = _c128(g)
    n = _dims(g.shape)
    N = _dims(N)
    out = np.empty(tuple(N), dtype=np.complex128)
    _load().or_nfft_deconv_adj(g.ndim, _p(N), _p(n), int(m), _p(g), _p(out))
    return out


def nfft_grid(fhat, n, m):
    """Steps 1-2 of Algorithm 2.1: the oversampled grid g = F D fhat."""
    fhat = _c128(fhat)
    N = _dims(fhat.shape)
    n = _dims(n)
    g = np.empty(tuple(n), dtype=np.complex128)
    _load().or_nfft_grid(fhat.ndim, _p(N), _p(n), int(m), _p(fhat), _p(g))
    return g


def nfft_adjoint_from_grid(g, N, m):
    """Steps 2-3 of Algorithm 2.2 applied to a grid: D^H F^H g."""
    g = _c128(g)
    n = _dims(g.shape)
    N = _dims(N)
    out = np.empty(tuple(N), dtype=np.complex128)
    _load().or_nfft_adjoint_from_grid(g.ndim, _p(N), _p(n), int(m), _p(g), _p(out))
    return out


def nfft_interp(x, g, N, m):
    """Step 3 of Algorithm 2.1 (B) on a given grid."""
    x = _f64(x)
    g = _c128(g)
    n = _dims(g.shape)
    N = _dims(N)
    M, d = x.shape
    f = np.empty(M, dtype=np.complex128)
    _load().or_nfft_interp(d, _p(N), _p(n), int(m), M, _p(x), _p(g), _p(f))
    return f


def nfft_spread(x, f, N, n, m):
    """Step 1 of Algorithm 2.2 (B^T): the grid g from node values f."""
    x = _f64(x)
    f = _c128(f)
    n = _dims(n)
    N = _dims(N)
    M, d = x.shape
    g = np.empty(tuple(n), dtype=np.complex128)
    _load().or_nfft_spread(d, _p(N), _p(n), int(m), M, _p(x), _p(f), _p(g))
    return g


def nfft_interp_dx(x, g, N, m):
    """d f_j / d x_{j,t} through the window (complex, shape (M, d))."""
    x = _f64(x)
    g = _c128(g)
    n = _dims(g.shape)
    N = _dims(N)
    M, d = x.shape
    out = np.empty((M, d), dtype=np.complex128)
    _load().or_nfft_interp_dx(d, _p(N), _p(n), int(m), M, _p(x), _p(g), _p(out))
    return out


def nfft_trafo(x, fhat, n=None, m=8):
    x = _f64(x)
    fhat = _c128(fhat)
    N = _dims(fhat.shape)
    n = _dims(default_n(fhat.shape) if n is None else n)
    M, d = x.shape
    f = np.empty(M, dtype=np.complex128)
    _load().or_nfft_trafo(d, _p(N), _p(n), int(m), M, _p(x), _p(fhat), _p(f))
    return f


def nfft_adjoint(x, f, N, n=None, m=8):
    x = _f64(x)
    f = _c128(f)
    N = _dims(N)
    n = _dims(default_n(tuple(N)) if n is None else n)
    M, d = x.shape
    out = np.empty(tuple(N), dtype=np.complex128)
    _load().or_nfft_adjoint(d, _p(N), _p(n), int(m), M, _p(x), _p(f), _p(out))
    return out


def err_l2(ref, approx):
    """E_2 of eq. (2.15)."""
    ref = _c128(ref).reshape(-1)
    approx = _c128(approx).reshape(-1)
    return _load().or_err_l2(_p(ref), _p(approx), ref.size)


def err_inf(ref, approx, l1):
    """E_inf of eq. (2.16) with the l1 norm of the input passed in."""
    ref = _c128(ref).reshape(-1)
    approx = _c128(approx).reshape(-1)
    return _load().or_err_inf(_p(ref), _p(approx), ref.size, float(l1))
