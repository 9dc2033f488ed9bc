"""Error measures for comparing an NFFT result with the oracle's when the deconvolution is
ill-conditioned (oversampled grids n close to N).  Test infrastructure: only the oracle is
called.

Near n = N the deconvolution factors w_k = 1 / (n phi_hat(k)) span many orders of magnitude,
so the rounding of any FP64 evaluation is amplified far beyond 1e-12 in the plain relative
error.  The measures below are the relative l2 error (E_2, eq. (2.15)) taken in the norms in
which each last step is well-conditioned, plus element-wise forms:

* transform: the rounding error of f_j after an accurate grid g is a small multiple of
  s_j = sum_l phi(x_j - l/n) |g_l| (the window is nonnegative), so
  e2 = ||f - f_ref||_2 / ||s||_2 and emax = max_j |f_j - f_ref_j| / s_j;
* adjoint: h_k = w_k y_k with y = F^H B^T f, whose rounding error per entry is a small
  multiple of ||B^T f||_2, so e2 = ||(h - h_ref) / w||_2 / ||h_ref / w||_2 (the relative error
  of y) and emax = max_k |h_k - h_ref_k| / (w_k ||B^T f||_2).

Where w_k is flat (n = 2N) these are within small factors of the plain E_2 and max errors.
"""
import numpy as np

from oracle import oracle as O


def trafo_errors(x, fhat, N, n, m, f, ref=None):
    """(e2, emax) of a transform result f against the oracle's (or ref)."""
    if ref is None:
        ref = O.nfft_trafo(x, fhat, n, m)
    g = O.nfft_grid(fhat, n, m)
    s = np.real(O.nfft_interp(x, np.abs(g).astype(np.complex128), N, m))
    diff = np.abs(np.ravel(f) - np.ravel(ref))
    return float(np.linalg.norm(diff) / np.linalg.norm(s)), float(np.max(diff / s))


def adjoint_errors(x, f_in, N, n, m, h, ref=None):
    """(e2, emax) of an adjoint result h against the oracle's (or ref)."""
    if ref is None:
        ref = O.nfft_adjoint(x, f_in, N, n, m)
    gs = O.nfft_spread(x, f_in, N, n, m)
    wk = np.ravel(np.abs(O.nfft_deconv_adj(np.ones(n, np.complex128), N, m)))
    diff = np.abs(np.ravel(h) - np.ravel(ref)) / wk
    return (float(np.linalg.norm(diff) / np.linalg.norm(np.ravel(ref) / wk)),
            float(np.max(diff) / np.linalg.norm(gs)))
