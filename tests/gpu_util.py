"""Helpers shared by the GPU tests (no transform arithmetic here)."""
import sys

import numpy as np
import torch

TOL = {torch.complex128: 1e-12, torch.complex64: 5e-6}


def announce(*parts):
    """Name the case on stderr before its GPU work starts (survives a crash of the run)."""
    sys.__stderr__.write("[case] " + " ".join(str(p) for p in parts) + "\n")
    sys.__stderr__.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def parity_err(ref, approx):
    """The larger of the relative l2 error (E_2 of eq. (2.15)) and the element-wise error
    max_j |ref_j - approx_j| / max_j |ref_j| (an E_inf-type bound in the spirit of eq. (2.16),
    normalised by the reference's own largest entry so that it is at least as strict as E_2
    for errors concentrated on a few outputs)."""
    ref = np.ravel(ref)
    approx = np.ravel(approx)
    diff = ref - approx
    e2 = np.linalg.norm(diff) / np.linalg.norm(ref)
    einf = np.max(np.abs(diff)) / np.max(np.abs(ref))
    return float(max(e2, einf))


def rel_l2(ref, approx):
    """E_2 of eq. (2.15): relative l2 error."""
    ref = np.ravel(ref)
    approx = np.ravel(approx)
    return float(np.linalg.norm(ref - approx) / np.linalg.norm(ref))


def e_inf(ref, approx, inp):
    """E_inf of eq. (2.16): max_j |ref_j - approx_j| / ||input||_1.  For comparisons whose
    bar is an approximation error of the method (not rounding), where an element-wise
    bound relative to the largest output is not what the method guarantees."""
    return float(np.max(np.abs(np.ravel(ref) - np.ravel(approx))) / np.sum(np.abs(np.ravel(inp))))
