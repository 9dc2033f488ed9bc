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


def rel_l2(ref, approx):
    ref = np.ravel(ref)
    approx = np.ravel(approx)
    return float(np.linalg.norm(ref - approx) / np.linalg.norm(ref))
