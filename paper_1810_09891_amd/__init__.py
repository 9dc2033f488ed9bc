"""MI355X-native NFFT: the transforms of arXiv:1810.09891 (Algorithm 2.1 / 2.2) as
hand-written HIP kernels for gfx950 behind a C ABI (include/nfft_mi355x.h).

    from paper_1810_09891_amd import Plan
    p = Plan((512, 512), M, m=8, dtype=torch.complex64).set_nodes(x)
    f = p.trafo(fhat)        # NFFT
    h = p.adjoint(f)         # adjoint NFFT
"""
from .nfft import Batch, NNPlan, Plan, default_n, fastsum, gaussian_coefficients, tune_plan_params  # noqa: F401
from .autograd import differentiable_plan, nfft  # noqa: F401
from ._lib import (NFFT_DETERMINISTIC, NFFT_KEEP_GRID, NFFT_PRE_LIN_PSI, NFFT_SORT_NODES, NFFT_WINDOW_BSPLINE, NFFT_WINDOW_GAUSSIAN,  # noqa: F401
                   NFFT_WINDOW_SINC, NfftError, load)
