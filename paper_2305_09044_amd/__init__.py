"""MI355X-native robust tensor-ring decomposition (AWRTRD / SAWRTRD per-core sweep).

The compute path is libtrd.so (hand-written HIP kernels for gfx950 behind the C ABI in
include/trd.h); this package is the thin Python binding plus a torch.autograd.Function
for the differentiation form.  Nothing here computes on the CPU.
"""
from ._lib import (TRD_FLAG_CLAMPED, TRD_FLAG_EMPTY, TRD_FLAG_NOTSPD, TRD_FLAG_ZERO_DEN, Problem, TrdError,  # noqa: F401
                   header_functions, load, make_sketch, trd_fgmc_gram_noalloc, trd_sample_mask,
                   trd_sample_rows, trd_sample_sketch, trd_weights, trd_workspace_bytes)
from .autograd import CorrentropyLoss, correntropy_loss  # noqa: F401
