"""The FGMC Gram entry point that allocates nothing (trd_fgmc_gram_noalloc) against the
context-based one (trd_fgmc_gram) and the oracle, on two calls in a row, the second on a
smaller input, both through the C ABI: the same kernels in the same order give the same
bits; the explicit A^T A agrees to FP64 rounding (1e-12 relative)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import awrtrd as aw  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from _helpers import device_cores, rel  # noqa: E402


def _cores(dims, ranks, seed, dtype):
    g = np.random.default_rng(seed)
    N = len(dims)
    Z = [g.standard_normal((ranks[j], dims[j], ranks[(j + 1) % N])) / np.sqrt(ranks[j]) for j in range(N)]
    Z = [z.astype(dtype).astype(np.float64) for z in Z]
    return Z, device_cores(Z, dtype)


CASES = [
    # (dims, ranks, dtype): ring in one work-group (sides <= 64), then the FP64 product chain
    # (sides 81 / 100 > 64), then a smaller input again
    (((37, 41, 29, 23, 11), (3, 4, 5, 2, 3)), np.float32),
    (((14, 13, 12, 11), (9, 10, 10, 9)), np.float64),
    (((9, 10, 11), (2, 3, 2)), np.float32),
]


def test_noalloc_gram_equals_context_gram_on_consecutive_calls():
    for (dims, ranks), dt in CASES:
        Z, cores = _cores(dims, ranks, len(dims), dt)
        tdt = torch.float32 if dt == np.float32 else torch.float64
        shape = trd.Problem(None, None, dims, ranks, dtype=tdt)
        for k in range(len(dims)):
            want = shape.fgmc_gram(cores, k)
            got = trd.trd_fgmc_gram_noalloc(cores, dims, ranks, k)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (dims, k)
            assert rel(got.cpu().numpy(), aw.gram_explicit(Z, k)) <= 1e-12, (dims, k)
        shape.close()


def test_noalloc_gram_rejects_shapes_beyond_its_scratch():
    dims, ranks = (3, 3, 3, 3, 3), (16, 16, 16, 16, 16)   # 4 factors of 256 x 256 + partials
    cores = [torch.zeros(16 * 3 * 16, dtype=torch.float32, device="cuda") for _ in dims]
    with pytest.raises(trd.TrdError) as ei:
        trd.trd_fgmc_gram_noalloc(cores, dims, ranks, 0)
    assert ei.value.code == trd._lib.TRD_EUNSUPPORTED
    assert "scratch" in str(ei.value)
    # a null output is an argument error, caught before any launch
    lib = trd._lib.load()
    d = (C.c_int64 * 3)(9, 10, 11)
    r = (C.c_int32 * 3)(2, 3, 2)
    small = [torch.zeros(2 * n * 3, dtype=torch.float32, device="cuda") for n in (9, 10, 11)]
    assert lib.trd_fgmc_gram_noalloc(3, d, r, 0, trd._lib._ptr_array(small), 0, None, None) == -1
