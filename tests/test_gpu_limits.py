"""The library's size limits against the oracle: the largest order (N = 8), the widest
subchain product the passes take (r_k r_s = 128, rank 16 next to rank 8, K = 128 matrix-core
passes and a 128 x 128 Gram), and the shapes beyond them, which are rejected with an error.
Bars as elsewhere: FP32 step 1e-5 (gradient 3e-5), FP64 1e-10, BF16 step 1e-2 (gradient
2e-2), Gram 1e-12."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import awrtrd as aw  # noqa: E402
from oracle import tr  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from _helpers import device_cores, device_problem, host_cores, host_problem, rel, unflatten_d  # noqa: E402

F32, F64 = np.float32, np.float64
TOL = {F32: 1e-5, F64: 1e-10}
LIMITS = [((4, 3, 3, 4, 3, 3, 2, 3), (2, 2, 3, 2, 2, 2, 3, 2)),   # N = 8
          ((24, 20, 18), (16, 8, 2))]                             # r_0 r_1 = 128


@pytest.mark.parametrize("dims,ranks", LIMITS)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_limits_grad_and_step(dims, ranks, dtype):
    X, P, Z0, _, _ = host_problem(dims, ranks, 0.6, 2, dtype, reconstruct=tr.reconstruct)
    prob = device_problem(X, P, dims, ranks, dtype)
    N = len(dims)
    for k in range(N):
        cores = device_cores(Z0, dtype)
        G = prob.fgmc_gram(cores, k).cpu().numpy()
        assert rel(G, aw.gram_explicit(Z0, k)) <= 1e-12, k
        d, stats = prob.grad(cores, k, 1.2)
        ref, info = aw.core_update(X, P, Z0, k, 1.2, 1e-9)
        got_d = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % N])
        assert rel(got_d, info.d) <= 3 * TOL[dtype], (k, rel(got_d, info.d))
        eta, flags = prob.step(cores, k, 1.2, 1e-9)
        assert int(flags) == 0
        assert rel(host_cores(cores, dims, ranks)[k], ref) <= TOL[dtype], k


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_widest_product_in_the_bf16_forms(prec):
    dims, ranks = LIMITS[1]
    X, P, Z0, _, _ = host_problem(dims, ranks, 0.6, 2, F32, reconstruct=tr.reconstruct)
    prob = device_problem(X, P, dims, ranks, F32)
    prob.set_precision(prec)
    for k in range(3):
        cores = device_cores(Z0, F32)
        d, _ = prob.grad(cores, k, 1.2)
        ref, info = aw.core_update(X, P, Z0, k, 1.2, 1e-9)
        got_d = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % 3])
        assert rel(got_d, info.d) <= 2e-2, (k, rel(got_d, info.d))
        eta, flags = prob.step(cores, k, 1.2, 1e-9)
        assert int(flags) == 0
        assert rel(host_cores(cores, dims, ranks)[k], ref) <= 1e-2, k


def test_shapes_beyond_the_limits_are_rejected():
    X = torch.zeros(8 ** 3, device="cuda")
    P = torch.ones(8 ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(trd.TrdError, match="128|split"):   # every r_k r_s = 256
        trd.Problem(X, P, (8, 8, 8), (16, 16, 16))
    with pytest.raises(trd.TrdError):                      # rank above 16
        trd.Problem(X, P, (8, 8, 8), (17, 2, 2))
    X9 = torch.zeros(2 ** 9, device="cuda")
    P9 = torch.ones(2 ** 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(trd.TrdError):                      # N = 9
        trd.Problem(X9, P9, (2,) * 9, (1,) * 9)
