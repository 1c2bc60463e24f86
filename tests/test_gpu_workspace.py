"""trd_workspace_bytes against what a bound problem actually holds.

For each shape and precision form the query is made before binding; then the problem is
bound and driven through every call that allocates (quantile fits, a step and a gradient on
every core, the differentiation form's backward), and the workspace it reports must stay
within the query's bound, and within its typical figure for the uniformly random masks the
tests draw.  A clustered mask (the first n_obs entries in storage order) checks the bound
where the typical figure does not apply."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import synth  # noqa: E402
from oracle import tr  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from _helpers import device_cores, device_problem, host_problem  # noqa: E402

F32, F64 = np.float32, np.float64

CASES = [
    ((13, 12, 11, 10, 9), (8,) * 5, 0.3, F32, "bf16"),
    ((13, 12, 11, 10, 9), (8,) * 5, 0.3, F32, "bf16x3"),
    ((13, 12, 11, 10, 9), (8,) * 5, 0.3, F32, "native"),
    ((26, 19, 23), (9, 10, 9), 0.4, F32, "bf16"),
    ((30, 30, 30), (3, 3, 3), 0.5, F64, "native"),
    ((130, 120), (10, 9), 0.4, F32, "native"),
    ((40, 50, 60, 3), (4, 4, 4, 4), 0.05, F32, "bf16"),
]


def _drive(prob, Z0, dims, ranks, dtype, prec):
    """every allocating call in this precision form"""
    cores = device_cores(Z0, dtype)
    prob.fit(cores, max_sweeps=2, tol=0.0, precision=prec)
    prob.fit(device_cores(Z0, dtype), max_sweeps=1, tol=0.0, precision=prec, sigma_mode="fixed",
             sigma=1.0)
    prob.set_precision(prec)
    for k in range(len(dims)):
        c = device_cores(Z0, dtype)
        prob.grad(c, k, 1.3)
        prob.step(c, k, 1.3, 1e-9)
    if dtype == F32 or prec == "native":
        prob.loss_bwd(device_cores(Z0, dtype), 1.3)
    prob.set_precision("native")
    torch.cuda.synchronize()


@pytest.mark.parametrize("dims,ranks,rho,dtype,prec", CASES)
def test_workspace_within_the_query(dims, ranks, rho, dtype, prec):
    X, P, Z0, Zt, xstar = host_problem(dims, ranks, rho, 0, dtype, reconstruct=tr.reconstruct)
    n_obs = int(P.sum())
    tdt = torch.float32 if dtype == F32 else torch.float64
    q = trd.trd_workspace_bytes(dims, ranks, n_obs, tdt, prec)
    prob = device_problem(X, P, dims, ranks, dtype)
    _drive(prob, Z0, dims, ranks, dtype, prec)
    got = prob.info()["workspace_bytes"]
    print(f"{dims} r{ranks} {prec}: held {got} B, typical {q['typical']} B, bound {q['bound']} B")
    assert q["typical"] <= q["bound"]
    assert got <= q["typical"]
    assert got <= q["bound"]


@pytest.mark.parametrize("prec", ["native", "bf16"])
def test_workspace_bound_holds_for_a_clustered_mask(prec):
    dims, ranks = (24, 20, 16, 12), (5, 5, 5, 5)
    X, _, Z0, _, _ = host_problem(dims, ranks, 0.3, 1, F32, reconstruct=tr.reconstruct)
    n = int(np.prod(dims))
    flat = np.zeros(n, dtype=np.uint8)
    flat[: n // 7] = 1                  # the first n/7 entries in storage (mode-0 fastest) order
    P = flat.reshape(dims, order="F")
    q = trd.trd_workspace_bytes(dims, ranks, int(P.sum()), torch.float32, prec)
    prob = device_problem(X, P, dims, ranks, F32)
    _drive(prob, Z0, dims, ranks, F32, prec)
    got = prob.info()["workspace_bytes"]
    print(f"clustered {prec}: held {got} B, bound {q['bound']} B")
    assert got <= q["bound"]


def test_workspace_query_rejects_bad_arguments():
    for dims, ranks, n_obs in (((10,), (2,), 5), ((10, 10), (2, 2), -1), ((10, 10), (2, 2), 101),
                               ((10, 10), (2, 17), 5)):
        with pytest.raises(trd.TrdError):
            trd.trd_workspace_bytes(dims, ranks, n_obs)
    with pytest.raises(trd.TrdError):   # the BF16 forms need an FP32 problem
        trd.trd_workspace_bytes((10, 10), (2, 2), 5, torch.float64, "bf16")
