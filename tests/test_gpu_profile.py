"""The measurement hooks that bench.py reads (trd_profile / trd_profile_read): every launch
of the fused gradient pass is timed with its own pair of HIP events, on the matrix-core
tile passes (events handed to the launch) and on the sliced-ELL passes (events recorded
around it), and the read returns the launches, their summed duration and the observed
entries they covered, then resets."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import numpy as np  # noqa: E402

from oracle import tr  # noqa: E402
from _helpers import device_cores, device_problem, host_problem  # noqa: E402

F32 = np.float32


def _problem(dims, ranks):
    X, P, Z0, _, _ = host_problem(dims, ranks, 0.4, 4, F32, reconstruct=tr.reconstruct)
    return Z0, device_problem(X, P, dims, ranks, F32)


@pytest.mark.parametrize("dims,ranks,precision,sketch", [
    ((30, 30, 30), (3, 3, 3), "native", None),          # sliced-ELL passes
    ((20, 70, 20, 20), (8, 8, 8, 8), "bf16", None),     # matrix-core tile passes
    ((30, 30, 30), (3, 3, 3), "native", [8, 7, 6]),     # RStS sketches
])
def test_profile_counts_every_gradient_pass(dims, ranks, precision, sketch):
    Z0, prob = _problem(dims, ranks)
    N, sweeps = len(dims), 2
    n_obs = prob.info()["n_obs"]
    cores = device_cores(Z0, F32)
    prob.fit(cores, max_sweeps=1, tol=0.0, precision=precision, sketch_sizes=sketch)  # warm-up
    prob.profile(True)
    rep = prob.fit(cores, max_sweeps=sweeps, tol=0.0, precision=precision, sketch_sizes=sketch)
    torch.cuda.synchronize()
    p = prob.profile_read()
    prob.profile(False)
    assert rep["sweeps"] == sweeps
    # the quantile kernel width: in the tile forms core 0's pass reads the stored residuals
    # (another kernel, not timed); every other update runs the timed gradient pass
    timed_per_sweep = N - 1 if precision != "native" and sketch is None else N
    assert p["launches"] == sweeps * timed_per_sweep
    assert 0.0 < p["total_ms"] / p["launches"] < 100.0
    if sketch is None:
        assert p["entries"] == p["launches"] * n_obs
    else:  # counted on the device: each sketch holds part of the observed entries
        assert 0 < p["entries"] < p["launches"] * n_obs
    again = prob.profile_read()  # the read resets the counters
    assert again["launches"] == 0 and again["entries"] == 0 and again["total_ms"] == 0.0
