"""trd_fit without a stop test (tol <= 0) queues its sweeps without waiting for each
sweep's report and reads the reports in batches (Alg. 1 with a fixed sweep count).  These
tests check that this changes nothing: the same cores, kernel widths, line-search steps
and D^t changes, bit for bit, as the run that reads every report before the next sweep
(a positive tol that never stops it), across the batch boundary; and that a sweep that hits
a G + lambda I that is not positive definite (eq. 10) still ends the run with the cores
that sweep left, although later sweeps were already queued."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import tr  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from paper_2305_09044_amd._lib import TRD_ENOTSPD, TRD_OK  # noqa: E402
from _helpers import device_cores, device_problem, host_problem  # noqa: E402

F32, F64 = np.float32, np.float64
NEVER = 1e-300  # a stop test that does not fire: every report is read before the next sweep


def _problem(dims, ranks, dtype, **kw):
    X, P, Z0, _, _ = host_problem(dims, ranks, kw.pop("rho", 0.5), 3, dtype,
                                  reconstruct=tr.reconstruct, **kw)
    return X, P, Z0, device_problem(X, P, dims, ranks, dtype)


CASES = [
    # (dims, ranks, dtype, fit options)
    ((20, 18, 16), (3, 3, 3), F32, {}),
    ((20, 18, 16), (3, 3, 3), F64, {}),
    # the BF16 form on B-major rows (TR rank 8), as the benchmark runs it
    ((20, 70, 20, 20), (8, 8, 8, 8), F32, {"precision": "bf16"}),
    # RStS: every update draws its sketch from (seed, sweep, core)
    ((20, 18, 16), (3, 3, 3), F32, {"sketch_sizes": [6, 5, 4], "seed": 11}),
]


@pytest.mark.parametrize("dims,ranks,dtype,opts", CASES)
def test_fit_without_stop_test_matches_per_sweep_reports(dims, ranks, dtype, opts):
    # 36 sweeps: the reports of the first 32 are read in one batch, the rest at the end
    _, _, Z0, prob = _problem(dims, ranks, dtype)
    runs = []
    for tol in (0.0, NEVER):
        cores = device_cores(Z0, dtype)
        rep = prob.fit(cores, max_sweeps=36, tol=tol, **opts)
        runs.append((cores, rep))
    (ca, ra), (cb, rb) = runs
    assert ra["status"] == rb["status"] == TRD_OK
    assert ra["sweeps"] == rb["sweeps"] == 36
    for a, b in zip(ca, cb):
        assert torch.equal(a, b)
    for key in ("e", "sigma", "eta", "flags", "last_e", "last_sigma"):
        assert ra[key] == rb[key], key
    assert all(math.isfinite(e) for e in ra["e"][1:])


@pytest.mark.parametrize("tol", [0.0, NEVER])
def test_fit_stops_with_the_cores_of_the_sweep_that_hit_not_spd(tol):
    # I_1 = I_2 = 1: G^{!=0} has rank 1 < R^2 = 4, so with lambda = 0 core 0's step fails in
    # every sweep while cores 1 and 2 (Grams of rank 4 from the 8 slices of core 0) move;
    # the run ends after the first sweep with that sweep's cores
    dims, ranks = (8, 1, 1), (2, 2, 2)
    _, _, Z0, prob = _problem(dims, ranks, F32, rho=1.0, outlier_frac=0.0)
    one = device_cores(Z0, F32)
    r1 = prob.fit(one, max_sweeps=1, tol=0.0, sigma_mode="fixed", sigma=math.inf, lambda_rel=0.0)
    cores = device_cores(Z0, F32)
    rep = prob.fit(cores, max_sweeps=5, tol=tol, sigma_mode="fixed", sigma=math.inf,
                   lambda_rel=0.0)
    assert r1["status"] == rep["status"] == TRD_ENOTSPD
    assert rep["sweeps"] == 1
    assert rep["flags"] & trd.TRD_FLAG_NOTSPD
    assert rep["eta"] == r1["eta"]
    z0 = device_cores(Z0, F32)
    assert torch.equal(cores[0], z0[0])            # the failed step left core 0
    assert not torch.equal(cores[1], z0[1])        # the sweep moved the others
    for a, b in zip(cores, one):
        assert torch.equal(a, b)
