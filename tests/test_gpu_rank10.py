"""Parity at TR ranks 9 and 10 (r_k r_{k+1} = 81, 90 and 100 > 64): the paths that only
ranks above 8 take, against the FP64 oracle.

At these ranks the Gram matrix G^{!=k} is 81..100 square, so the FGMC ring runs as
separate FP64 products (its sides exceed the one-work-group form), the Gauss-Jordan
inverse works on a matrix larger than its register form, the matrix-core passes use
K = 96 / 128 (three and four k-steps of 32 per m-tile), the FP32/FP64 passes keep their
column items in LDS only, and the convergence product reads G from global memory.
The differentiation form is checked at the rank of its workload (200^4, TR rank 10) on
the leading 12^4 slice of that workload's cores: central differences of the GPU loss
over every one of the 4,800 core parameters, and the oracle gradient.

Bars as elsewhere: FP32 one step 1e-5 (gradient 3e-5), FP64 1e-10, Gram 1e-12,
BF16 forms gradient 2e-2 and step 1e-2 relative Frobenius."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import synth  # noqa: E402
from oracle import awrtrd as aw  # noqa: E402
from oracle import tr  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from _helpers import device_cores, device_problem, host_cores, host_problem, rel, unflatten_d  # noqa: E402

F32, F64 = np.float32, np.float64
TOL = {F32: 1e-5, F64: 1e-10}

SHAPES = [
    ((14, 13, 12, 11), (10, 10, 10, 10)),   # R = 100, K = 128
    ((26, 19, 23), (9, 10, 9)),             # R = 90 / 81, K = 128 / 96
    ((130, 120), (10, 9)),                  # N = 2 (each I_j > R: G^{!=k} nonsingular)
]


def _setup(dims, ranks, rho=0.4, seed=0, dtype=F32):
    X, P, Z0, Zt, xstar = host_problem(dims, ranks, rho, seed, dtype, reconstruct=tr.reconstruct)
    prob = device_problem(X, P, dims, ranks, dtype)
    return X, P, Z0, prob


@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_rank10_fgmc_gram_and_reconstruction(dims, ranks):
    X, P, Z0, prob = _setup(dims, ranks)
    cores = device_cores(Z0, F32)
    for k in range(len(dims)):
        G = prob.fgmc_gram(cores, k).cpu().numpy()
        assert rel(G, aw.gram_explicit(Z0, k)) <= 1e-12, k
    full = prob.reconstruct(cores).cpu().numpy()
    assert rel(full, tr.reconstruct(Z0).ravel(order="F")) <= 1e-6


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_rank10_grad(dims, ranks, dtype):
    X, P, Z0, prob = _setup(dims, ranks, dtype=dtype)
    cores = device_cores(Z0, dtype)
    sigma = 1.3
    for k in range(len(dims)):
        d, stats = prob.grad(cores, k, sigma)
        _, info = aw.core_update(X, P, Z0, k, sigma)
        got = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % len(dims)])
        assert rel(got, info.d) <= 3 * TOL[dtype], (k, rel(got, info.d))
        s = stats.cpu().numpy()
        assert s[2] == info.n_obs
        assert s[0] == pytest.approx(info.loss, rel=1e-5 if dtype == F32 else 1e-11)


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_rank10_step_teacher_forced(dims, ranks, dtype):
    X, P, Z0, prob = _setup(dims, ranks, dtype=dtype)
    sigma = 1.1
    for k in range(len(dims)):
        cores = device_cores(Z0, dtype)
        eta, flags = prob.step(cores, k, sigma, 1e-9)
        ref, info = aw.core_update(X, P, Z0, k, sigma, 1e-9)
        got = host_cores(cores, dims, ranks)
        assert int(flags) == 0
        assert rel(got[k], ref) <= TOL[dtype], (k, rel(got[k], ref))
        assert float(eta) == pytest.approx(info.eta, rel=1e-4 if dtype == F32 else 1e-9)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("dims,ranks", SHAPES[:2])
def test_rank10_bf16_grad_step_and_backward(dims, ranks, prec):
    X, P, Z0, prob = _setup(dims, ranks)
    prob.set_precision(prec)
    sigma = 1.2
    worst = 0.0
    for k in range(len(dims)):
        cores = device_cores(Z0, F32)
        d, stats = prob.grad(cores, k, sigma)
        ref, info = aw.core_update(X, P, Z0, k, sigma, 1e-9)
        got = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % len(dims)])
        worst = max(worst, rel(got, info.d))
        assert rel(got, info.d) <= 2e-2, (k, rel(got, info.d))
        assert stats[2].item() == info.n_obs
        eta, flags = prob.step(cores, k, sigma, 1e-9)
        assert int(flags) == 0
        assert rel(host_cores(cores, dims, ranks)[k], ref) <= 1e-2, k
    cores = device_cores(Z0, F32)
    grads = prob.loss_bwd(cores, sigma)
    gref = aw.loss_grads(X, P, Z0, sigma)
    for k in range(len(dims)):
        assert rel(host_cores(grads, dims, ranks)[k], gref[k]) <= 2e-2, k
    print(f"{prec} rank-10 gradient worst relative error {worst:.2e}")


def test_rank10_fit_given_sigma_matches_oracle():
    dims, ranks = (14, 13, 12, 11), (10, 10, 10, 10)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5, dtype=F64)
    sig = [2.0, 1.2, 0.9]
    cores = device_cores(Z0, F64)
    rep = prob.fit(cores, max_sweeps=len(sig), tol=0.0, sigma_mode="given", sigma_given=sig)
    ref, hist = aw.fit(X, P, Z0, aw.FitOptions(max_sweeps=len(sig), tol=0.0, sigma_mode="given",
                                               sigma_given=sig))
    got = host_cores(cores, dims, ranks)
    assert max(rel(g, r) for g, r in zip(got, ref)) <= 1e-9
    for a, b in zip(rep["e"][1:], hist["e"][1:]):
        assert a == pytest.approx(b, rel=1e-7)


def _cfg5_slice(seed=0, n=12):
    """The differentiation-form workload (200^4, TR rank 10, 5 % observed, 10 % outliers
    U[-10 std, 10 std]) cut to its leading n^4 block: the cores' first n lateral slices (the
    block of a TR tensor is the TR tensor of those slices), the recipe's mask and outliers
    drawn on the block, and the evaluation point = true cores + N(0, 0.1/r) per entry."""
    w = synth.WORKLOADS["tr4_200_r10"]
    std = 1.0 / math.sqrt(w.ranks[0])
    full = synth.gaussian_cores(w.dims, w.ranks, seed, std)
    Zt = [z[:, :n, :].copy() for z in full]
    dims = (n,) * 4
    ws = synth.scaled(w, dims)
    xstar = tr.reconstruct(Zt)
    mask = synth.bernoulli_mask(dims, ws.rho, seed)
    X = synth.assemble(ws, xstar, mask, seed)
    Z = synth.perturbed_cores(Zt, seed, rel=0.1)
    return dims, w.ranks, X, mask, Z


def test_rank10_backward_central_differences_on_the_12x12x12x12_slice():
    dims, ranks, X, P, Z = _cfg5_slice()
    assert int(P.sum()) > 0
    prob = device_problem(X, P, dims, ranks, F64)
    # kernel width by the quantile rule at this point (the workload's fixed sigma)
    e = aw.residual_abs(X, P, Z)
    sigma = aw.quantile_sigma(e, 0.5, 5.0, 1e-6 * float(np.max(np.abs(X[P.astype(bool)]))))
    cores = [c.requires_grad_(True) for c in device_cores(Z, F64)]
    L = trd.correntropy_loss(prob, cores, sigma)
    assert float(L) == pytest.approx(aw.loss(X, P, Z, sigma), rel=1e-12)
    L.backward()
    g = [c.grad.detach().cpu().numpy() for c in cores]
    ref = aw.loss_grads(X, P, Z, sigma)
    ref_flat = synth.cores_to_flat(ref, np.float64)
    for k in range(4):
        assert rel(g[k], ref_flat[k]) <= 1e-11, k
    # central differences, h = 1e-6, over all 4 x 10 x 12 x 10 = 4800 parameters
    h = 1e-6
    base = [c.detach().clone() for c in cores]
    worst = 0.0
    nparam = 0
    for k in range(4):
        vals = base[k].cpu().numpy().copy()
        fd = np.empty(vals.size)
        for i in range(vals.size):
            with torch.no_grad():
                base[k][i] = float(vals[i]) + h
                lp = float(prob.loss_fwd(base, sigma))
                base[k][i] = float(vals[i]) - h
                lm = float(prob.loss_fwd(base, sigma))
                base[k][i] = float(vals[i])
            fd[i] = (lp - lm) / (2 * h)
        nparam += fd.size
        err = np.max(np.abs(fd - g[k]) / np.maximum(1.0, np.abs(fd)))
        worst = max(worst, float(err))
        assert err <= 1e-6, (k, err)
    assert nparam == 4800
    print(f"rank-10 slice: worst |FD - grad| / max(1, |FD|) = {worst:.2e} over {nparam} parameters")
