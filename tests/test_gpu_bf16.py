"""BF16 precision forms (matrix-core passes) against the FP64 oracle.

bf16: the subchain tables are rounded to bf16 (relative 2^-9) and y = w e is rounded to
bf16 as an MFMA operand, so these results are not FP32-exact.  bf16x3: the
reconstruction uses split tables (hi + lo) and three products, so residuals carry about
16 bits; the gradient contraction is still one bf16 product.  The bars below are the
measured error with a margin, stated per result: gradient <= 2e-2, one step <= 1e-2
relative Frobenius, counts exact.  Everything that is not rounded (the observed-entry
layout, counts, FGMC Gram) is compared exactly or to FP64 precision."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2305_09044_amd as trd  # noqa: E402
from oracle import awrtrd as aw  # noqa: E402
from oracle import tr  # noqa: E402
from _helpers import device_cores, device_problem, host_cores, host_problem, rel, unflatten_d  # noqa: E402

F32 = np.float32
SHAPES = [
    ((30, 30, 30), (3, 3, 3)),            # K = 32, one column tile, ragged 64-row blocks
    ((37, 41, 29, 23), (2, 3, 4, 2)),     # non-uniform ranks
    ((70, 60, 50), (5, 5, 5)),            # 3000 columns: several column tiles
    ((21, 19, 17), (8, 8, 8)),            # r_k r_s = 64 -> K = 64
    ((48, 40, 36), (8, 8, 8)),            # K = 64, full blocks of ~820 entries: eight
                                          # register rounds and the rounds read past them
    ((300, 257), (4, 3)),                 # N = 2
    # B-major block rows (TR ranks 8, >= 64 B items per slice): the gradient pass contracts
    # its row factors with U(m_B) itself
    ((20, 70, 20, 20), (8, 8, 8, 8)),     # core 0: 70 items per slice (blocks straddle two
                                          # slices), three column groups
    ((12, 11, 10, 9, 8), (8,) * 5),       # cores 2, 3: U(m_B) from two B modes
]

# the cores of the shapes above whose block rows are B-major, by the library's rule
B_MAJOR = {(20, 70, 20, 20): [0], (12, 11, 10, 9, 8): [2, 3]}


PRECS = ["bf16", "bf16x3"]


def _setup(dims, ranks, rho=0.4, seed=0, prec="bf16"):
    X, P, Z0, Zt, xstar = host_problem(dims, ranks, rho, seed, F32, reconstruct=tr.reconstruct)
    prob = device_problem(X, P, dims, ranks, F32)
    prob.set_precision(prec)
    return X, P, Z0, prob


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_bf16_grad(dims, ranks, prec):
    X, P, Z0, prob = _setup(dims, ranks, prec=prec)
    cores = device_cores(Z0, F32)
    sigma = 1.3
    worst = 0.0
    for k in range(len(dims)):
        d, stats = prob.grad(cores, k, sigma)
        _, info = aw.core_update(X, P, Z0, k, sigma)
        got = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % len(dims)])
        err = rel(got, info.d)
        worst = max(worst, err)
        assert err <= 2e-2, (k, err)
        s = stats.cpu().numpy()
        assert s[2] == info.n_obs                      # every observed entry visited once
        assert s[0] == pytest.approx(info.loss, rel=2e-2)
    print(f"{prec} gradient worst relative error {worst:.2e}")


@pytest.mark.parametrize("dims", sorted(B_MAJOR))
def test_b_major_shapes_take_the_b_major_rows(dims):
    # B-major rows need a split with B modes (split >= 1) whose items number >= 64 at TR
    # ranks 8; the split is the library's own choice, read back from trd_problem_info
    ranks = (8,) * len(dims)
    X, P, Z0, prob = _setup(dims, ranks)
    split = prob.info()["split"]
    N = len(dims)
    for k in range(N):
        nB = math.prod(dims[(k + t) % N] for t in range(1, split[k] + 1))
        assert (split[k] >= 1 and nB >= 64) == (k in B_MAJOR[dims]), (k, split[k], nB)
    # straddling blocks: a slice's rows do not fill whole 64-row blocks
    k0 = B_MAJOR[dims][0]
    assert math.prod(dims[(k0 + t) % N] for t in range(1, split[k0] + 1)) % 64 != 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", sorted(B_MAJOR))
def test_bf16_backward_on_b_major_rows(dims, prec):
    # the differentiation form's all-core backward (eq. 9 at one point, -d per core) through
    # the B-major passes: their partials of d are added with the caller's scale and output
    ranks = (8,) * len(dims)
    X, P, Z0, prob = _setup(dims, ranks, prec=prec)
    sigma = 1.2
    cores = device_cores(Z0, F32)
    grads = prob.loss_bwd(cores, sigma)
    gref = aw.loss_grads(X, P, Z0, sigma)
    errs = [rel(g, r) for g, r in zip(host_cores(grads, dims, ranks), gref)]
    print(f"{prec} backward on {dims}: relative errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= 2e-2, errs


# B-major edge cases for core 0: slices of exactly one 64-row block (no block straddles two
# slices), of 65 rows (almost every block straddles), and a single slice (I_0 = 1)
B_MAJOR_EDGES = [(9, 64, 10, 11), (12, 65, 9, 10), (1, 80, 9, 11)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", B_MAJOR_EDGES)
def test_b_major_edge_shapes(dims, prec):
    ranks = (8,) * len(dims)
    X, P, Z0, prob = _setup(dims, ranks, prec=prec)
    split = prob.info()["split"]
    assert split[0] >= 1 and math.prod(dims[1:1 + split[0]]) >= 64, split
    sigma = 1.3
    d, stats = prob.grad(device_cores(Z0, F32), 0, sigma)
    _, info = aw.core_update(X, P, Z0, 0, sigma)
    got = unflatten_d(d.cpu().numpy(), ranks[0], dims[0], ranks[1])
    assert rel(got, info.d) <= 2e-2, rel(got, info.d)
    assert stats[2].item() == info.n_obs
    cores = device_cores(Z0, F32)
    eta, flags = prob.step(cores, 0, 1.1, 1e-9)
    ref, info = aw.core_update(X, P, Z0, 0, 1.1, 1e-9)
    assert int(flags) == 0
    assert rel(host_cores(cores, dims, ranks)[0], ref) <= 1e-2
    assert float(eta) == pytest.approx(info.eta, rel=3e-2)


@pytest.mark.parametrize("prec", PRECS)
def test_gradient_direction_step_on_b_major_rows(prec):
    # h = d (no Gram, no inverse): the per-slice kernel takes d itself as the direction
    dims, ranks = (20, 70, 20, 20), (8, 8, 8, 8)
    X, P, Z0, prob = _setup(dims, ranks, prec=prec)
    prob.set_variant("gradient", "global")
    cores = device_cores(Z0, F32)
    eta, flags = prob.step(cores, 0, 1.1, 1e-9)
    ref, info = aw.core_update(X, P, Z0, 0, 1.1, 1e-9, direction="gradient")
    assert int(flags) == 0
    assert rel(host_cores(cores, dims, ranks)[0], ref) <= 1e-2
    assert float(eta) == pytest.approx(info.eta, rel=3e-2)


def test_not_spd_gram_on_b_major_rows_leaves_the_core():
    # the first column of every slice of core 3 is zero, so is the first column of every
    # subchain product of core 0: G^{!=0} (64 x 64) has rank 56, with lambda = 0 the inverse
    # fails, the step reports it, takes eta = 0 and leaves core 0 as it was (d is not zero)
    dims, ranks = (20, 70, 20, 20), (8, 8, 8, 8)
    X, P, Z0, prob = _setup(dims, ranks, prec="bf16")
    Z = [z.copy() for z in Z0]
    Z[3][:, :, 0] = 0.0  # r_3 x I_3 x r_0
    assert np.linalg.matrix_rank(aw.gram_fgmc(Z, 0)) < 64
    cores = device_cores(Z, F32)
    eta, flags = prob.step(cores, 0, math.inf, 0.0)
    assert int(flags) & trd.TRD_FLAG_NOTSPD
    assert float(eta) == 0.0
    np.testing.assert_array_equal(host_cores(cores, dims, ranks)[0], np.asarray(Z[0], np.float32))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_bf16_step(dims, ranks, prec):
    X, P, Z0, prob = _setup(dims, ranks, prec=prec)
    sigma = 1.1
    for k in range(len(dims)):
        cores = device_cores(Z0, F32)
        eta, flags = prob.step(cores, k, sigma, 1e-9)
        ref, info = aw.core_update(X, P, Z0, k, sigma, 1e-9)
        got = host_cores(cores, dims, ranks)
        assert int(flags) == 0
        assert rel(got[k], ref) <= 1e-2, (k, rel(got[k], ref))
        assert float(eta) == pytest.approx(info.eta, rel=3e-2)


@pytest.mark.parametrize("prec", PRECS)
def test_bf16_loss_and_quantile_sigma(prec):
    dims, ranks = (40, 30, 20), (3, 3, 3)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5, prec=prec)
    cores = device_cores(Z0, F32)
    L = float(prob.loss_fwd(cores, 0.8))
    assert L == pytest.approx(aw.loss(X, P, Z0, 0.8), rel=1e-2)
    rep = prob.fit(cores, max_sweeps=1, tol=0.0, precision=prec)
    e = aw.residual_abs(X, P, Z0)
    s_ref = aw.quantile_sigma(e, 0.5, 5.0, 1e-6 * float(np.max(np.abs(X[P.astype(bool)]))))
    assert rep["sigma"][0] == pytest.approx(s_ref, rel=1e-2)


def test_bf16_fit_recovers_like_fp32():
    # exact-rank data with outliers: BF16 and FP32 sweeps from the same start reach
    # recovery errors within 1e-2 of each other (the BF16 plateau is stated in DESIGN)
    import synth
    w = synth.scaled(synth.WORKLOADS["tr3_30_r3"], (24, 26, 22))
    w = synth.Workload(w.name, w.dims, w.ranks, w.rho, w.outlier_frac, w.outlier_law, w.outlier_scale,
                       core_std=1.0)
    Zt, xstar, P, X = synth.make_workload(w, 3, tr.reconstruct)
    X = X.astype(F32).astype(np.float64)
    Z0 = [z.astype(F32).astype(np.float64) for z in synth.perturbed_cores(Zt, 3, rel=0.2)]
    out = {}
    for prec in ("native", "bf16", "bf16x3"):
        prob = device_problem(X, P, w.dims, w.ranks, F32)
        cores = device_cores(Z0, F32)
        prob.fit(cores, max_sweeps=40, tol=0.0, precision=prec)
        out[prec] = aw.relative_error(host_cores(cores, w.dims, w.ranks), xstar)
    print("recovery error fp32 %.3e bf16 %.3e bf16x3 %.3e" % (out["native"], out["bf16"],
                                                             out["bf16x3"]))
    assert out["native"] < 1e-3
    assert abs(out["bf16"] - out["native"]) <= 1e-2
    # the split reconstruction removes the bf16 residual floor
    assert abs(out["bf16x3"] - out["native"]) <= 1e-4
