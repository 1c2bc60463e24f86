"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded inputs.

Sizes are small enough for the oracle yet span several 256-row groups, several column
tiles and ragged tails.  Bars: bit-exact for index sampling; FP32 per-step relative
Frobenius error <= 1e-5 (teacher forced: both sides start from the same FP32 cores);
FP64 problems to 1e-10."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import synth  # noqa: E402
from oracle import awrtrd as aw  # noqa: E402
from oracle import rng as orng  # noqa: E402
from oracle import tr  # noqa: E402
import paper_2305_09044_amd as trd  # noqa: E402
from _helpers import device_cores, device_problem, host_cores, host_problem, rel, unflatten_d  # noqa: E402

F32, F64 = np.float32, np.float64
TOL = {F32: 1e-5, F64: 1e-10}

SHAPES = [
    # (dims, ranks) -- several tiles / ragged tails / N = 2..5 / non-uniform ranks
    ((30, 30, 30), (3, 3, 3)),
    ((37, 41, 29, 23), (2, 3, 4, 2)),
    ((300, 257), (4, 3)),
    ((9, 10, 11, 8, 7), (2, 2, 3, 2, 2)),
    ((70, 60, 50), (5, 5, 5)),          # 3000-column rows: several column tiles
]


def _setup(dims, ranks, rho=0.4, seed=0, dtype=F32, **kw):
    X, P, Z0, Zt, xstar = host_problem(dims, ranks, rho, seed, dtype, reconstruct=tr.reconstruct, **kw)
    prob = device_problem(X, P, dims, ranks, dtype)
    return X, P, Z0, prob


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_reconstruct(dims, ranks, dtype):
    X, P, Z0, prob = _setup(dims, ranks, dtype=dtype)
    cores = device_cores(Z0, dtype)
    full = prob.reconstruct(cores).cpu().numpy()
    ref = tr.reconstruct(Z0).ravel(order="F")
    assert rel(full, ref) <= (1e-6 if dtype == F32 else 1e-13)
    g = np.random.default_rng(1)
    lin = g.integers(0, ref.size, 257)
    part = prob.reconstruct(cores, torch.from_numpy(lin).to("cuda")).cpu().numpy()
    np.testing.assert_allclose(part, tr.reconstruct_at(Z0, lin), rtol=1e-5 if dtype == F32 else 1e-12,
                               atol=1e-6 if dtype == F32 else 1e-13)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_weights(dtype):
    e = np.linspace(-4, 4, 1001).astype(dtype)
    ed = torch.from_numpy(e).to("cuda")
    for s in (0.3, 2.0, math.inf):
        w = trd.trd_weights(ed, s).cpu().numpy()
        # exp(-u) inherits a relative error of about u * eps from rounding of its argument
        # u = e^2 / 2 sigma^2 (up to ~90 here); FP32 results below FLT_MIN are subnormal
        np.testing.assert_allclose(w, aw.weights(e.astype(np.float64), s), rtol=1e-5 if dtype == F32 else 5e-14,
                                   atol=1e-37 if dtype == F32 else 1e-300)
    with pytest.raises(trd.TrdError):
        trd.trd_weights(ed, 0.0)
    with pytest.raises(trd.TrdError):
        trd.trd_weights(ed, float("nan"))


@pytest.mark.parametrize("seed,t,k", [(0, 0, 0), (7, 3, 2), (123456789, 29, 1), (2**63 + 5, 1, 3)])
def test_sample_sketch_bit_exact(seed, t, k):
    dims, sizes = (100, 240, 3, 320), (20, 32, 3, 7)
    got = trd.trd_sample_sketch(seed, t, k, dims, sizes)
    ref = orng.sketch_indices(seed, t, k, dims, sizes)
    for j in range(4):
        assert got[j].cpu().numpy().tolist() == ref[j], j


@pytest.mark.parametrize("dims,sizes", [((262144, 300000, 5), (900, 300, 4)),    # LDS bitmap / global list
                                        ((70000, 33, 2), (69999, 32, 1)),        # nearly every index
                                        ((1, 64, 65), (1, 63, 1))])
def test_sample_sketch_bit_exact_large_and_edge_sizes(dims, sizes):
    for k in range(3):
        got = trd.trd_sample_sketch(5, 2, k, dims, sizes)
        ref = orng.sketch_indices(5, 2, k, dims, sizes)
        for j in range(3):
            assert got[j].cpu().numpy().tolist() == ref[j], (k, j)


@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_fgmc_gram(dims, ranks):
    X, P, Z0, prob = _setup(dims, ranks)
    cores = device_cores(Z0, F32)
    for k in range(len(dims)):
        G = prob.fgmc_gram(cores, k).cpu().numpy()
        assert rel(G, aw.gram_explicit(Z0, k)) <= 1e-12


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_grad_full(dims, ranks, dtype):
    X, P, Z0, prob = _setup(dims, ranks, dtype=dtype)
    cores = device_cores(Z0, dtype)
    sigma = 1.3
    for k in range(len(dims)):
        d, stats = prob.grad(cores, k, sigma)
        _, info = aw.core_update(X, P, Z0, k, sigma)
        got = unflatten_d(d.cpu().numpy(), ranks[k], dims[k], ranks[(k + 1) % len(dims)])
        assert rel(got, info.d) <= 3 * TOL[dtype], k
        s = stats.cpu().numpy()
        assert s[2] == info.n_obs
        assert s[0] == pytest.approx(info.loss, rel=1e-5 if dtype == F32 else 1e-11)
        assert s[1] == pytest.approx(info.wls, rel=1e-5 if dtype == F32 else 1e-11)


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_step_full_teacher_forced(dims, ranks, dtype):
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
        for j in range(len(dims)):
            if j != k:
                np.testing.assert_array_equal(got[j], Z0[j])


@pytest.mark.parametrize("explicit", [True, False])
def test_step_sketch(explicit):
    dims, ranks = (60, 50, 40, 30), (3, 4, 3, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    sizes = (12, 9, 17, 8)
    sigma, seed, t = 0.9, 42, 3
    for k in range(4):
        idx = orng.sketch_indices(seed, t, k, dims, sizes)
        if explicit:
            dev = [None if j == k else torch.tensor(idx[j], dtype=torch.int32, device="cuda") for j in range(4)]
            sk, keep = trd.make_sketch(sizes, seed, t, dev)
        else:
            sk, keep = trd.make_sketch(sizes, seed, t)
        cores = device_cores(Z0, F32)
        eta, flags = prob.step(cores, k, sigma, 1e-9, sketch=sk)
        ref, info = aw.core_update(X, P, Z0, k, sigma, 1e-9, sketch=idx)
        got = host_cores(cores, dims, ranks)
        assert rel(got[k], ref) <= 1e-5, k
        assert float(eta) == pytest.approx(info.eta, rel=1e-4)


def test_step_sketch_clamps_out_of_range_caller_lists_and_flags_them():
    # a caller's list with indices outside [0, I_j): the step runs on the clamped lists and
    # raises TRD_FLAG_CLAMPED (the same lists in range give the same core, without the flag)
    dims, ranks = (30, 25, 20), (2, 3, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    bad = [None, torch.tensor([-3, 4, 7, 40], dtype=torch.int32, device="cuda"),
           torch.tensor([0, 5, 19, 25], dtype=torch.int32, device="cuda")]
    good = [None, torch.tensor([0, 4, 7, 24], dtype=torch.int32, device="cuda"),
            torch.tensor([0, 5, 19, 19], dtype=torch.int32, device="cuda")]
    a, b = device_cores(Z0, F32), device_cores(Z0, F32)
    sk, keep = trd.make_sketch((30, 4, 4), 3, 0, bad)
    _, fa = prob.step(a, 0, 0.9, sketch=sk)
    sk2, keep2 = trd.make_sketch((30, 4, 4), 3, 0, good)
    _, fb = prob.step(b, 0, 0.9, sketch=sk2)
    assert int(fa) & trd.TRD_FLAG_CLAMPED and not int(fb) & trd.TRD_FLAG_CLAMPED
    assert torch.equal(a[0], b[0])
    _, fc = prob.step(device_cores(Z0, F32), 0, 0.9)   # the next step starts clean
    assert not int(fc) & trd.TRD_FLAG_CLAMPED


ORACLE_GRAM = {"global": "fgmc", "local": "local"}


@pytest.mark.parametrize("direction,gram", [("gradient", "global"), ("scaled", "local"),
                                            ("gradient", "local")])
def test_step_sketch_ablation_variants(direction, gram):
    # Sec. 6.1 ablations: h = d, or the Gram matrix of the sampled cores
    dims, ranks = (60, 50, 40, 30), (3, 4, 3, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    sizes = (12, 9, 17, 8)
    sigma, seed, t = 0.9, 42, 3
    prob.set_variant(direction, gram)
    for k in range(4):
        idx = orng.sketch_indices(seed, t, k, dims, sizes)
        sk, keep = trd.make_sketch(sizes, seed, t)
        cores = device_cores(Z0, F32)
        eta, flags = prob.step(cores, k, sigma, 1e-9, sketch=sk)
        ref, info = aw.core_update(X, P, Z0, k, sigma, 1e-9, sketch=idx, gram=ORACLE_GRAM[gram],
                                   direction=direction)
        got = host_cores(cores, dims, ranks)
        assert int(flags) == 0
        assert rel(got[k], ref) <= 1e-5, (k, rel(got[k], ref))
        assert float(eta) == pytest.approx(info.eta, rel=1e-4)


@pytest.mark.parametrize("dims,ranks", SHAPES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_step_full_gradient_direction(dims, ranks, dtype):
    X, P, Z0, prob = _setup(dims, ranks, dtype=dtype)
    prob.set_variant("gradient", "global")
    for k in range(len(dims)):
        cores = device_cores(Z0, dtype)
        eta, flags = prob.step(cores, k, 1.1, 1e-9)
        ref, info = aw.core_update(X, P, Z0, k, 1.1, 1e-9, direction="gradient")
        got = host_cores(cores, dims, ranks)
        assert int(flags) == 0
        assert rel(got[k], ref) <= TOL[dtype], (k, rel(got[k], ref))
        assert float(eta) == pytest.approx(info.eta, rel=1e-4 if dtype == F32 else 1e-9)


def test_local_gram_without_sketch_is_the_method():
    dims, ranks = (37, 41, 29, 23), (2, 3, 4, 2)
    X, P, Z0, prob = _setup(dims, ranks)
    for k in range(4):
        a, b = device_cores(Z0, F32), device_cores(Z0, F32)
        prob.set_variant("scaled", "global")
        prob.step(a, k, 0.9)
        prob.set_variant("scaled", "local")
        prob.step(b, k, 0.9)
        assert torch.equal(a[k], b[k])
    lib = trd._lib.load()
    assert lib.trd_set_variant(prob._ctx, 2, 0, 0) == -1   # TRD_EINVAL
    assert lib.trd_set_variant(prob._ctx, 0, 2, 0) == -1


@pytest.mark.parametrize("direction,gram", [("gradient", "global"), ("scaled", "local")])
def test_fit_rsts_ablation_variants(direction, gram):
    dims, ranks = (40, 36, 30, 24), (3, 3, 2, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    sizes, seed, sig = (10, 8, 9, 7), 7, [2.0, 1.2, 0.9]
    prob.set_variant(direction, gram)
    cores = device_cores(Z0, F32)
    rep = prob.fit(cores, max_sweeps=len(sig), tol=0.0, sigma_mode="given", sigma_given=sig,
                   sketch_sizes=sizes, seed=seed)
    ref, hist = aw.fit(X, P, Z0, aw.FitOptions(max_sweeps=len(sig), tol=0.0, sigma_mode="given",
                                               sigma_given=sig, sketch_sizes=sizes, seed=seed,
                                               gram=ORACLE_GRAM[gram], direction=direction))
    got = host_cores(cores, dims, ranks)
    err = max(rel(g, r) for g, r in zip(got, ref))
    assert err <= 1e-4, err
    # the stop test uses D^t with the Gram of the full cores whatever the variant
    for a, b in zip(rep["e"][1:], hist["e"][1:]):
        assert a == pytest.approx(b, rel=1e-3)
    # and stops where the oracle stops: a tolerance just above the change after sweep 2
    tol = 1.01 * max(hist["e"][1:])
    rep = prob.fit(device_cores(Z0, F32), max_sweeps=len(sig), tol=tol, sigma_mode="given",
                   sigma_given=sig, sketch_sizes=sizes, seed=seed)
    _, hist = aw.fit(X, P, Z0, aw.FitOptions(max_sweeps=len(sig), tol=tol, sigma_mode="given",
                                             sigma_given=sig, sketch_sizes=sizes, seed=seed,
                                             gram=ORACLE_GRAM[gram], direction=direction))
    assert rep["sweeps"] == len(hist["e"]) == 2


@pytest.mark.parametrize("dtype", [F32, F64])
def test_full_observation_ls_step_is_tr_als(dtype):
    # TR-ALS as a special case of the step: P = 1, sigma = inf, lambda = 0 give eta = 1 and
    # the least-squares solution of each core given the others (textbook lstsq)
    dims, ranks = (21, 17, 13, 9), (2, 3, 2, 3)
    X, _, Z0, _ = _setup(dims, ranks, dtype=dtype)
    P = np.ones(dims, dtype=np.uint8)
    prob = device_problem(X, P, dims, ranks, dtype)
    for k in range(4):
        cores = device_cores(Z0, dtype)
        eta, flags = prob.step(cores, k, math.inf, 0.0)
        got = host_cores(cores, dims, ranks)
        A = tr.subchain_unfolding(Z0, k)
        sol = np.linalg.lstsq(A, tr.unfold_cyclic(X, k).T, rcond=None)[0].T
        assert int(flags) == 0
        assert float(eta) == pytest.approx(1.0, abs=1e-5 if dtype == F32 else 1e-10)
        assert rel(tr.unfold_core(got[k]), sol) <= (1e-5 if dtype == F32 else 1e-9), k


def test_sketch_with_full_sizes_equals_full_step():
    dims, ranks = (20, 15, 12), (2, 3, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    for k in range(3):
        a = device_cores(Z0, F32)
        b = device_cores(Z0, F32)
        prob.step(a, k, 0.8)
        sk, _ = trd.make_sketch(dims, 5, 0)
        prob.step(b, k, 0.8, sketch=sk)
        ha, hb = host_cores(a, dims, ranks), host_cores(b, dims, ranks)
        assert rel(ha[k], hb[k]) <= 1e-6


def test_unobserved_values_never_used():
    dims, ranks = (33, 20, 17), (3, 2, 3)
    X, P, Z0, _ = _setup(dims, ranks)
    X2 = X.copy()
    X2[P == 0] = 3.0e4
    out = []
    for XX in (X, X2):
        prob = device_problem(XX, P, dims, ranks, F32)
        cores = device_cores(Z0, F32)
        for k in range(3):
            prob.step(cores, k, 0.7)
        out.append(host_cores(cores, dims, ranks))
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_empty_mask_gives_zero_step_and_flag():
    dims, ranks = (10, 12, 9), (2, 2, 2)
    X, P, Z0, _ = _setup(dims, ranks)
    P0 = np.zeros_like(P)
    prob = device_problem(X, P0, dims, ranks, F32)
    cores = device_cores(Z0, F32)
    eta, flags = prob.step(cores, 0, 1.0)
    assert float(eta) == 0.0
    assert int(flags) & trd.TRD_FLAG_EMPTY
    np.testing.assert_array_equal(host_cores(cores, dims, ranks)[0], Z0[0])


def test_not_positive_definite_flag():
    # I_j = 1 for the other modes: G^{!=k} has rank 1 < R^2, so with lambda = 0 it is singular
    dims, ranks = (8, 1, 1), (2, 2, 2)
    X, P, Z0, prob = _setup(dims, ranks, rho=1.0, outlier_frac=0.0)
    cores = device_cores(Z0, F32)
    eta, flags = prob.step(cores, 0, math.inf, 0.0)
    assert int(flags) & trd.TRD_FLAG_NOTSPD
    assert float(eta) == 0.0
    np.testing.assert_array_equal(host_cores(cores, dims, ranks)[0], Z0[0])


@pytest.mark.parametrize("dtype", [F32, F64])
def test_fit_given_sigma_matches_oracle(dtype):
    dims, ranks = (26, 31, 22), (3, 3, 3)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5, dtype=dtype)
    sig = [3.0, 2.0, 1.5, 1.0, 0.8, 0.6]
    cores = device_cores(Z0, dtype)
    rep = prob.fit(cores, max_sweeps=len(sig), tol=0.0, sigma_mode="given", sigma_given=sig)
    ref, hist = aw.fit(X, P, Z0, aw.FitOptions(max_sweeps=len(sig), tol=0.0, sigma_mode="given",
                                               sigma_given=sig))
    got = host_cores(cores, dims, ranks)
    err = max(rel(g, r) for g, r in zip(got, ref))
    assert err <= (1e-4 if dtype == F32 else 1e-9), err
    assert rep["sweeps"] == len(sig)
    for a, b in zip(rep["e"][1:], hist["e"][1:]):
        assert a == pytest.approx(b, rel=1e-3 if dtype == F32 else 1e-7)


def test_fit_quantile_sigma_first_sweep():
    dims, ranks = (40, 30, 20), (3, 3, 3)
    X, P, Z0, prob = _setup(dims, ranks, rho=0.5)
    cores = device_cores(Z0, F32)
    rep = prob.fit(cores, max_sweeps=1, tol=0.0)
    e = aw.residual_abs(X, P, Z0)
    s_ref = aw.quantile_sigma(e, 0.5, 5.0, 1e-6 * float(np.max(np.abs(X[P.astype(bool)]))))
    assert rep["sigma"][0] == pytest.approx(s_ref, rel=1e-5)


@pytest.mark.parametrize("precision,tol", [("native", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("q", [0.5, 0.9])
def test_quantile_sigma_when_most_keys_share_the_top_digit(precision, tol, q):
    # residuals all close to 1.125 (X = reconstruction of the start + 1.125): every key
    # shares the first radix digit, so the candidate segments of the third digit fill up
    dims, ranks = (64, 48, 40), (3, 4, 3)
    _, P, Z0, _ = _setup(dims, ranks, rho=0.6)
    X = (tr.reconstruct(Z0) + 1.125).astype(np.float32).astype(np.float64)
    prob = device_problem(X, P, dims, ranks, F32)
    cores = device_cores(Z0, F32)
    rep = prob.fit(cores, max_sweeps=1, tol=0.0, q=q, precision=precision)
    e = aw.residual_abs(X, P, Z0)
    assert np.mean((e >= 1.0) & (e < 1.25)) > 0.9   # one first digit: 0x3f8 in bits 31..21
    s_ref = aw.quantile_sigma(e, q, 5.0, 1e-6 * float(np.max(np.abs(X[P.astype(bool)]))))
    assert rep["sigma"][0] == pytest.approx(s_ref, rel=tol)


@pytest.mark.parametrize("sigma", [0.7, math.inf])
def test_loss_fwd_bwd(sigma):
    dims, ranks = (23, 19, 21, 6), (2, 3, 2, 2)
    X, P, Z0, prob = _setup(dims, ranks)
    cores = device_cores(Z0, F32)
    L = float(prob.loss_fwd(cores, sigma))
    assert L == pytest.approx(aw.loss(X, P, Z0, sigma), rel=1e-5)
    grads = prob.loss_bwd(cores, sigma)
    ref = aw.loss_grads(X, P, Z0, sigma)
    for k in range(4):
        g = host_cores(grads, dims, ranks)[k]
        assert rel(g, ref[k]) <= 3e-5, k


def test_autograd_function_fd():
    dims, ranks = (12, 12, 12, 12), (2, 2, 2, 2)
    X, P, Z0, prob = _setup(dims, ranks, dtype=F64)
    sigma = 0.9
    cores = [c.requires_grad_(True) for c in device_cores(Z0, F64)]
    L = trd.correntropy_loss(prob, cores, sigma)
    L.backward()
    g = [c.grad.detach().cpu().numpy() for c in cores]
    h = 1e-6
    rng = np.random.default_rng(0)
    for k in range(4):
        for idx in rng.integers(0, cores[k].numel(), 5):
            with torch.no_grad():
                cp = [c.detach().clone() for c in cores]
                cm = [c.detach().clone() for c in cores]
                cp[k][idx] += h
                cm[k][idx] -= h
                fd = (float(prob.loss_fwd(cp, sigma)) - float(prob.loss_fwd(cm, sigma))) / (2 * h)
            assert abs(g[k][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, idx, g[k][idx], fd)


@pytest.mark.parametrize("seed,dims,rho,block,frac", [
    (0, (30, 30, 30), 0.5, 0, 0.1),
    (7, (37, 41, 29, 23), 0.3, 0, 0.2),
    (2**63 + 11, (40, 36, 3, 7), 0.2, 16, 0.1),      # ragged 16 x 16 tiles, channel mode
    (5, (300, 257), 0.05, 0, 0.0),
    (9, (9, 10, 11, 8, 7), 1.0, 0, 1.0),
    (9, (9, 10, 11, 8, 7), 0.0, 0, 0.5),
    (4, (17, 33, 5), 0.4, 4, 0.15),
])
def test_sample_mask_bit_exact(seed, dims, rho, block, frac):
    m, s, u = trd.trd_sample_mask(seed, dims, rho, block, frac, outliers=True, uniforms=True)
    rm, rs, ru = orng.sample_mask(seed, dims, rho, block, frac)
    np.testing.assert_array_equal(m.cpu().numpy(), rm)
    np.testing.assert_array_equal(s.cpu().numpy(), rs)
    np.testing.assert_array_equal(u.cpu().numpy(), ru)
    # the mask alone (no optional outputs) is the same
    m2, _, _ = trd.trd_sample_mask(seed, dims, rho, block, frac)
    assert torch.equal(m, m2)


@pytest.mark.parametrize("dims,ranks", [((20, 18, 16), (3, 3, 3)), ((9, 10, 11, 8), (2, 3, 2, 2))])
def test_fit_with_the_als_options_runs_tr_als_sweeps(dims, ranks):
    # trd_fit with P = 1, sigma = inf, lambda = 0 runs TR-ALS: two sweeps equal two sweeps of
    # per-core least-squares solves on the explicit unfoldings (Thm. 1), every eta = 1
    g = np.random.default_rng(5)
    X = g.standard_normal(dims)
    P = np.ones(dims, dtype=np.uint8)
    Z0 = synth.init_cores(dims, ranks, 5)
    prob = device_problem(X, P, dims, ranks, F64)
    cores = device_cores(Z0, F64)
    rep = prob.fit(cores, max_sweeps=2, tol=0.0, sigma_mode="fixed", sigma=math.inf, lambda_rel=0.0)
    Z = [z.copy() for z in Z0]
    for _ in range(2):
        for k in range(len(dims)):
            A = tr.subchain_unfolding(Z, k)
            sol, *_ = np.linalg.lstsq(A, tr.unfold_cyclic(X, k).T, rcond=None)
            Z[k] = tr.fold_core(sol.T, ranks[k], ranks[(k + 1) % len(dims)])
    got = host_cores(cores, dims, ranks)
    assert max(rel(a, b) for a, b in zip(got, Z)) <= 1e-8
    assert all(abs(e - 1.0) < 1e-9 for sweep in rep["eta"] for e in sweep)
