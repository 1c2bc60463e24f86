"""Pins for the FP64 oracle: each check ties it to something other than itself
(brute force, a closed form, a textbook/library solution, an invariant, published
generator outputs), so a dropped term, a wrong sign, a wrong index or a transposed
operand anywhere in it fails at least one test.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import awrtrd as aw
from oracle import rng as orng
from oracle import tr

HERE = os.path.dirname(os.path.abspath(__file__))


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rand_cores(dims, ranks, seed, std=1.0):
    g = np.random.default_rng(seed)
    N = len(dims)
    return [g.standard_normal((ranks[j], dims[j], ranks[(j + 1) % N])) * std for j in range(N)]


CASES = [((3, 4, 5), (2, 3, 2)), ((3, 4, 2, 3), (2, 3, 2, 3)), ((2, 3, 2, 2, 3), (1, 2, 3, 2, 2)),
         ((4, 5), (3, 2))]


# ---------------------------------------------------------------- TR format (Def. 1-2, Thm. 1)

@pytest.mark.parametrize("dims,ranks", CASES)
def test_merge_reconstruction_equals_bruteforce(dims, ranks):
    Z = rand_cores(dims, ranks, 1)
    np.testing.assert_allclose(tr.reconstruct(Z), tr.reconstruct_bruteforce(Z), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_cyclic_shift_invariance(dims, ranks):
    # R(Z_2..Z_N, Z_1)[i_2..i_N, i_1] = R(Z)[i_1..i_N]  (trace is cyclic)
    Z = rand_cores(dims, ranks, 2)
    X = tr.reconstruct(Z)
    Xs = tr.reconstruct(Z[1:] + Z[:1])
    np.testing.assert_allclose(np.moveaxis(Xs, -1, 0), X, rtol=1e-12, atol=1e-12)


def test_rank_one_is_outer_product():
    g = np.random.default_rng(3)
    vs = [g.standard_normal(n) for n in (3, 4, 5)]
    Z = [v.reshape(1, -1, 1) for v in vs]
    np.testing.assert_allclose(tr.reconstruct(Z), np.multiply.outer(np.multiply.outer(vs[0], vs[1]), vs[2]),
                               rtol=1e-13)


def test_reconstruct_layout_is_column_major():
    Z = rand_cores((3, 4, 5), (2, 2, 2), 4)
    X = tr.reconstruct(Z)
    lin = np.array([0, 1, 3, 7, 59])
    np.testing.assert_allclose(X.ravel(order="F")[lin], tr.reconstruct_at(Z, lin), rtol=1e-12)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_theorem1_unfolding(dims, ranks):
    Z = rand_cores(dims, ranks, 5)
    X = tr.reconstruct(Z)
    for k in range(len(dims)):
        A = tr.subchain_unfolding(Z, k)
        np.testing.assert_allclose(tr.unfold_cyclic(X, k), tr.unfold_core(Z[k]) @ A.T, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(tr.fold_cyclic(tr.unfold_cyclic(X, k), k, dims), X)


def test_subchain_row_by_hand():
    dims, ranks = (3, 4, 2, 3), (2, 3, 2, 3)
    Z = rand_cores(dims, ranks, 6)
    k = 1
    A = tr.subchain_unfolding(Z, k)
    # row for (i_2, i_3, i_0) = (1, 2, 2): little-endian in the cyclic order 2, 3, 0
    i2, i3, i0 = 1, 2, 2
    m = i2 + dims[2] * (i3 + dims[3] * i0)
    Am = Z[2][:, i2, :] @ Z[3][:, i3, :] @ Z[0][:, i0, :]    # r_2 x r_1
    rk = ranks[k]
    for a in range(ranks[k]):
        for b in range(ranks[k + 1]):
            assert abs(A[m, a + b * rk] - Am[b, a]) < 1e-12


def test_core_unfold_roundtrip_and_layout():
    Z = rand_cores((4,), (3,), 7)[0][:, :, :2] if False else np.random.default_rng(7).standard_normal((3, 4, 2))
    U = tr.unfold_core(Z)
    assert U.shape == (4, 6)
    assert U[2, 1 + 1 * 3] == Z[1, 2, 1]
    np.testing.assert_array_equal(tr.fold_core(U, 3, 2), Z)


# ---------------------------------------------------------------- weights (eq. 7) and loss

def test_weight_properties():
    e = np.linspace(-5, 5, 101)
    w = aw.weights(e, 1.3)
    assert np.all(w > 0) and np.all(w <= 1)
    assert aw.weights(np.array([0.0]), 0.7)[0] == 1.0
    # half-height at |e| = sigma sqrt(2 ln 2)
    s = 0.9
    assert abs(aw.weights(np.array([s * math.sqrt(2 * math.log(2))]), s)[0] - 0.5) < 1e-14
    assert np.all(aw.weights(e, math.inf) == 1.0)
    # large sigma tends to the least-squares weights (sec. 4.1)
    assert np.max(np.abs(aw.weights(e, 1e8) - 1)) < 1e-14


def test_welsch_limits():
    e = np.array([0.0, 1e-4, 0.3, 2.0])
    np.testing.assert_allclose(aw.welsch(e, 1e6), 0.5 * e * e, rtol=1e-9)
    np.testing.assert_array_equal(aw.welsch(e, math.inf), 0.5 * e * e)
    # bounded by sigma^2 for gross errors (the robustness of eq. 4)
    assert aw.welsch(np.array([1e3]), 2.0)[0] == pytest.approx(4.0)


# ---------------------------------------------------------------- gradient (eq. 9)

def _masked_problem(dims, ranks, seed, rho=0.6):
    g = np.random.default_rng(seed)
    Z = rand_cores(dims, ranks, seed, 0.7)
    P = (g.random(dims) < rho).astype(np.uint8)
    X = tr.reconstruct(rand_cores(dims, ranks, seed + 100, 0.7)) + 0.1 * g.standard_normal(dims)
    return Z, P, X


@pytest.mark.parametrize("sigma", [0.8, math.inf])
def test_gradient_is_minus_fd_of_frozen_weight_objective(sigma):
    dims, ranks = (3, 4, 3, 2), (2, 3, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 11)
    k = 2
    _, info = aw.core_update(X, P, Z, k, sigma, lambda_rel=1e-9)
    W = info.W
    A = tr.subchain_unfolding(Z, k)
    Pk = tr.unfold_cyclic(P, k).astype(bool)
    Xk = np.where(Pk, tr.unfold_cyclic(X, k), 0)

    def f(Zk2):  # 1/2 || sqrt(W) o P o (X - Z A^T) ||^2 with W frozen (eq. 8)
        E = np.where(Pk, Xk - Zk2 @ A.T, 0)
        return 0.5 * np.sum(W * E * E)

    Zk2 = tr.unfold_core(Z[k])
    fd = np.zeros_like(Zk2)
    h = 1e-6
    for idx in np.ndindex(*Zk2.shape):
        Zp = Zk2.copy(); Zp[idx] += h
        Zm = Zk2.copy(); Zm[idx] -= h
        fd[idx] = (f(Zp) - f(Zm)) / (2 * h)
    np.testing.assert_allclose(info.d, -fd, rtol=1e-6, atol=1e-8)


def test_loss_grads_match_finite_differences():
    dims, ranks = (3, 3, 4), (2, 2, 3)
    Z, P, X = _masked_problem(dims, ranks, 12)
    sigma = 0.5
    grads = aw.loss_grads(X, P, Z, sigma)
    h = 1e-6
    for k in range(3):
        for idx in [(0, 0, 0), (1, 2, 1), (Z[k].shape[0] - 1, 1, Z[k].shape[2] - 1)]:
            Zp = [z.copy() for z in Z]; Zp[k][idx] += h
            Zm = [z.copy() for z in Z]; Zm[k][idx] -= h
            fd = (aw.loss(X, P, Zp, sigma) - aw.loss(X, P, Zm, sigma)) / (2 * h)
            assert abs(grads[k][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, idx, grads[k][idx], fd)


def test_unobserved_values_never_used():
    dims, ranks = (3, 4, 3), (2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 13)
    X2 = X.copy()
    X2[P == 0] = 1e30
    a, ia = aw.core_update(X, P, Z, 1, 0.7)
    b, ib = aw.core_update(X2, P, Z, 1, 0.7)
    np.testing.assert_array_equal(a, b)
    assert ia.eta == ib.eta


# ---------------------------------------------------------------- FGMC (eq. 13)

@pytest.mark.parametrize("dims,ranks", CASES)
def test_fgmc_equals_explicit_gram(dims, ranks):
    Z = rand_cores(dims, ranks, 21)
    for k in range(len(dims)):
        Ge = aw.gram_explicit(Z, k)
        Gf = aw.gram_fgmc(Z, k)
        np.testing.assert_allclose(Gf, Ge, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(Gf, Gf.T, rtol=1e-12, atol=1e-12)
        assert np.min(np.linalg.eigvalsh(Gf)) > -1e-9 * np.max(np.abs(Gf))


@pytest.mark.parametrize("dims,ranks", CASES)
def test_fgmc_trace_identities(dims, ranks):
    Z = rand_cores(dims, ranks, 22)
    X = tr.reconstruct(Z)
    nrm2 = float(np.sum(X * X))
    K = [aw.fgmc_factor(z) for z in Z]
    P = K[0]
    for Kj in K[1:]:
        P = P @ Kj
    assert np.trace(P) == pytest.approx(nrm2, rel=1e-11)
    for k in range(len(dims)):
        Zk = tr.unfold_core(Z[k])
        assert np.trace(Zk @ aw.gram_fgmc(Z, k) @ Zk.T) == pytest.approx(nrm2, rel=1e-11)


def test_fgmc_factor_by_hand():
    Z = np.random.default_rng(23).standard_normal((2, 3, 3))
    K = aw.fgmc_factor(Z)
    # K[(a r + a'), (b r' + b')] = sum_i Z(i)[a, b] Z(i)[a', b']
    a, a2, b, b2 = 1, 0, 2, 1
    ref = sum(Z[a, i, b] * Z[a2, i, b2] for i in range(3))
    assert K[a * 2 + a2, b * 3 + b2] == pytest.approx(ref, rel=1e-14)


# ---------------------------------------------------------------- step (eqs. 10-12)

@pytest.mark.parametrize("k", [0, 1, 3])
def test_full_ls_step_is_tr_als(k):
    # P = 1, sigma = inf, lambda = 0: eta = 1 and Z + eta h solves the LS problem (1)
    dims, ranks = (3, 4, 3, 4), (2, 2, 3, 2)
    Z = rand_cores(dims, ranks, 31, 0.8)
    X = np.random.default_rng(32).standard_normal(dims)
    P = np.ones(dims, dtype=np.uint8)
    new, info = aw.core_update(X, P, Z, k, math.inf, lambda_rel=0.0)
    assert info.eta == pytest.approx(1.0, abs=1e-10)
    A = tr.subchain_unfolding(Z, k)
    sol = np.linalg.lstsq(A, tr.unfold_cyclic(X, k).T, rcond=None)[0].T
    np.testing.assert_allclose(tr.unfold_core(new), sol, rtol=1e-8, atol=1e-9)


def _wls(X, P, Z, k, W, Zk2):
    A = tr.subchain_unfolding(Z, k)
    Pk = tr.unfold_cyclic(P, k).astype(bool)
    E = np.where(Pk, tr.unfold_cyclic(X, k) - Zk2 @ A.T, 0)
    return 0.5 * np.sum(W * E * E)


@pytest.mark.parametrize("sigma", [0.6, math.inf])
def test_eta_is_exact_line_minimiser_and_decreases(sigma):
    dims, ranks = (4, 3, 3, 2), (2, 3, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 33)
    k = 1
    new, info = aw.core_update(X, P, Z, k, sigma, lambda_rel=1e-6)
    Zk2 = tr.unfold_core(Z[k])
    # fit a parabola through three points of L(Z + t h) and locate its minimum
    ts = np.array([0.0, 0.5, 1.0]) * 2 * info.eta
    Ls = [_wls(X, P, Z, k, info.W, Zk2 + t * info.h) for t in ts]
    c2, c1, _ = np.polyfit(ts, Ls, 2)
    assert -c1 / (2 * c2) == pytest.approx(info.eta, rel=1e-7)
    assert _wls(X, P, Z, k, info.W, tr.unfold_core(new)) < _wls(X, P, Z, k, info.W, Zk2)
    # the opposite sign (as printed in eq. 11) increases the objective
    assert _wls(X, P, Z, k, info.W, Zk2 - info.eta * info.h) > _wls(X, P, Z, k, info.W, Zk2)


def test_repeated_masked_steps_reach_rowwise_least_squares():
    # with W fixed (sigma = inf) repeating the step on one core converges to the
    # weighted masked LS solution, row by row (textbook lstsq)
    dims, ranks = (3, 4, 4, 3), (2, 2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 34, rho=0.7)
    k = 0
    cur = [z.copy() for z in Z]
    for _ in range(300):
        cur[k], info = aw.core_update(X, P, cur, k, math.inf, lambda_rel=1e-12)
    A = tr.subchain_unfolding(Z, k)
    Pk = tr.unfold_cyclic(P, k).astype(bool)
    Xk = tr.unfold_cyclic(X, k)
    ref = np.stack([np.linalg.lstsq(A[Pk[i]], Xk[i, Pk[i]], rcond=None)[0] for i in range(dims[k])])
    np.testing.assert_allclose(tr.unfold_core(cur[k]), ref, rtol=1e-6, atol=1e-7)


def test_gradient_direction_variant_also_descends():
    dims, ranks = (3, 3, 4), (2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 35)
    new, info = aw.core_update(X, P, Z, 2, 0.9, direction="gradient")
    assert _wls(X, P, Z, 2, info.W, tr.unfold_core(new)) < _wls(X, P, Z, 2, info.W, tr.unfold_core(Z[2]))


def test_gradient_direction_steps_along_d_with_exact_eta():
    # ablation of Sec. 6.1: h = d of eq. (15); eta of eq. (18) is still the exact minimiser
    dims, ranks = (4, 3, 3), (2, 2, 3)
    Z, P, X = _masked_problem(dims, ranks, 37)
    k = 0
    sk = orng.sketch_indices(9, 1, k, dims, (4, 2, 2))
    new, info = aw.core_update(X, P, Z, k, 0.7, sketch=sk, direction="gradient")
    np.testing.assert_array_equal(info.h, info.d)
    assert info.num == pytest.approx(float(np.sum(info.d * info.d)), rel=1e-14)
    Zs = [z[:, s, :] for z, s in zip(Z, sk)]
    Xs, Ps = X[np.ix_(*sk)], P[np.ix_(*sk)]
    Zk2 = tr.unfold_core(Z[k])
    ts = np.array([0.0, 0.5, 1.0]) * 2 * info.eta
    Ls = [_wls(Xs, Ps, Zs, k, info.W, Zk2 + t * info.d) for t in ts]
    c2, c1, _ = np.polyfit(ts, Ls, 2)
    assert -c1 / (2 * c2) == pytest.approx(info.eta, rel=1e-7)


def test_local_gram_is_fgmc_of_sampled_cores():
    # ablation of Sec. 6.1: the scaled term from the sampled cores.  A_I^T A_I must equal
    # the FGMC product (eq. 13) of the sampled cores' factors (a route through Kronecker
    # sums, pinned against A^T A above), differ from the global Gram, and equal it when
    # the sketch takes every index
    dims, ranks = (5, 4, 6, 3), (2, 3, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 38)
    k = 2
    sk = orng.sketch_indices(4, 0, k, dims, (3, 2, 6, 2))
    _, info = aw.core_update(X, P, Z, k, 0.8, sketch=sk, gram="local")
    Zs = [z[:, s, :] for z, s in zip(Z, sk)]
    np.testing.assert_allclose(info.G, aw.gram_fgmc(Zs, k), rtol=1e-12, atol=1e-12)
    assert np.linalg.norm(info.G - aw.gram_fgmc(Z, k)) > 1e-3 * np.linalg.norm(info.G)
    full = [list(range(n)) for n in dims]
    _, infg = aw.core_update(X, P, Z, k, 0.8, sketch=full, gram="local")
    np.testing.assert_allclose(infg.G, aw.gram_fgmc(Z, k), rtol=1e-12, atol=1e-12)
    # h solves (G_I + lambda I) h^T = d^T
    R2 = info.G.shape[0]
    lam = 1e-9 * np.trace(info.G) / R2
    np.testing.assert_allclose(info.h @ (info.G + lam * np.eye(R2)), info.d, rtol=1e-8, atol=1e-10)


def test_empty_update_gives_zero_step():
    dims, ranks = (3, 3, 3), (2, 2, 2)
    Z, _, X = _masked_problem(dims, ranks, 36)
    P = np.zeros(dims, dtype=np.uint8)
    new, info = aw.core_update(X, P, Z, 0, 1.0)
    assert info.eta == 0.0 and info.n_obs == 0
    np.testing.assert_array_equal(new, Z[0])


# ---------------------------------------------------------------- sweep / fit (Alg. 1)

def test_exact_rank_full_observation_fits_to_zero():
    dims, ranks = (6, 5, 7, 4), (2, 3, 2, 2)
    Zt = rand_cores(dims, ranks, 41, 0.8)
    X = tr.reconstruct(Zt)
    P = np.ones(dims, dtype=np.uint8)
    g = np.random.default_rng(42)
    Z0 = [z + 0.05 * g.standard_normal(z.shape) for z in Zt]
    opts = aw.FitOptions(max_sweeps=60, tol=0.0, sigma_mode="fixed", sigma=math.inf, lambda_rel=1e-13)
    Z, hist = aw.fit(X, P, Z0, opts)
    assert aw.relative_error(Z, X) < 1e-8


def test_convergence_matrix_invariants():
    dims, ranks = (3, 4, 5), (2, 3, 2)
    Z = rand_cores(dims, ranks, 43)
    D = aw.convergence_matrix(Z)
    X = tr.reconstruct(Z)
    np.testing.assert_allclose(D, D.T, rtol=1e-12, atol=1e-12)
    assert np.trace(D) == pytest.approx(float(np.sum(X * X)), rel=1e-12)
    Xn = tr.unfold_cyclic(X, 2)
    np.testing.assert_allclose(D, Xn @ Xn.T, rtol=1e-10, atol=1e-10)


def test_robust_fit_downweights_outliers():
    import synth
    w = synth.WORKLOADS["tr3_30_r3"]
    w = synth.scaled(w, (16, 16, 16))
    Zt, xstar, mask, X = synth.make_workload(w, 0, tr.reconstruct)
    sel, _ = synth.select_observed(mask, w.outlier_frac, 0)
    Z0 = synth.perturbed_cores(Zt, 0, rel=0.3)
    opts = aw.FitOptions(max_sweeps=40, tol=1e-9)
    Z, hist = aw.fit(X, mask, Z0, opts)
    assert aw.relative_error(Z, xstar) < 1e-3
    e = np.abs(X - tr.reconstruct(Z))
    wts = aw.weights(e, hist["sigma"][-1])
    assert np.all(wts[sel.astype(bool)] < 1e-3)


def test_rsts_with_full_sizes_equals_full_path():
    dims, ranks = (4, 3, 5), (2, 2, 3)
    Z, P, X = _masked_problem(dims, ranks, 44)
    a = aw.FitOptions(max_sweeps=2, tol=0, sigma_mode="fixed", sigma=0.9)
    b = aw.FitOptions(max_sweeps=2, tol=0, sigma_mode="fixed", sigma=0.9, sketch_sizes=dims)
    Za, _ = aw.fit(X, P, Z, a)
    Zb, _ = aw.fit(X, P, Z, b)
    for u, v in zip(Za, Zb):
        np.testing.assert_array_equal(u, v)


def test_rsts_step_uses_subtensor_identity():
    # eq. (14): the sketch of the reconstruction is the reconstruction of the sampled cores
    dims, ranks = (6, 5, 7), (2, 3, 2)
    Z = rand_cores(dims, ranks, 45)
    sk = orng.sketch_indices(3, 0, 1, dims, (3, 5, 4))
    X = tr.reconstruct(Z)
    np.testing.assert_allclose(X[np.ix_(*sk)], tr.reconstruct([z[:, s, :] for z, s in zip(Z, sk)]),
                               rtol=1e-12, atol=1e-12)


def test_quantile_rule():
    assert aw.quantile_sigma(np.array([5.0, 1.0, 3.0, 2.0, 4.0]), 0.5, 1.0, 0.0) == 3.0
    assert aw.quantile_sigma(np.array([5.0, 1.0, 3.0, 2.0]), 0.5, 2.0, 0.0) == 4.0   # rank floor(1.5) = 1
    assert aw.quantile_sigma(np.array([1e-9]), 0.5, 3.0, 1e-3) == 1e-3


# ---------------------------------------------------------------- sampling (RStS index sets)

def test_splitmix64_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64_kat.txt")) if l[0] != "#"]
    for seed, n, val in rows:
        seed, n, val = int(seed), int(n), int(val, 16)
        assert orng.splitmix64_stream(seed, n)[-1] == val
        assert orng.counter_u64(seed, n - 1) == val


def test_floyd_sample_properties():
    for key in range(50):
        s = orng.floyd_sample(orng.mix64(key), 37, 9)
        assert len(s) == 9 and s == sorted(set(s)) and 0 <= s[0] and s[-1] < 37
    assert orng.floyd_sample(5, 7, 7) == list(range(7))
    assert orng.floyd_sample(5, 7, 10) == list(range(7))


def test_floyd_inclusion_is_uniform():
    n, s, trials = 20, 5, 4000
    cnt = np.zeros(n)
    for t in range(trials):
        for i in orng.floyd_sample(orng.sketch_key(9, t, 0, 1), n, s):
            cnt[i] += 1
    expected = trials * s / n
    chi2 = np.sum((cnt - expected) ** 2 / expected)
    assert chi2 < 45.0        # 19 dof; p ~ 1e-3 threshold


def test_bounded_is_uniform_and_in_range():
    n = 7
    cnt = np.zeros(n)
    ctr = 0
    for _ in range(7000):
        v, ctr = orng.bounded(12345, ctr, n)
        cnt[v] += 1
    assert np.sum((cnt - 1000) ** 2 / 1000) < 22.5   # 6 dof


def test_sizes_from_J():
    assert orng.sizes_from_J(30000, (240, 320, 3, 200)) == [32, 32, 3, 32]
    assert orng.sizes_from_J(8000, (100, 100, 100, 100)) == [20, 20, 20, 20]
    assert orng.sizes_from_J(27, (9, 9, 9, 9)) == [3, 3, 3, 3]


@pytest.mark.parametrize("dims,ranks,k", [((6, 5, 7, 4), (2, 3, 2, 3), 1),
                                         ((5, 6, 4), (3, 2, 4), 2)])
def test_gradient_row_matches_unfolded_gradient(dims, ranks, k):
    # eq. (9) one row at a time (the form used on tensors too large to unfold) equals the
    # explicit (W o P o E) A of the full update, row by row and with non-square ranks
    Z, P, X = _masked_problem(dims, ranks, 5, rho=0.5)
    sigma = 0.7
    _, info = aw.core_update(X, P, Z, k, sigma)
    obs = np.argwhere(P.astype(bool))
    for i in range(dims[k]):
        sel = obs[obs[:, k] == i]
        row = aw.gradient_row(Z, k, sel, X[tuple(sel.T)], sigma, chunk=7)
        np.testing.assert_allclose(row, info.d[i], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- kernel-width schedule (own rule)
#
# The quantile rule is this project's reading of the adaptive kernel width the paper leaves to
# an earlier work; nothing in the paper fixes its values.  These pins fix the rule as stated:
# rank floor((n-1) q) of the sorted |e| over the observed entries of the sweep's first update,
# scaled by c, floored at sigma_min and at shrink * sigma_{t-1}.  Residuals are made exact by
# rank-1 cores of ones (every reconstructed entry is 1) and X = 1 + e with e(i, j, l) =
# i + 3 j + 6 l on a 3 x 2 x 2 tensor, so the sorted residuals can be written down by hand.

def _ones_problem():
    dims, ranks = (3, 2, 2), (1, 1, 1)
    Z = [np.ones((1, I, 1)) for I in dims]
    i, j, l = np.meshgrid(np.arange(3), np.arange(2), np.arange(2), indexing="ij")
    E = (i + 3 * j + 6 * l).astype(np.float64)          # residuals 0..11, each once
    return dims, Z, 1.0 + E, E


def test_sweep_sigma_by_hand_full_path():
    dims, Z, X, E = _ones_problem()
    P = np.ones(dims, dtype=np.uint8)
    o = aw.FitOptions(q=0.5, c=2.0, shrink=0.5)
    # 12 residuals 0..11: rank floor(11 * 0.5) = 5 -> |e| = 5, sigma = 2 * 5
    assert aw.sweep_sigma(X, P, Z, o, 0, 0.0) == 10.0
    # q = 0.9: rank floor(9.9) = 9 -> 9, sigma 18; q = 0 -> smallest residual 0 -> sigma_min
    assert aw.sweep_sigma(X, P, Z, aw.FitOptions(q=0.9, c=2.0), 0, 0.0) == 18.0
    assert aw.sweep_sigma(X, P, Z, aw.FitOptions(q=0.0, c=2.0), 0, 0.25) == 0.25
    # floor sigma_min above the quantile
    assert aw.sweep_sigma(X, P, Z, o, 0, 12.0) == 12.0
    # shrink limit: active when shrink * sigma_prev exceeds c * Q (30 * 0.5 = 15 > 10) ...
    assert aw.sweep_sigma(X, P, Z, o, 1, 0.0, sigma_prev=30.0) == 15.0
    # ... inactive when it does not (16 * 0.5 = 8 < 10), and absent at the first sweep
    assert aw.sweep_sigma(X, P, Z, o, 1, 0.0, sigma_prev=16.0) == 10.0
    assert aw.sweep_sigma(X, P, Z, o, 0, 0.0, sigma_prev=math.inf) == 10.0
    # shrink = 0 disables the limit
    assert aw.sweep_sigma(X, P, Z, aw.FitOptions(q=0.5, c=2.0, shrink=0.0), 1, 0.0, 30.0) == 10.0


def test_sweep_sigma_by_hand_masked_and_fixed_modes():
    dims, Z, X, E = _ones_problem()
    P = np.ones(dims, dtype=np.uint8)
    P[:, 0, 0] = 0                                       # drops residuals 0, 1, 2
    X = X.copy()
    X[P == 0] = 1e6                                      # never read
    # 9 residuals 3..11: rank floor(8 * 0.5) = 4 -> 7, sigma 2 * 7
    assert aw.sweep_sigma(X, P, Z, aw.FitOptions(q=0.5, c=2.0), 0, 0.0) == 14.0
    assert aw.sweep_sigma(X, P, Z, aw.FitOptions(sigma_mode="fixed", sigma=0.7), 3, 0.0, 9.0) == 0.7
    o = aw.FitOptions(sigma_mode="given", sigma_given=(3.0, 2.5, 1.0))
    assert [aw.sweep_sigma(X, P, Z, o, t, 0.0, 99.0) for t in range(3)] == [3.0, 2.5, 1.0]


@pytest.mark.parametrize("t", [0, 1, 4])
def test_sweep_sigma_by_hand_under_rsts(t):
    # under a sketch the quantile runs over the observed entries of the sweep's first update
    # (core 0: mode 0 whole, one sampled index in each of modes 1 and 2), so its residuals are
    # i + 3 j + 6 l for i = 0, 1, 2 at the drawn (j, l): median 1 + 3 j + 6 l
    dims, Z, X, E = _ones_problem()
    P = np.ones(dims, dtype=np.uint8)
    o = aw.FitOptions(q=0.5, c=2.0, sketch_sizes=(3, 1, 1), seed=17)
    sk = orng.sketch_indices(17, t, 0, dims, (3, 1, 1))
    assert sk[0] == [0, 1, 2] and len(sk[1]) == 1 and len(sk[2]) == 1
    j, l = sk[1][0], sk[2][0]
    assert aw.sweep_sigma(X, P, Z, o, t, 0.0) == 2.0 * (1 + 3 * j + 6 * l)


def test_fit_records_the_schedule_it_used():
    # the fit's sigma history follows the rule step by step: sweep 0 has no shrink limit;
    # later sweeps never fall below half the previous width
    import synth
    w = synth.scaled(synth.WORKLOADS["tr3_30_r3"], (12, 11, 10))
    Zt, xstar, mask, X = synth.make_workload(w, 2, tr.reconstruct)
    Z0 = synth.perturbed_cores(Zt, 2, rel=0.2)
    o = aw.FitOptions(max_sweeps=8, tol=0.0)
    Z, hist = aw.fit(X, mask, Z0, o)
    smin = 1e-6 * float(np.max(np.abs(X[mask.astype(bool)])))
    assert hist["sigma"][0] == aw.quantile_sigma(aw.residual_abs(X, mask, Z0), 0.5, 5.0, smin)
    for a, b in zip(hist["sigma"], hist["sigma"][1:]):
        assert b >= 0.5 * a
    # exact data with a shrinking residual: the limit is reached at least once
    assert any(b == 0.5 * a for a, b in zip(hist["sigma"], hist["sigma"][1:]))


# ---------------------------------------------------------------- observation pattern sampler

def test_vector_counter_generator_matches_published_outputs():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64_kat.txt")) if l[0] != "#"]
    for seed, n, val in rows:
        assert int(orng.counter_u64_np(int(seed), np.array([int(n) - 1]))[0]) == int(val, 16)


def test_probability_thresholds_are_exact():
    assert orng.threshold(0.5) == 1 << 63
    assert orng.threshold(0.25) == 1 << 62
    assert orng.threshold(0.1) == int(math.ldexp(0.1, 64)) == 1844674407370955264
    assert orng.threshold(1.0) is None and orng.threshold(0.0) == 0 and orng.threshold(-1.0) == 0


def test_bernoulli_mask_density_and_outliers():
    dims = (101, 99, 100)                                # 999,900 entries
    m, s, u = orng.sample_mask(7, dims, 0.3, 0, 0.2)
    n = m.size
    assert abs(m.mean() - 0.3) < 5 * math.sqrt(0.3 * 0.7 / n)
    assert np.all(s <= m)                                # outliers only where observed
    k = int(m.sum())
    assert abs(s.sum() / k - 0.2) < 5 * math.sqrt(0.2 * 0.8 / k)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.002
    assert np.all(np.floor(u * 2.0 ** 53) == u * 2.0 ** 53)   # 53-bit grid
    # seeds and keys are independent streams
    m2, _, _ = orng.sample_mask(8, dims, 0.3)
    assert np.mean(m == m2) < 0.6
    assert orng.sample_mask(7, dims, 1.0)[0].all() and not orng.sample_mask(7, dims, 0.0)[0].any()


def test_block_mask_is_tiled_and_shared_by_the_channel_mode():
    dims, B = (40, 36, 3, 7), 16                         # ragged tiles along both modes
    m, _, _ = orng.sample_mask(3, dims, 0.2, B)
    M = m.reshape(dims, order="F")
    assert np.all(M == M[:, :, :1, :])                   # shared by mode 2
    nbh, nbw = 3, 3
    tiles = []
    for f in range(dims[3]):
        for bh in range(nbh):
            for bw in range(nbw):
                t = M[bh * B:(bh + 1) * B, bw * B:(bw + 1) * B, 0, f]
                assert t.min() == t.max()                # a tile is all observed or all missing
                tiles.append(int(t[0, 0]))
    assert len(tiles) == 63
    big, _, _ = orng.sample_mask(3, (16 * 50, 16 * 40, 3, 20), 0.2, B)
    Mb = big.reshape((16 * 50, 16 * 40, 3, 20), order="F")[::B, ::B, 0, :]
    assert abs(Mb.mean() - 0.2) < 5 * math.sqrt(0.2 * 0.8 / Mb.size)


# ---------------------------------------------------------------- uniform row sampling (Sec. 6.1)

@pytest.mark.parametrize("k", [0, 1, 2])
def test_row_sampling_every_row_once_is_the_full_step(k):
    # every row of Z^{!=k}_{[2]} once, in any order: the sampled update is the full update
    dims, ranks = (4, 3, 5), (2, 3, 2)
    Z, P, X = _masked_problem(dims, ranks, 61)
    M = int(np.prod(dims)) // dims[k]
    full, fi = aw.core_update(X, P, Z, k, 0.8)
    for rows in (np.arange(M), np.random.default_rng(k).permutation(M)):
        new, info = aw.core_update(X, P, Z, k, 0.8, rows=rows)
        np.testing.assert_allclose(new, full, rtol=1e-12, atol=1e-12)
        assert info.n_obs == fi.n_obs and info.eta == pytest.approx(fi.eta, rel=1e-12)


def test_row_sampling_repeated_rows_leave_the_step_unchanged():
    # every row twice: d and h double, eta halves, the step eta h is the full one
    dims, ranks = (4, 3, 5), (2, 3, 2)
    Z, P, X = _masked_problem(dims, ranks, 62)
    M = int(np.prod(dims)) // dims[1]
    full, fi = aw.core_update(X, P, Z, 1, 1.1)
    new, info = aw.core_update(X, P, Z, 1, 1.1, rows=np.repeat(np.arange(M), 2))
    np.testing.assert_allclose(info.d, 2 * fi.d, rtol=1e-12, atol=1e-12)
    assert info.eta == pytest.approx(fi.eta / 2, rel=1e-12)
    np.testing.assert_allclose(new, full, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [0, 2, 3])
def test_row_sampled_gradient_by_brute_force(k):
    # eq. (9) on the sampled rows, summed entry by entry with A(m) multiplied out from the
    # slices and x-hat from Def. 1, repeated rows counted each time they are drawn
    dims, ranks = (3, 2, 4, 3), (2, 3, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 63)
    N, sigma = len(dims), 0.7
    idx = orng.uniform_row_indices(5, 1, k, dims, 40)
    rows = orng.uniform_rows(5, 1, k, dims, 40)
    _, info = aw.core_update(X, P, Z, k, sigma, rows=rows)
    rk, rk1 = ranks[k], ranks[(k + 1) % N]
    d = np.zeros((dims[k], rk * rk1))
    for n in range(40):
        Am = np.eye(rk1)
        for s in range(1, N):
            j = (k + s) % N
            Am = Am @ Z[j][:, idx[n, j], :]
        for i in range(dims[k]):
            full = [int(v) for v in idx[n]]
            full[k] = i
            if not P[tuple(full)]:
                continue
            e = X[tuple(full)] - tr.reconstruct_entry(Z, full)
            y = np.exp(-e * e / (2 * sigma * sigma)) * e
            for a in range(rk):
                for b in range(rk1):
                    d[i, a + b * rk] += y * Am[b, a]
    np.testing.assert_allclose(info.d, d, rtol=1e-12, atol=1e-12)


def test_uniform_rows_decode_and_range():
    dims = (5, 3, 7, 2)
    for k in range(4):
        idx = orng.uniform_row_indices(11, 2, k, dims, 300)
        rows = orng.uniform_rows(11, 2, k, dims, 300)
        M = int(np.prod(dims)) // dims[k]
        assert rows.min() >= 0 and rows.max() < M
        for j in range(4):
            assert (idx[:, j] >= 0).all() and (idx[:, j] < dims[j]).all()
        assert (idx[:, k] == 0).all()
        # the row index is little-endian over modes k+1, ..., k-1
        rest = rows.copy()
        for s in range(1, 4):
            j = (k + s) % 4
            np.testing.assert_array_equal(rest % dims[j], idx[:, j])
            rest //= dims[j]
    # streams differ by sweep and by update
    assert not np.array_equal(orng.uniform_rows(11, 0, 1, dims, 50), orng.uniform_rows(11, 1, 1, dims, 50))


def test_uniform_rows_are_uniform():
    dims = (2, 3, 5, 2)      # k = 0: M = 30 rows
    rows = orng.uniform_rows(3, 0, 0, dims, 15000)
    cnt = np.bincount(rows, minlength=30)
    chi2 = np.sum((cnt - 500.0) ** 2 / 500.0)
    assert chi2 < 58.3       # 29 dof; p ~ 1e-3 threshold


def test_row_sampled_fit_and_quantile_use_the_update_rows():
    dims, ranks = (5, 4, 6), (2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 64)
    opts = aw.FitOptions(max_sweeps=2, tol=0, sketch_sizes=(3, 2, 4), sampling="rows", seed=9)
    rows = aw.rows_for(opts, 1, 2, dims)
    assert rows.size == 3 * 2                                 # the RStS sketch's row count
    np.testing.assert_array_equal(rows, orng.uniform_rows(9, 1, 2, dims, 6))
    e = aw.residual_abs(X, P, Z, rows=aw.rows_for(opts, 0, 0, dims), k=0)
    sig = aw.sweep_sigma(X, P, Z, opts, 0, 1e-12)
    assert sig == aw.quantile_sigma(e, 0.5, 5.0, 1e-12)
    # the sampled residuals are those of the explicit reconstruction at those fibres
    r0 = aw.rows_for(opts, 0, 0, dims)
    Xk, Pk = tr.unfold_cyclic(X, 0)[:, r0], tr.unfold_cyclic(P, 0)[:, r0].astype(bool)
    Xh = tr.unfold_cyclic(tr.reconstruct(Z), 0)[:, r0]
    np.testing.assert_allclose(np.sort(e), np.sort(np.abs(Xk - Xh)[Pk]), rtol=1e-12, atol=1e-14)
    cores, hist = aw.fit(X, P, Z, opts)
    assert len(hist["sigma"]) == 2 and all(np.isfinite(cores[0]).ravel())


# ---------------------------------------------------------------- leverage-score sampling (Sec. 6.1)

def _orthonormal_core(r, I, r2, seed):
    # a core whose mode-2 unfolding (I x r r2) has orthonormal columns
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((I, r * r2)))
    return tr.fold_core(Q, r, r2)


def test_core_leverage_closed_forms():
    # orthonormal columns: the leverage of row i is its squared norm, and they sum to r r'
    Z = _orthonormal_core(2, 11, 3, 1)
    lev = aw.core_leverage(Z, 1e-12)
    np.testing.assert_allclose(lev, np.sum(tr.unfold_core(Z) ** 2, axis=1), rtol=1e-9, atol=1e-12)
    assert lev.sum() == pytest.approx(6.0, rel=1e-9)
    # fewer slices than r r' (full row rank): every row has leverage 1 (up to the ridge)
    Z = np.random.default_rng(2).standard_normal((3, 4, 2))
    np.testing.assert_allclose(aw.core_leverage(Z, 1e-12), np.ones(4), rtol=1e-6)
    # invariant to a rescaling of the core and to an invertible change of basis of Z_(2)
    Z = np.random.default_rng(3).standard_normal((2, 9, 2))
    B = np.random.default_rng(4).standard_normal((4, 4)) + 3 * np.eye(4)
    Zb = tr.fold_core(tr.unfold_core(Z) @ B, 2, 2)
    np.testing.assert_allclose(aw.core_leverage(7.0 * Z, 1e-12), aw.core_leverage(Z, 1e-12), rtol=1e-8)
    np.testing.assert_allclose(aw.core_leverage(Zb, 1e-12), aw.core_leverage(Z, 1e-12), rtol=1e-7)


def test_leverage_draws_follow_the_leverage_distribution():
    dims, ranks = (3, 12, 4), (2, 2, 3)
    Z = rand_cores(dims, ranks, 70)
    rows, w, idx = aw.leverage_rows(Z, 0, 12000, 5, 0)
    lev = aw.core_leverage(Z[1])
    q = lev / lev.sum()
    cnt = np.bincount(idx[:, 1], minlength=12)
    chi2 = np.sum((cnt - 12000 * q) ** 2 / (12000 * q))
    assert chi2 < 32.9       # 11 dof; p ~ 1e-3 threshold
    # the weight is 1 / (J p) with p the product of the per-mode probabilities
    q2 = aw.core_leverage(Z[2]) / aw.core_leverage(Z[2]).sum()
    np.testing.assert_allclose(w, 1.0 / (12000 * q[idx[:, 1]] * q2[idx[:, 2]]), rtol=1e-12)
    np.testing.assert_array_equal(rows, idx[:, 1] + 12 * idx[:, 2])


def test_leverage_weighted_gradient_is_unbiased():
    # E[sum_n omega_n (W P E)_n A_n] over the draws is the full gradient of eq. (9)
    dims, ranks = (3, 4, 5), (2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 71, rho=1.0)
    _, full = aw.core_update(X, P, Z, 0, 0.9)
    acc = np.zeros_like(full.d)
    trials = 300
    for t in range(trials):
        rows, w, _ = aw.leverage_rows(Z, 0, 20, 9, t)
        _, info = aw.core_update(X, P, Z, 0, 0.9, rows=rows, row_weights=w)
        acc += info.d
    assert rel_err(acc / trials, full.d) < 0.08


def test_uniform_leverage_gives_constant_weights_and_the_unweighted_step():
    # cores whose unfoldings are square orthogonal: every leverage is 1, p is uniform, the
    # weights are all M / J, and a common weight leaves the step unchanged
    dims, ranks = (4, 6, 6), (2, 2, 3)
    Z = [_orthonormal_core(2, 4, 2, 11), _orthonormal_core(2, 6, 3, 12), _orthonormal_core(3, 6, 2, 13)]
    g = np.random.default_rng(14)
    P = (g.random(dims) < 0.7).astype(np.uint8)
    X = tr.reconstruct(rand_cores(dims, ranks, 15)) + 0.1 * g.standard_normal(dims)
    rows, w, _ = aw.leverage_rows(Z, 0, 30, 3, 1, lambda_rel=1e-13)
    np.testing.assert_allclose(w, np.full(30, 36 / 30), rtol=1e-9)
    a, ia = aw.core_update(X, P, Z, 0, 1.2, rows=rows, row_weights=w)
    b, ib = aw.core_update(X, P, Z, 0, 1.2, rows=rows)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ia.d, ib.d * 36 / 30, rtol=1e-9, atol=1e-12)


def test_leverage_weighted_gradient_by_brute_force():
    dims, ranks = (3, 2, 4, 3), (2, 3, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 72)
    N, k, sigma = 4, 1, 0.7
    rows, w, idx = aw.leverage_rows(Z, k, 25, 4, 2)
    _, info = aw.core_update(X, P, Z, k, sigma, rows=rows, row_weights=w)
    rk, rk1 = ranks[k], ranks[(k + 1) % N]
    d = np.zeros((dims[k], rk * rk1))
    for n in range(25):
        Am = np.eye(rk1)
        for s in range(1, N):
            j = (k + s) % N
            Am = Am @ Z[j][:, idx[n, j], :]
        for i in range(dims[k]):
            full = [int(v) for v in idx[n]]
            full[k] = i
            if not P[tuple(full)]:
                continue
            e = X[tuple(full)] - tr.reconstruct_entry(Z, full)
            y = w[n] * np.exp(-e * e / (2 * sigma * sigma)) * e
            for a in range(rk):
                for b in range(rk1):
                    d[i, a + b * rk] += y * Am[b, a]
    np.testing.assert_allclose(info.d, d, rtol=1e-12, atol=1e-12)


def test_leverage_fit_draws_from_the_current_cores():
    dims, ranks = (5, 4, 6), (2, 2, 2)
    Z, P, X = _masked_problem(dims, ranks, 73)
    opts = aw.FitOptions(max_sweeps=2, tol=0, sketch_sizes=(3, 2, 4), sampling="leverage", seed=9,
                         sigma_mode="fixed", sigma=1.0)
    cores, hist = aw.fit(X, P, Z, opts)
    # sweep 0, update 1 draws from the cores after update 0
    c1 = list(Z)
    c1[0], _ = aw.core_update(X, P, Z, 0, 1.0, rows=aw.rows_for(opts, 0, 0, dims, Z)[0],
                              row_weights=aw.rows_for(opts, 0, 0, dims, Z)[1])
    r_fit = aw.rows_for(opts, 0, 1, dims, c1)
    r_old = aw.rows_for(opts, 0, 1, dims, Z)
    assert r_fit[0].size == 3 * 4
    assert not np.allclose(r_fit[1], r_old[1])        # weights follow the updated core 0
    assert len(hist["sigma"]) == 2 and np.isfinite(cores[1]).all()


def test_leverage_of_a_zero_core_falls_back_to_uniform_draws():
    dims, ranks = (4, 6, 5), (2, 2, 2)
    Z = rand_cores(dims, ranks, 74)
    Z[1] = np.zeros_like(Z[1])
    rows, w, idx = aw.leverage_rows(Z, 0, 3000, 2, 0)
    u = orng.uniform01(orng.lev_key(2, 0, 0, 1), np.arange(3000))
    np.testing.assert_array_equal(idx[:, 1], np.floor(u * 6).astype(np.int64))
    q2 = aw.core_leverage(Z[2]) / aw.core_leverage(Z[2]).sum()
    np.testing.assert_allclose(w, 1.0 / (3000 * (1.0 / 6) * q2[idx[:, 2]]), rtol=1e-12)
    assert np.isfinite(w).all()
