"""AWRTRD / SAWRTRD per-core update sweep in plain FP64 numpy (oracle).

TEST INFRASTRUCTURE ONLY: the HIP library never imports or calls this module, and
only the tests, the smoke check and the bench's CPU-baseline leg use it.

Everything is explicit: the subchain unfolding A = Z^{!=k}_{[2]} and the cyclic
unfolding X_[k] are formed in full (Thm. 1), the Gram matrix is formed both as
A^T A and by FGMC (Prop. 2, eq. 13), and the weight, gradient, scaled direction,
step length and update follow eqs. (7) and (9)-(12) (sketched form: (14)-(18)) in
the order of Alg. 1.

Readings of passages the paper leaves open or prints garbled (each is also listed
with its justification in the design notes):
  * weight (eq. 7): w = exp(-e^2 / (2 sigma^2)) in (0, 1], w(0) = 1; the printed
    g'(x)/x has the opposite sign for the stated g.  sigma = +inf gives w = 1.
  * update (eqs. 11, 17): Z_k <- Z_k + eta * fold(h).  d of eq. (9) is the negative
    gradient of the weighted LS objective and eta of eq. (12) is the exact minimiser
    along +h, so the printed minus sign would climb.
  * FGMC (eq. 13): Phi is not defined; the Kronecker form K_j = sum_i Z_j(i) (x) Z_j(i)
    with the explicit realignment below is used and pinned against A^T A.
  * lambda (eq. 10): lambda = lambda_rel * tr(G) / R^2 (scale free).
  * W is recomputed from the current cores at every core update.
  * eta = 0 (core unchanged) when the line-search denominator is 0.
  * convergence (Alg. 1): no stop test after the first sweep.
  * uniform row sampling (ablation of Sec. 6.1): J rows of Z^{!=k}_{[2]} drawn
    independently and uniformly with replacement, J = the row count of the RStS sketch
    of the same sizes; no rescaling of the sampled rows (a common factor on them leaves
    the step eta h unchanged); the Gram matrix stays the global one.
  * leverage-score sampling (ablation of Sec. 6.1, TRALS-S's sampler): the same J, each
    mode's index drawn from that core's leverage distribution (leverage of the rows of
    its mode-2 unfolding, with the ridge of eq. 10), the row weighted by 1 / (J p) in the
    gradient, the line search and the loss; the quantile residuals stay unweighted.
  * sigma schedule: 'fixed', 'given' (one value per sweep) or 'quantile'.  The paper
    defers to an external adaptive rule that is not reproduced in its text; the
    quantile rule is this project's own choice: PARITY UNPINNED beyond the
    sigma -> inf limit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import rng as _rng
from .tr import (cyclic_order, fold_core, reconstruct, subchain_unfolding, unfold_core,
                 unfold_cyclic)


# ----------------------------------------------------------------------------------
# entry-wise pieces
# ----------------------------------------------------------------------------------

def weights(E: np.ndarray, sigma: float) -> np.ndarray:
    """Correntropy weights of eq. (7): exp(-E^2 / (2 sigma^2))."""
    if math.isinf(sigma):
        return np.ones_like(E)
    return np.exp(-(E * E) / (2.0 * sigma * sigma))


def welsch(E: np.ndarray, sigma: float) -> np.ndarray:
    """Per-entry loss sigma^2 (1 - exp(-e^2 / 2 sigma^2)), i.e. g_sigma(0) - g_sigma(e) for
    the Gaussian-kernel correntropy g of eq. (4); its sigma -> inf limit is e^2 / 2."""
    if math.isinf(sigma):
        return 0.5 * E * E
    return -(sigma * sigma) * np.expm1(-(E * E) / (2.0 * sigma * sigma))


# ----------------------------------------------------------------------------------
# FGMC
# ----------------------------------------------------------------------------------

def fgmc_factor(Z: np.ndarray) -> np.ndarray:
    """K = sum_i Z(i) (x) Z(i)  (r_k^2 x r_{k+1}^2, numpy kron index order)."""
    r0, I, r1 = Z.shape
    K = np.zeros((r0 * r0, r1 * r1))
    for i in range(I):
        K += np.kron(Z[:, i, :], Z[:, i, :])
    return K


def realign(P: np.ndarray, rk: int, rk1: int) -> np.ndarray:
    """G[(a + b r_k), (a' + b' r_k)] = P[(b r_{k+1} + b'), (a r_k + a')]."""
    return P.reshape(rk1, rk1, rk, rk).transpose(0, 2, 1, 3).reshape(rk1 * rk, rk1 * rk)


def gram_fgmc(cores: Sequence[np.ndarray], k: int) -> np.ndarray:
    """G^{!=k} by the ring product of the other cores' factors (eq. 13)."""
    order = cyclic_order(len(cores), k)
    P = fgmc_factor(cores[order[0]])
    for j in order[1:]:
        P = P @ fgmc_factor(cores[j])
    return realign(P, cores[k].shape[0], cores[order[0]].shape[0])


def gram_explicit(cores: Sequence[np.ndarray], k: int) -> np.ndarray:
    """G^{!=k} = A^T A with A formed explicitly (the cost FGMC avoids)."""
    A = subchain_unfolding(cores, k)
    return A.T @ A


# ----------------------------------------------------------------------------------
# one core update
# ----------------------------------------------------------------------------------

@dataclasses.dataclass
class StepInfo:
    d: np.ndarray            # gradient, eq. (9)/(15)   (I_k x R^2)
    h: np.ndarray            # scaled direction, eq. (10)/(16)
    G: np.ndarray            # Gram of the full subchain (eq. 13)
    eta: float               # step length, eq. (12)/(18)
    num: float               # <d, h>
    den: float               # || sqrt(W) o P o (h A^T) ||^2
    loss: float              # sum over the update's observed entries of sigma^2 (1 - w)
    wls: float               # sum of w e^2 over the same entries
    n_obs: int               # observed entries the update touched
    W: np.ndarray            # weights on the update's unfolded entries (x P)
    E: np.ndarray            # residual on the update's unfolded entries (x P)


def _sub(cores, idx):
    return [Z[:, ix, :] for Z, ix in zip(cores, idx)]


def _sampled_rows(X, P, cores, k, rows):
    """X_[k], P_[k] and A = Z^{!=k}_{[2]} restricted to the sampled rows of A (and the
    same columns of the unfoldings), duplicates kept."""
    rows = np.asarray(rows, dtype=np.int64)
    A = subchain_unfolding(cores, k)[rows]
    return unfold_cyclic(X, k)[:, rows], unfold_cyclic(P, k)[:, rows], A


def core_leverage(Z: np.ndarray, lambda_rel: float = 1e-9) -> np.ndarray:
    """Leverage scores of the rows of the classical mode-2 unfolding Z_(2) (I x r r'): row i
    scores z_i^T (C + lambda I)^{-1} z_i with C = Z_(2)^T Z_(2) and lambda = lambda_rel tr(C) / R
    (the ridge of eq. 10, which keeps a core with fewer slices than r r' well defined)."""
    Z2 = unfold_core(Z)
    C = Z2.T @ Z2
    R = C.shape[0]
    if not np.trace(C) > 0.0:                            # a zero core: no leverage
        return np.zeros(Z2.shape[0])
    lam = lambda_rel * np.trace(C) / R
    Y = np.linalg.solve(C + lam * np.eye(R), Z2.T)      # (C + lam I)^{-1} z_i, column i
    return np.einsum("ip,pi->i", Z2, Y)


def leverage_rows(cores: Sequence[np.ndarray], k: int, J: int, seed: int, t: int,
                  lambda_rel: float = 1e-9):
    """TRALS-S's leverage-score row sampling of Z^{!=k}_{[2]} (the ablation of Sec. 6.1):
    every sample draws the index of each mode j != k independently, with probability
    q_j(i) = l_j(i) / sum_i l_j(i) from the leverage scores of core j, by inverse CDF of the
    running sums in slice order; its row has probability p = prod_j q_j(i_j) and importance
    weight 1 / (J p).  A core whose leverages are all zero (a zero core) is sampled
    uniformly instead.  Returns (rows (J,), weights (J,), per-mode indices (J, N))."""
    N = len(cores)
    dims = [Z.shape[1] for Z in cores]
    idx = np.zeros((J, N), dtype=np.int64)
    p = np.ones(J)
    for j in range(N):
        if j == k:
            continue
        lev = core_leverage(cores[j], lambda_rel)
        cdf = np.cumsum(lev)
        total = cdf[-1]
        u = _rng.uniform01(_rng.lev_key(seed, t, k, j), np.arange(J))
        if total > 0.0:
            ij = np.minimum(np.searchsorted(cdf, u * total, side="right"), dims[j] - 1)
            p *= lev[ij] / total
        else:  # a zero core has no leverage: draw its index uniformly
            ij = np.minimum(np.floor(u * dims[j]).astype(np.int64), dims[j] - 1)
            p *= 1.0 / dims[j]
        idx[:, j] = ij
    rows = np.zeros(J, dtype=np.int64)
    stride = 1
    for s_ in range(1, N):
        j = (k + s_) % N
        rows += idx[:, j] * stride
        stride *= dims[j]
    return rows, 1.0 / (J * p), idx


def core_update(X: np.ndarray, P: np.ndarray, cores: List[np.ndarray], k: int, sigma: float,
                lambda_rel: float = 1e-9, sketch: Optional[Sequence[Sequence[int]]] = None,
                gram: str = "fgmc", direction: str = "scaled", rows: Optional[np.ndarray] = None,
                row_weights: Optional[np.ndarray] = None):
    """One update of core k (Alg. 1 body).  Returns (new core k, StepInfo).

    sketch: None for the full path (AWRTRD), else index lists I_1..I_N (RStS,
    eqs. 14-18): the gradient and the line search use the subtensor, the Gram matrix
    always uses the full cores.
    rows: the row-sampling ablations of Sec. 6.1 instead of a sketch: indices of rows of
    A = Z^{!=k}_{[2]} (with repeats); the gradient and the line search use those rows of A
    and the same columns of X_[k], P_[k], the Gram matrix the full cores.
    row_weights: importance weight of each sampled row (leverage sampling): every entry of
    sampled row n counts with weight omega_n in the gradient, the line-search denominator
    and the reported loss.
    gram: 'fgmc' (eq. 13) or 'explicit' (A^T A), both of the full cores; or 'local',
    the ablation of Sec. 6.1 that scales with the Gram matrix of the sampled cores only,
    A_I^T A_I of the sketched subchain unfolding (the full one without a sketch).
    direction: 'scaled' (eq. 10 / 16) or 'gradient' (the ablation of Sec. 6.1 that steps
    along d of eq. 9 / 15 itself, with the same exact line search).
    """
    N = len(cores)
    rk, rk1 = cores[k].shape[0], cores[k].shape[2]
    if rows is not None:
        assert sketch is None and gram != "local", "row sampling replaces the sketch"
        Xr, Pr, A = _sampled_rows(X, P, cores, k, rows)
        Pk = Pr.astype(bool)
        Xk = np.where(Pk, Xr, 0.0)
    else:
        if sketch is None:
            Xs, Ps, cs = X, P, cores
        else:
            ix = np.ix_(*[np.asarray(s, dtype=np.int64) for s in sketch])
            Xs, Ps = X[ix], P[ix]
            cs = _sub(cores, sketch)
            assert len(sketch[k]) == cores[k].shape[1], "mode k must be taken whole"
        A = subchain_unfolding(cs, k)                   # (M x R^2)
        Pk = unfold_cyclic(Ps, k).astype(bool)
        Xk = np.where(Pk, unfold_cyclic(Xs, k), 0.0)    # unobserved values never used
    Zk2 = unfold_core(cores[k])
    E = np.where(Pk, Xk - Zk2 @ A.T, 0.0)               # residual on observed entries
    W = np.where(Pk, weights(E, sigma), 0.0)            # eq. (7)
    Om = np.ones(Pk.shape[1]) if row_weights is None else np.asarray(row_weights, dtype=np.float64)
    d = (W * E * Om) @ A                                 # eq. (9) / (15)
    if gram == "local":
        G = A.T @ A
    elif gram == "fgmc":
        G = gram_fgmc(cores, k)
    else:
        G = gram_explicit(cores, k)
    if direction == "scaled":
        R2 = G.shape[0]
        lam = lambda_rel * np.trace(G) / R2
        C = G + lam * np.eye(R2)
        h = cho_solve(cho_factor(C, lower=True), d.T).T  # eq. (10) / (16)
    else:
        h = d.copy()
    num = float(np.sum(d * h))
    Q = h @ A.T
    den = float(np.sum(W * Q * Q * Om))                   # eq. (12) / (18) denominator
    eta = num / den if den > 0.0 else 0.0
    new = fold_core(Zk2 + eta * h, rk, rk1)              # eq. (11) / (17), sign '+'
    loss = float(np.sum(np.where(Pk, welsch(E, sigma), 0.0) * Om))
    info = StepInfo(d=d, h=h, G=G, eta=eta, num=num, den=den, loss=loss,
                    wls=float(np.sum(W * E * E * Om)), n_obs=int(Pk.sum()), W=W, E=E)
    return new, info


def gradient_row(cores: List[np.ndarray], k: int, idx: np.ndarray, vals: np.ndarray,
                 sigma: float, chunk: int = 1 << 16) -> np.ndarray:
    """Row i of eq. (9) from the observed entries of slice i_k = i, for tensors too large
    for the explicit unfolding: d(i)[a + b r_k] = sum over the entries of
    w(e) e A(m)[b, a], with A(m) = Z_{k+1}(i_{k+1}) ... Z_{k-1}(i_{k-1}) (Thm. 1),
    e = x - Tr(Z_k(i) A(m)) and w of eq. (7).

    idx: (n, N) integer indices of the entries (all with idx[:, k] == i); vals: (n,) values.
    Returns the r_k * r_{k+1} row in the column order of unfold_core."""
    N = len(cores)
    idx = np.asarray(idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    i = int(idx[0, k]) if len(idx) else 0
    Zi = cores[k][:, i, :]                               # r_k x r_{k+1}
    rk, rk1 = Zi.shape
    D = np.zeros((rk1, rk))                              # accumulates sum y A(m)
    for s in range(0, len(vals), chunk):
        sl = slice(s, s + chunk)
        order = cyclic_order(N, k)
        A = cores[order[0]][:, idx[sl, order[0]], :].transpose(1, 0, 2)   # (n, r, r')
        for j in order[1:]:
            A = np.matmul(A, cores[j][:, idx[sl, j], :].transpose(1, 0, 2))
        xhat = np.einsum("ab,nba->n", Zi, A)             # Tr(Z_k(i) A(m))
        e = vals[sl] - xhat
        y = weights(e, sigma) * e
        D += np.einsum("n,nba->ba", y, A)
    return D.reshape(-1)                                 # index b * r_k + a


# ----------------------------------------------------------------------------------
# sweep, convergence, sigma, fit
# ----------------------------------------------------------------------------------

def convergence_matrix(cores: Sequence[np.ndarray]) -> np.ndarray:
    """D^t = Z_{N(2)} G^{!=N} Z_{N(2)}^T (Alg. 1), equal to Xhat_[N] Xhat_[N]^T."""
    N = len(cores)
    Z = unfold_core(cores[N - 1])
    return Z @ gram_fgmc(cores, N - 1) @ Z.T


def residual_abs(X, P, cores, sketch=None, rows=None, k=0) -> np.ndarray:
    """|x - xhat| on the observed entries (of the sketch, or of update k's sampled rows,
    if given), in a fixed order."""
    if rows is not None:
        Xr, Pr, A = _sampled_rows(X, P, cores, k, rows)
        m = Pr.astype(bool)
        return np.abs(Xr - unfold_core(cores[k]) @ A.T)[m]
    if sketch is None:
        Xs, Ps, cs = X, P, cores
    else:
        ix = np.ix_(*[np.asarray(s, dtype=np.int64) for s in sketch])
        Xs, Ps, cs = X[ix], P[ix], _sub(cores, sketch)
    Xh = reconstruct(cs)
    m = Ps.astype(bool)
    return np.abs(Xs[m] - Xh[m])


def quantile_sigma(abs_e: np.ndarray, q: float, c: float, sigma_min: float) -> float:
    """sigma = max(sigma_min, c * Q_q(|e|)), Q_q the element of rank floor((n-1) q) of the
    ascending sort (no interpolation).  Own rule (parity unpinned)."""
    n = abs_e.size
    if n == 0:
        return sigma_min if sigma_min > 0 else 1.0
    srt = np.sort(abs_e)
    return max(sigma_min, c * float(srt[int(math.floor((n - 1) * q))]))


@dataclasses.dataclass
class FitOptions:
    max_sweeps: int = 30
    tol: float = 1e-3
    lambda_rel: float = 1e-9
    sigma_mode: str = "quantile"    # 'fixed' | 'given' | 'quantile'
    sigma: float = math.inf         # 'fixed'
    sigma_given: Sequence[float] = ()
    q: float = 0.5
    c: float = 5.0
    shrink: float = 0.5             # sigma_t >= shrink * sigma_{t-1} (quantile mode)
    sigma_min_rel: float = 1e-6     # sigma_min = sigma_min_rel * max |x| over observed
    sketch_sizes: Optional[Sequence[int]] = None
    seed: int = 0
    gram: str = "fgmc"
    direction: str = "scaled"
    sampling: str = "rsts"          # with sketch_sizes: 'rsts', 'rows' or 'leverage' (Sec. 6.1)


def sketch_for(opts: FitOptions, t: int, k: int, dims):
    if opts.sketch_sizes is None or opts.sampling != "rsts":
        return None
    return _rng.sketch_indices(opts.seed, t, k, dims, opts.sketch_sizes)


def _rows_J(opts: FitOptions, k: int, dims) -> int:
    J = 1
    for j, (I, s) in enumerate(zip(dims, opts.sketch_sizes)):
        if j != k:
            J *= min(max(1, int(s)), int(I))
    return J


def rows_for(opts: FitOptions, t: int, k: int, dims, cores=None):
    """Row sample of update (t, k), as many rows as the RStS sketch of the same sizes holds
    (the product of the other modes' clamped sizes): uniform ('rows'), or by leverage
    ('leverage', from the cores as they stand), then with its importance weights."""
    if opts.sketch_sizes is None or opts.sampling not in ("rows", "leverage"):
        return None
    J = _rows_J(opts, k, dims)
    if opts.sampling == "rows":
        return _rng.uniform_rows(opts.seed, t, k, dims, J)
    rows, w, _ = leverage_rows(cores, k, J, opts.seed, t, opts.lambda_rel)
    return rows, w


def _rows_and_weights(opts, t, k, dims, cores):
    r = rows_for(opts, t, k, dims, cores)
    if isinstance(r, tuple):
        return r
    return r, None


def sweep_sigma(X, P, cores, opts: FitOptions, t: int, sigma_min: float,
                sigma_prev: float = math.inf) -> float:
    """Kernel width for sweep t.  'quantile' (own rule, parity unpinned): over the
    observed entries the sweep's first update touches (all of them on the full path,
    its sketch under RStS, its sampled rows under uniform row sampling), sigma_t = max(c * Q_q(|e|), sigma_min, shrink * sigma_{t-1})
    with the cores as they stand at the start of the sweep."""
    if opts.sigma_mode == "fixed":
        return float(opts.sigma)
    if opts.sigma_mode == "given":
        return float(opts.sigma_given[t])
    dims = [Z.shape[1] for Z in cores]
    e = residual_abs(X, P, cores, sketch_for(opts, t, 0, dims), _rows_and_weights(opts, t, 0, dims, cores)[0])
    s = quantile_sigma(e, opts.q, opts.c, sigma_min)
    if math.isfinite(sigma_prev):
        s = max(s, opts.shrink * sigma_prev)
    return s


def sweep(X, P, cores: List[np.ndarray], sigma: float, opts: FitOptions, t: int = 0):
    """One pass over k = 1..N, each update seeing the latest cores (Alg. 1)."""
    dims = [Z.shape[1] for Z in cores]
    infos = []
    cores = list(cores)
    for k in range(len(cores)):
        rows, rw = _rows_and_weights(opts, t, k, dims, cores)
        new, info = core_update(X, P, cores, k, sigma, opts.lambda_rel,
                                sketch_for(opts, t, k, dims), opts.gram, opts.direction,
                                rows, rw)
        cores[k] = new
        infos.append(info)
    return cores, infos


def fit(X, P, cores: List[np.ndarray], opts: FitOptions):
    """Alg. 1: sweeps until t = C or the change of D^t falls below tol."""
    cores = [np.array(Z, dtype=np.float64) for Z in cores]
    Pb = P.astype(bool)
    sigma_min = opts.sigma_min_rel * float(np.max(np.abs(X[Pb]))) if Pb.any() else 0.0
    hist: Dict[str, list] = {"sigma": [], "e": [], "eta": [], "loss": []}
    D_prev = None
    sigma = math.inf
    for t in range(opts.max_sweeps):
        sigma = sweep_sigma(X, P, cores, opts, t, sigma_min, sigma)
        cores, infos = sweep(X, P, cores, sigma, opts, t)
        D = convergence_matrix(cores)
        e = math.inf if D_prev is None else float(np.linalg.norm(D - D_prev) / np.linalg.norm(D))
        D_prev = D
        hist["sigma"].append(sigma)
        hist["e"].append(e)
        hist["eta"].append([i.eta for i in infos])
        hist["loss"].append([i.loss for i in infos])
        if e < opts.tol:
            break
    return cores, hist


# ----------------------------------------------------------------------------------
# differentiation form and metrics
# ----------------------------------------------------------------------------------

def loss(X, P, cores, sigma: float) -> float:
    """L = sum over observed entries of sigma^2 (1 - exp(-e^2 / 2 sigma^2))."""
    Xh = reconstruct(cores)
    m = P.astype(bool)
    return float(np.sum(welsch(X[m] - Xh[m], sigma)))


def loss_grads(X, P, cores, sigma: float) -> List[np.ndarray]:
    """dL/dZ_k = -fold(d_k) for every k, d_k of eq. (9) with W = w(E) at these cores."""
    grads = []
    for k in range(len(cores)):
        N = len(cores)
        A = subchain_unfolding(cores, k)
        Pk = unfold_cyclic(P, k).astype(bool)
        Xk = np.where(Pk, unfold_cyclic(X, k), 0.0)
        E = np.where(Pk, Xk - unfold_core(cores[k]) @ A.T, 0.0)
        d = (np.where(Pk, weights(E, sigma), 0.0) * E) @ A
        grads.append(fold_core(-d, cores[k].shape[0], cores[k].shape[2]))
    return grads


def relative_error(cores, xstar) -> float:
    """||Xhat - X*||_F / ||X*||_F over every entry."""
    Xh = reconstruct(cores)
    return float(np.linalg.norm(Xh - xstar) / np.linalg.norm(xstar))
