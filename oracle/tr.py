"""Tensor-ring data model in plain FP64 numpy (oracle; test infrastructure only).

Follows the preliminaries of the paper:
  * Def. 1 (TR decomposition): X[i_1..i_N] = Tr(Z_1(i_1) ... Z_N(i_N)), Z_k(i) the
    i-th lateral slice (r_k x r_{k+1}) of core k, r_{N+1} = r_1.
  * Def. 2 (core merging): the merged core's slice at the little-endian index
    i_k + I_k * i_{k+1} is Z_k(i_k) Z_{k+1}(i_{k+1}).
  * Theorem 1: X_[k] = Z_{k(2)} (Z^{!=k}_{[2]})^T with the subchain taken in the cyclic
    order k+1, ..., N, 1, ..., k-1 and the cyclic mode-k unfolding X_[k].

Indices are 0-based here.  Cores are arrays of shape (r_k, I_k, r_{k+1}).
"""
from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np


def slice_of(Z: np.ndarray, i: int) -> np.ndarray:
    """Lateral slice Z_k(i) (Def. 1)."""
    return Z[:, i, :]


def reconstruct_entry(cores: Sequence[np.ndarray], idx: Sequence[int]) -> float:
    """One entry by Def. 1: the trace of the product of the selected slices."""
    M = np.eye(cores[0].shape[0])
    for Z, i in zip(cores, idx):
        M = M @ Z[:, i, :]
    return float(np.trace(M))


def reconstruct_bruteforce(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Whole tensor by looping Def. 1 over every index (small tensors only)."""
    dims = [Z.shape[1] for Z in cores]
    X = np.empty(dims)
    for idx in itertools.product(*[range(I) for I in dims]):
        X[idx] = reconstruct_entry(cores, idx)
    return X


def merge(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Def. 2: merge two adjacent (possibly already merged) cores.

    L: (r0, m1, r1), R: (r1, m2, r2) -> (r0, m1*m2, r2) whose slice at i + m1*j is
    L(i) @ R(j)."""
    r0, m1, r1 = L.shape
    r1b, m2, r2 = R.shape
    assert r1 == r1b, "adjacent ranks must agree"
    out = np.einsum("aib,bjc->ajic", L, R)          # [a, j, i, c]
    return out.reshape(r0, m2 * m1, r2)             # middle index j*m1 + i


def reconstruct(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Whole tensor by sequential merging (Def. 2) and a final trace (Def. 1)."""
    S = cores[0]
    for Z in cores[1:]:
        S = merge(S, Z)
    x = np.einsum("aia->i", S)
    dims = [Z.shape[1] for Z in cores]
    return x.reshape(dims, order="F")


def cyclic_order(N: int, k: int) -> List[int]:
    """Modes k+1, ..., N, 1, ..., k-1 (0-based, mod N): the subchain order of Thm. 1."""
    return [(k + s) % N for s in range(1, N)]


def subchain(cores: Sequence[np.ndarray], k: int) -> np.ndarray:
    """Z^{!=k}: all cores but k merged in cyclic order; shape (r_{k+1}, M_k, r_k)."""
    order = cyclic_order(len(cores), k)
    S = cores[order[0]]
    for j in order[1:]:
        S = merge(S, cores[j])
    return S


def subchain_unfolding(cores: Sequence[np.ndarray], k: int) -> np.ndarray:
    """A = Z^{!=k}_{[2]} (M_k x r_k r_{k+1}).

    Row m is the little-endian index over (i_{k+1}, ..., i_{k-1}); column a + b*r_k holds
    A(m)[b, a] where A(m) = Z_{k+1}(i_{k+1}) ... Z_{k-1}(i_{k-1}) is r_{k+1} x r_k."""
    S = subchain(cores, k)                           # [b, m, a]
    rk1, M, rk = S.shape
    return S.transpose(1, 0, 2).reshape(M, rk1 * rk)


def unfold_cyclic(X: np.ndarray, k: int) -> np.ndarray:
    """X_[k] (I_k x M_k): column = little-endian index over (i_{k+1}, ..., i_{k-1})."""
    N = X.ndim
    perm = [(k + s) % N for s in range(N)]
    return np.transpose(X, perm).reshape(X.shape[k], -1, order="F")


def fold_cyclic(Xk: np.ndarray, k: int, dims: Sequence[int]) -> np.ndarray:
    """Inverse of unfold_cyclic."""
    N = len(dims)
    perm = [(k + s) % N for s in range(N)]
    Xt = Xk.reshape([dims[p] for p in perm], order="F")
    inv = np.argsort(perm)
    return np.transpose(Xt, inv)


def unfold_core(Z: np.ndarray) -> np.ndarray:
    """Z_{k(2)} (I_k x r_k r_{k+1}), column a + b*r_k holds Z_k(i)[a, b]."""
    r, I, r2 = Z.shape
    return Z.transpose(1, 2, 0).reshape(I, r2 * r)


def fold_core(Zk2: np.ndarray, r: int, r2: int) -> np.ndarray:
    """Inverse of unfold_core: (I, r*r2) -> (r, I, r2)."""
    I = Zk2.shape[0]
    return Zk2.reshape(I, r2, r).transpose(2, 0, 1).copy()


def reconstruct_at(cores: Sequence[np.ndarray], lin: np.ndarray) -> np.ndarray:
    """Entries at column-major linear indices, each by Def. 1 (slow, exact)."""
    dims = [Z.shape[1] for Z in cores]
    idx = np.unravel_index(np.asarray(lin, dtype=np.int64), dims, order="F")
    out = np.empty(len(lin))
    for t in range(len(lin)):
        out[t] = reconstruct_entry(cores, [int(a[t]) for a in idx])
    return out
