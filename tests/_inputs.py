"""The full-size workloads' inputs recomputed on the host, entry by entry, from the seed
alone: the same recipe as bench.build_inputs, with the oracle's own reconstruction (Def. 1
as chain products of the seeded cores, FP64) and the oracle's counter generator for the
mask, the outlier selection, the outlier values and the noise.  Nothing here reads a value
the library computed, so the full-size parity tests feed the oracle inputs that are
independent of the HIP path."""
from __future__ import annotations

import math

import numpy as np

import synth
from oracle import awrtrd as aw
from oracle import rng as orng
from oracle import tr


def _noise_seed(seed: int, stream: int) -> int:
    # the derivation of bench.noise_seed, restated
    return (int(seed) ^ (0x4E4F495345000000 + stream)) & ((1 << 64) - 1)


class OracleInputs:
    def __init__(self, wname: str, seed: int = 0, dims=None):
        w = synth.WORKLOADS[wname]
        self.w, self.seed = w, int(seed)
        self.dims = tuple(dims or w.dims)
        self.n = int(np.prod(self.dims))
        self.strides = np.cumprod((1,) + self.dims[:-1]).astype(np.int64)
        std = w.core_std if w.core_std is not None else 1.0 / math.sqrt(w.ranks[0])
        cores = (synth.lowpass_cores(self.dims, w.ranks, seed, std) if w.lowpass
                 else synth.gaussian_cores(self.dims, w.ranks, seed, std))
        npdt = np.float64 if w.dtype == "f64" else np.float32
        # the cores as the device holds them (rounded to the problem dtype), in FP64
        self.cores = [z.astype(npdt).astype(np.float64) for z in cores]
        self.scale = 1.0
        if w.normalise_max:
            self.scale = 1.0 / self.max_abs_clean()
        self.block = 16 if w.mask_kind == "block16" else 0
        self._sd = None
        self._mx = None

    # ---- the clean tensor
    def clean_at(self, idx: np.ndarray, chunk: int = 1 << 18) -> np.ndarray:
        """X*(i) = Tr(Z_1(i_1) ... Z_N(i_N)) (Def. 1) at multi-indices idx (n, N)."""
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty(len(idx))
        for s in range(0, len(idx), chunk):
            sl = idx[s:s + chunk]
            A = self.cores[0][:, sl[:, 0], :].transpose(1, 0, 2)
            for j in range(1, len(self.dims)):
                A = np.matmul(A, self.cores[j][:, sl[:, j], :].transpose(1, 0, 2))
            out[s:s + chunk] = np.trace(A, axis1=1, axis2=2)
        return out * self.scale

    def max_abs_clean(self) -> float:
        """max |X*| over the whole tensor: the first N - 1 cores merged once (Def. 2), then
        one slice of the last mode at a time."""
        S = self.cores[0]
        for Z in self.cores[1:-1]:
            S = tr.merge(S, Z)                              # (r_0, prod I_0..I_{N-2}, r_{N-1})
        last = self.cores[-1]
        mx = 0.0
        for i in range(last.shape[1]):
            x = np.einsum("amb,ba->m", S, last[:, i, :])
            mx = max(mx, float(np.max(np.abs(x))))
        return mx

    def std_clean(self) -> float:
        """Population standard deviation of X* from two traces: sum X* = Tr(prod_j S_j) with
        S_j = sum_i Z_j(i), and ||X*||^2 = Tr(prod_j K_j) with K_j = sum_i Z_j(i) (x) Z_j(i)."""
        if self._sd is None:
            Ssum = np.eye(self.cores[0].shape[0])
            K = None
            for Z in self.cores:
                Ssum = Ssum @ Z.sum(axis=1)
                Kj = aw.fgmc_factor(Z)
                K = Kj if K is None else K @ Kj
            mean = float(np.trace(Ssum)) * self.scale / self.n
            sq = float(np.trace(K)) * self.scale ** 2 / self.n
            self._sd = math.sqrt(max(sq - mean * mean, 0.0))
        return self._sd

    # ---- observed values
    def lin_of(self, idx: np.ndarray) -> np.ndarray:
        return np.asarray(idx, dtype=np.int64) @ self.strides

    def entries(self, idx: np.ndarray):
        """(observed bits, values of X) at multi-indices idx (n, N)."""
        w = self.w
        lin = self.lin_of(idx)
        obs, sel, u = orng.sample_mask_at(self.seed, self.dims, w.rho, self.block, w.outlier_frac, lin)
        x = self.clean_at(idx)
        if w.noise_var > 0:
            u1 = orng.sample_mask_at(_noise_seed(self.seed, 1), self.dims, 1.0, 0, 0.0, lin)[2]
            u2 = orng.sample_mask_at(_noise_seed(self.seed, 2), self.dims, 1.0, 0, 0.0, lin)[2]
            x = x + np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2) * math.sqrt(w.noise_var)
        pick = sel.astype(bool)
        if pick.any():
            if w.outlier_law == "uniform_std":
                val = (2.0 * u[pick] - 1.0) * (w.outlier_scale * self.std_clean())
            elif w.outlier_law == "saltpepper":
                if self._mx is None:
                    self._mx = self.max_abs_clean() * self.scale
                val = np.where(u[pick] < 0.5, -self._mx, self._mx)
            elif w.outlier_law == "uniform01":
                val = u[pick]
            else:
                raise ValueError(w.outlier_law)
            x = x.copy()
            x[pick] = val
        return obs, x

    def mask_of_slice(self, k: int, i: int) -> np.ndarray:
        """Observed multi-indices (n, N) of the slice i_k = i, in column-major order."""
        dims = self.dims
        rest = [d for j, d in enumerate(dims) if j != k]
        m = int(np.prod(rest))
        sub = np.unravel_index(np.arange(m, dtype=np.int64), rest, order="F")
        idx = np.empty((m, len(dims)), dtype=np.int64)
        c = 0
        for j in range(len(dims)):
            if j == k:
                idx[:, j] = i
            else:
                idx[:, j] = sub[c]
                c += 1
        obs, _, _ = orng.sample_mask_at(self.seed, dims, self.w.rho, self.block, self.w.outlier_frac,
                                        self.lin_of(idx))
        return idx[obs.astype(bool)]
