"""Seeded synthetic inputs shared by the tests, the bench and the CPU oracle runs.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no tensor-ring contraction, no weights, no steps).  Building
the clean tensor from its cores is left to a caller-supplied ``reconstruct``
function, so the tests can use the oracle and the bench can use the library.

Conventions (the same as the C-ABI):
  * a core j is a float64 array of shape (r_j, I_j, r_{j+1}) (r_{N+1} = r_1),
    the layout of the TR definition (Def. 1);
  * a tensor is an N-d numpy array with shape ``dims``; its flat form handed to the
    library is ``ravel(order="F")`` (first index fastest, the paper's index
    linearisation of Def. 2);
  * a mask is a uint8 array of the same shape, 1 = observed.

Recipes follow the five synthetic workloads that stand in for the paper's image and
video data (Sec. 6): ranks, sizes, missing ratios and outlier laws are the ones
listed for them; continuous values come from numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "rng", "gaussian_cores", "lowpass_cores", "bernoulli_mask",
    "block_mask", "select_observed", "assemble", "make_workload", "cores_to_flat",
    "flat_to_cores", "core_offsets",
]


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (seed, stream)."""
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


# ----------------------------------------------------------------------------------
# layout helpers (pure data movement)
# ----------------------------------------------------------------------------------

def core_offsets(dims: Sequence[int], ranks: Sequence[int]) -> List[int]:
    """Start offset of every core inside one flat buffer (ABI layout)."""
    N = len(dims)
    off, o = [], 0
    for j in range(N):
        off.append(o)
        o += ranks[j] * dims[j] * ranks[(j + 1) % N]
    off.append(o)
    return off


def cores_to_flat(cores: Sequence[np.ndarray], dtype=np.float64) -> List[np.ndarray]:
    """(r, I, r') arrays -> flat ABI arrays: element (a, i, b) at i*r*r' + b*r + a."""
    return [np.ascontiguousarray(np.asarray(Z).transpose(1, 2, 0)).ravel().astype(dtype)
            for Z in cores]


def flat_to_cores(flat: Sequence[np.ndarray], dims, ranks) -> List[np.ndarray]:
    N = len(dims)
    out = []
    for j in range(N):
        r, I, r2 = ranks[j], dims[j], ranks[(j + 1) % N]
        out.append(np.asarray(flat[j], dtype=np.float64).reshape(I, r2, r).transpose(2, 0, 1).copy())
    return out


# ----------------------------------------------------------------------------------
# random cores
# ----------------------------------------------------------------------------------

def gaussian_cores(dims, ranks, seed: int, std: float = 1.0, stream: int = 1) -> List[np.ndarray]:
    """iid N(0, std^2) cores of shape (r_j, I_j, r_{j+1})."""
    g = rng(seed, stream)
    N = len(dims)
    return [g.standard_normal((ranks[j], dims[j], ranks[(j + 1) % N])) * std for j in range(N)]


def lowpass_cores(dims, ranks, seed: int, std: float, smooth_modes=(0, 1), width: float = 4.0,
                  stream: int = 1) -> List[np.ndarray]:
    """Gaussian cores whose lateral slices vary smoothly along i for the listed modes
    (circular Gaussian smoothing along the mode index, std ``width`` samples)."""
    cores = gaussian_cores(dims, ranks, seed, std, stream)
    for j in smooth_modes:
        I = dims[j]
        t = np.arange(I)
        d = np.minimum(t, I - t).astype(np.float64)
        ker = np.exp(-0.5 * (d / width) ** 2)
        ker /= np.sqrt(np.sum(ker ** 2))
        # circular convolution along axis 1 via FFT
        F = np.fft.rfft(cores[j], axis=1) * np.fft.rfft(ker)[None, :, None]
        cores[j] = np.fft.irfft(F, n=I, axis=1)
    return cores


# ----------------------------------------------------------------------------------
# masks and outliers
# ----------------------------------------------------------------------------------

_CHUNK = 1 << 24


def bernoulli_mask(dims, rho: float, seed: int, stream: int = 2) -> np.ndarray:
    """uint8 mask, each entry observed independently with probability rho."""
    g = rng(seed, stream)
    n = int(np.prod(dims))
    flat = np.empty(n, dtype=np.uint8)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        flat[s:e] = g.random(e - s) < rho
    return flat.reshape(dims, order="F")


def block_mask(dims, block: int, p_missing: float, seed: int, stream: int = 2) -> np.ndarray:
    """Video-style mask: per frame (last mode) the (mode0, mode1) plane is cut into
    block x block tiles, each missing with probability p_missing, shared by all
    channels (mode 2)."""
    g = rng(seed, stream)
    H, W = dims[0], dims[1]
    nbh, nbw = -(-H // block), -(-W // block)
    frames = int(np.prod(dims[3:])) if len(dims) > 3 else 1
    keep = g.random((nbh, nbw, frames)) >= p_missing
    plane = np.repeat(np.repeat(keep, block, axis=0), block, axis=1)[:H, :W, :]
    chans = dims[2] if len(dims) > 2 else 1
    m = np.broadcast_to(plane[:, :, None, :], (H, W, chans, frames)).astype(np.uint8)
    return np.asfortranarray(m.reshape(dims))


def select_observed(mask: np.ndarray, frac: float, seed: int, stream: int = 3):
    """Pick each observed entry independently with probability frac.

    Returns (sel, u): sel is a uint8 array (1 = chosen), u an array of uniforms in
    [0, 1) drawn for every entry (used for outlier values / signs)."""
    g = rng(seed, stream)
    n = mask.size
    sel = np.empty(n, dtype=np.uint8)
    u = np.empty(n, dtype=np.float64)
    mflat = mask.ravel(order="F")
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        sel[s:e] = (g.random(e - s) < frac) & (mflat[s:e] != 0)
        u[s:e] = g.random(e - s)
    return sel.reshape(mask.shape, order="F"), u.reshape(mask.shape, order="F")


# ----------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple
    ranks: tuple
    rho: float                 # observed fraction
    outlier_frac: float        # fraction of observed entries replaced
    outlier_law: str           # 'uniform_std', 'saltpepper', 'uniform01'
    outlier_scale: float = 0.0 # k in U[-k*std, k*std]
    noise_var: float = 0.0     # additive Gaussian noise variance on all entries
    core_std: Optional[float] = None   # default 1/sqrt(r) (unit-variance entries)
    mask_kind: str = "bernoulli"
    lowpass: bool = False
    normalise_max: bool = False
    sketch: Optional[tuple] = None     # per-mode sample sizes for the RStS path
    dtype: str = "f32"


WORKLOADS = {
    # 30^3, ranks 3, N(0,1) cores, 50% missing, 10% outliers U[-10 std, 10 std], FP64
    "tr3_30_r3": Workload("tr3_30_r3", (30, 30, 30), (3, 3, 3), 0.5, 0.10, "uniform_std", 10.0,
                          core_std=1.0, dtype="f64"),
    # 100^4, rank 5, 70% missing, N(0, 1e-3) noise, 20% salt and pepper at +-max|X|,
    # RStS with 20 indices per mode
    "tr4_100_r5": Workload("tr4_100_r5", (100, 100, 100, 100), (5, 5, 5, 5), 0.3, 0.20,
                           "saltpepper", noise_var=1e-3, sketch=(20, 20, 20, 20)),
    # video-shaped 240x320x3x200, rank 8, smooth modes 0/1, 80% missing in 16x16 blocks,
    # 10% outliers U[0,1], RStS with s_j = min(I_j, 32)
    "video_240x320x3x200_r8": Workload("video_240x320x3x200_r8", (240, 320, 3, 200), (8, 8, 8, 8),
                                       0.2, 0.10, "uniform01", mask_kind="block16", lowpass=True,
                                       normalise_max=True, sketch=(32, 32, 3, 32)),
    # 60^5, rank 8, 90% missing, 15% outliers U[-20 std, 20 std]
    "tr5_60_r8": Workload("tr5_60_r8", (60, 60, 60, 60, 60), (8, 8, 8, 8, 8), 0.1, 0.15,
                          "uniform_std", 20.0),
    # 200^4, rank 10, 95% missing, 10% outliers U[-10 std, 10 std]
    "tr4_200_r10": Workload("tr4_200_r10", (200, 200, 200, 200), (10, 10, 10, 10), 0.05, 0.10,
                            "uniform_std", 10.0),
}


def scaled(w: Workload, dims) -> Workload:
    """The same recipe on other dimensions (for small parity cases)."""
    return dataclasses.replace(w, dims=tuple(dims), name=f"{w.name}@{'x'.join(map(str, dims))}")


def assemble(w: Workload, xstar: np.ndarray, mask: np.ndarray, seed: int) -> np.ndarray:
    """Observed tensor = clean tensor + noise, with a fraction of observed entries
    replaced by gross outliers.  Pure input assembly (no method arithmetic)."""
    X = np.array(xstar, dtype=np.float64, order="F", copy=True)
    if w.noise_var > 0:
        g = rng(seed, 4)
        flat = X.reshape(-1, order="F")
        for s in range(0, flat.size, _CHUNK):
            e = min(flat.size, s + _CHUNK)
            flat[s:e] += g.standard_normal(e - s) * math.sqrt(w.noise_var)
        X = flat.reshape(X.shape, order="F")
    if w.outlier_frac > 0:
        sel, u = select_observed(mask, w.outlier_frac, seed)
        sel = sel.astype(bool)
        if w.outlier_law == "uniform_std":
            std = float(np.std(xstar))
            X[sel] = (2.0 * u[sel] - 1.0) * w.outlier_scale * std
        elif w.outlier_law == "saltpepper":
            mx = float(np.max(np.abs(xstar)))
            X[sel] = np.where(u[sel] < 0.5, -mx, mx)
        elif w.outlier_law == "uniform01":
            X[sel] = u[sel]
        else:
            raise ValueError(w.outlier_law)
    return X


def make_workload(w: Workload, seed: int, reconstruct: Callable[[List[np.ndarray]], np.ndarray],
                  dims=None):
    """Draw one instance: (cores_true, xstar, mask, X).

    ``reconstruct(cores) -> ndarray(dims)`` builds the clean tensor from its cores."""
    dims = tuple(dims or w.dims)
    ranks = w.ranks
    std = w.core_std if w.core_std is not None else 1.0 / math.sqrt(ranks[0])
    if w.lowpass:
        cores = lowpass_cores(dims, ranks, seed, std)
    else:
        cores = gaussian_cores(dims, ranks, seed, std)
    xstar = np.asarray(reconstruct(cores), dtype=np.float64)
    if w.normalise_max:
        mx = float(np.max(np.abs(xstar)))
        xstar = xstar / mx
        # keep exact TR rank: scale the first core by the same factor
        cores = [cores[0] / mx] + list(cores[1:])
    if w.mask_kind == "bernoulli":
        mask = bernoulli_mask(dims, w.rho, seed)
    elif w.mask_kind == "block16":
        mask = block_mask(dims, 16, 1.0 - w.rho, seed)
    else:
        raise ValueError(w.mask_kind)
    X = assemble(w, xstar, mask, seed)
    return cores, xstar, mask, X


def init_cores(dims, ranks, seed: int, std: Optional[float] = None) -> List[np.ndarray]:
    """Starting cores for a fit: iid N(0, std^2), std defaults to 1/sqrt(r)."""
    if std is None:
        std = 1.0 / math.sqrt(ranks[0])
    return gaussian_cores(dims, ranks, seed + 1, std, stream=7)


def perturbed_cores(cores, seed: int, rel: float = 0.1) -> List[np.ndarray]:
    """Cores near a given point: Z + N(0, rel/r) per entry."""
    g = rng(seed, 8)
    out = []
    for Z in cores:
        r = Z.shape[0]
        out.append(Z + g.standard_normal(Z.shape) * math.sqrt(rel / r))
    return out
