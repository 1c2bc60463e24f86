"""Counter-based index sampling for randomized subtensor sketching (oracle side).

RStS (Sec. 4.3.2 and Alg. 1) draws, for every core update k of sweep t and every
mode j != k, an index set I_j of s_j lateral slices uniformly at random; I_k is the
whole range.  The paper does not fix the sampling law or generator.  Reading used
here (and by the library, which implements the same published generator on its
own): uniform without replacement, sorted ascending, fresh for every (t, k, j).

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  The n-th output (n = 1, 2, ...) of a SplitMix64 stream
seeded with s is mix64(s + n * GOLDEN); ``counter_u64(key, c)`` is output c + 1.
Bounded integers: Lemire's multiply-shift with rejection ("Fast random integer
generation in an interval", ACM TOMACS 2019) on the top 32 bits.
Subset: Floyd's algorithm (Bentley and Floyd, "A sample of brilliance", CACM 1987).
Everything is integer-only, so any two faithful implementations agree bit for bit.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
DOMAIN_RSTS = 0x5253545300000000  # "RStS" tag separating this use from others


def mix64(z: int) -> int:
    """SplitMix64 output function."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, n: int) -> List[int]:
    """First n outputs of the sequential SplitMix64 generator seeded with ``seed``."""
    s = seed & M64
    out = []
    for _ in range(n):
        s = (s + GOLDEN) & M64
        out.append(mix64(s))
    return out


def counter_u64(key: int, ctr: int) -> int:
    """Output number ctr + 1 of the SplitMix64 stream seeded with key."""
    return mix64((key + (ctr + 1) * GOLDEN) & M64)


def sketch_key(seed: int, t: int, k: int, j: int) -> int:
    """Stream key for sweep t, core update k, sampled mode j."""
    a = counter_u64((seed ^ DOMAIN_RSTS) & M64, t)
    b = counter_u64(a, k)
    return counter_u64(b, j)


def bounded(key: int, ctr: int, n: int):
    """Uniform integer in [0, n) (1 <= n <= 2^32) and the next counter value."""
    assert 1 <= n <= (1 << 32)
    threshold = ((1 << 32) - n) % n
    while True:
        x = counter_u64(key, ctr) >> 32
        ctr += 1
        m = x * n
        if (m & 0xFFFFFFFF) >= threshold:
            return m >> 32, ctr


def floyd_sample(key: int, n: int, s: int) -> List[int]:
    """s distinct indices from [0, n), uniform, sorted ascending (s >= n: all)."""
    if s >= n:
        return list(range(n))
    chosen = set()
    ctr = 0
    for jj in range(n - s, n):
        t, ctr = bounded(key, ctr, jj + 1)
        chosen.add(jj if t in chosen else t)
    return sorted(chosen)


def sketch_indices(seed: int, t: int, k: int, dims: Sequence[int], sizes: Sequence[int]):
    """Index sets I_1..I_N for update k of sweep t; mode k takes every index."""
    out = []
    for j, (I, s) in enumerate(zip(dims, sizes)):
        if j == k:
            out.append(list(range(I)))
        else:
            out.append(floyd_sample(sketch_key(seed, t, k, j), I, s))
    return out


# ----------------------------------------------------------------------------------
# uniform row sampling (the ablation of Sec. 6.1 that replaces RStS)
#
# Update k of sweep t draws J rows of Z^{!=k}_{[2]} independently and uniformly, with
# replacement: sample n takes, for every mode j != k, the index
# bounded(counter_u64(row_key(seed, t, k, j), n), 0, I_j) -- a fresh stream per (sample,
# mode), so every sample can be drawn on its own.  The row is the little-endian index over
# the cyclic modes k+1, ..., k-1 (the row order of Thm. 1).

DOMAIN_ROWS = 0x55524F5700000000  # "UROW"


def row_key(seed: int, t: int, k: int, j: int) -> int:
    """Stream key for sweep t, core update k, mode j of the uniform row sampler."""
    a = counter_u64((seed ^ DOMAIN_ROWS) & M64, t)
    b = counter_u64(a, k)
    return counter_u64(b, j)


def uniform_row_indices(seed: int, t: int, k: int, dims: Sequence[int], J: int) -> np.ndarray:
    """(J, N) per-mode indices of the sampled rows; column k is 0."""
    N = len(dims)
    out = np.zeros((J, N), dtype=np.int64)
    for j in range(N):
        if j == k:
            continue
        key = row_key(seed, t, k, j)
        for n in range(J):
            out[n, j] = bounded(counter_u64(key, n), 0, int(dims[j]))[0]
    return out


def uniform_rows(seed: int, t: int, k: int, dims: Sequence[int], J: int) -> np.ndarray:
    """(J,) row indices m of Z^{!=k}_{[2]} (little-endian over modes k+1, ..., k-1)."""
    N = len(dims)
    idx = uniform_row_indices(seed, t, k, dims, J)
    m = np.zeros(J, dtype=np.int64)
    stride = 1
    for s in range(1, N):
        j = (k + s) % N
        m += idx[:, j] * stride
        stride *= int(dims[j])
    return m


# ----------------------------------------------------------------------------------
# leverage-score row sampling (the ablation of Sec. 6.1 that applies TRALS-S's sampler)
#
# Sample n of update (t, k) draws, for every mode j != k, the uniform
# u = (u64 >> 11) 2^-53 of counter_u64(lev_key(seed, t, k, j), n); the index is then taken
# by inverse CDF from that mode's leverage distribution (computed by the caller).

DOMAIN_LEV = 0x4C45564500000000  # "LEVE"


def lev_key(seed: int, t: int, k: int, j: int) -> int:
    """Stream key for sweep t, core update k, mode j of the leverage sampler."""
    a = counter_u64((seed ^ DOMAIN_LEV) & M64, t)
    b = counter_u64(a, k)
    return counter_u64(b, j)


def uniform01(key: int, n) -> np.ndarray:
    """(counter_u64(key, c) >> 11) * 2^-53 for the counters c (exact doubles in [0, 1))."""
    return (counter_u64_np(key, np.asarray(n, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def sizes_from_J(J: int, dims: Sequence[int]) -> List[int]:
    """Per-mode sample size from the sample parameter J.

    The printed size rule is garbled (it evaluates to 1 for any real tensor); the
    reading used here takes the (N-1)-th root: s_j = min(I_j, ceil(J^(1/(N-1)))),
    computed exactly as the least integer s with s^(N-1) >= J."""
    N = len(dims)
    lo, hi = 1, max(1, int(J))
    while lo < hi:
        mid = (lo + hi) // 2
        if mid ** (N - 1) >= J:
            hi = mid
        else:
            lo = mid + 1
    return [min(I, lo) for I in dims]


# ----------------------------------------------------------------------------------
# observation pattern: mask, outlier selection, per-entry uniforms
#
# Same generator, other keys: u(seed ^ "MASK", 0) for the mask, 1 for the outlier
# selection, 2 for the uniforms.  An event of probability p happens when the draw is below
# floor(p 2^64) (p >= 1: always; p <= 0: never).  Entry l is the column-major linear index.
# The mask draws once per entry, or once per block x block tile of modes 0 and 1 at each
# index of modes 3.. (shared by every index of mode 2, the colour channel of a video).

DOMAIN_MASK = 0x4D41534B00000000  # "MASK"


def mix64_np(z):
    """mix64 over a numpy uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def counter_u64_np(key: int, ctr):
    """counter_u64(key, c) for a numpy array of counters c."""
    c = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & M64) + (c + np.uint64(1)) * np.uint64(GOLDEN)
    return mix64_np(z)


def threshold(p: float):
    """floor(p 2^64) as a Python int, or None for an event that always happens."""
    if p >= 1.0:
        return None
    if not p > 0.0:
        return 0
    return int(math.ldexp(p, 64))


def _below(draws, p: float):
    thr = threshold(p)
    if thr is None:
        return np.ones(draws.shape, dtype=bool)
    return draws < np.uint64(thr)


def mask_keys(seed: int):
    base = (seed ^ DOMAIN_MASK) & M64
    return counter_u64(base, 0), counter_u64(base, 1), counter_u64(base, 2)


def mask_draw_index(lin, dims: Sequence[int], block: int):
    """Counter of the mask draw for entries lin: lin itself, or the entry's tile."""
    lin = np.asarray(lin, dtype=np.int64)
    if block <= 0:
        return lin.astype(np.uint64)
    i0 = lin % dims[0]
    rest = lin // dims[0]
    i1 = rest % dims[1]
    rest = rest // dims[1]
    if len(dims) >= 3:
        rest = rest // dims[2]
    nbh = -(-dims[0] // block)
    nbw = -(-dims[1] // block)
    return (i0 // block + nbh * (i1 // block + nbw * rest)).astype(np.uint64)


def sample_mask_at(seed: int, dims: Sequence[int], rho: float, block: int, frac: float, lin):
    """(mask, outlier selection, uniform) at the linear indices lin."""
    km, ko, ku = mask_keys(seed)
    lin = np.asarray(lin, dtype=np.int64)
    obs = _below(counter_u64_np(km, mask_draw_index(lin, dims, block)), rho)
    sel = obs & _below(counter_u64_np(ko, lin.astype(np.uint64)), frac) if frac > 0 else np.zeros_like(obs)
    u = (counter_u64_np(ku, lin.astype(np.uint64)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return obs.astype(np.uint8), sel.astype(np.uint8), u


def sample_mask(seed: int, dims: Sequence[int], rho: float, block: int = 0, frac: float = 0.0):
    """The whole pattern as flat column-major arrays (small tensors only)."""
    n = int(np.prod(dims))
    return sample_mask_at(seed, dims, rho, block, frac, np.arange(n, dtype=np.int64))
