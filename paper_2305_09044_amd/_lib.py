"""ctypes binding of libtrd (include/trd.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch tensors to
device pointers, the current torch stream to a hipStream_t and status codes to
exceptions.  Importing it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrd.so")

TRD_OK = 0
TRD_EINVAL = -1
TRD_ENOMEM = -2
TRD_EDEVICE = -3
TRD_ENOTSPD = -4
TRD_ESTATE = -5
TRD_EUNSUPPORTED = -6
TRD_F32, TRD_F64 = 0, 1
TRD_PREC_NATIVE, TRD_PREC_BF16, TRD_PREC_BF16X3 = 0, 1, 2
PRECISIONS = {"native": TRD_PREC_NATIVE, "bf16": TRD_PREC_BF16, "bf16x3": TRD_PREC_BF16X3}
TRD_DIR_SCALED, TRD_DIR_GRADIENT = 0, 1
TRD_GRAM_GLOBAL, TRD_GRAM_LOCAL = 0, 1
DIRECTIONS = {"scaled": TRD_DIR_SCALED, "gradient": TRD_DIR_GRADIENT}
GRAMS = {"global": TRD_GRAM_GLOBAL, "local": TRD_GRAM_LOCAL}
TRD_SAMPLE_RSTS, TRD_SAMPLE_ROWS, TRD_SAMPLE_LEVERAGE = 0, 1, 2
SAMPLINGS = {"rsts": TRD_SAMPLE_RSTS, "rows": TRD_SAMPLE_ROWS, "leverage": TRD_SAMPLE_LEVERAGE}
TRD_FLAG_EMPTY, TRD_FLAG_ZERO_DEN, TRD_FLAG_NOTSPD, TRD_FLAG_CLAMPED = 1, 2, 4, 8
TRD_SIGMA_FIXED, TRD_SIGMA_GIVEN, TRD_SIGMA_QUANTILE = 0, 1, 2

_NAMES = {0: "TRD_OK", -1: "TRD_EINVAL", -2: "TRD_ENOMEM", -3: "TRD_EDEVICE", -4: "TRD_ENOTSPD",
          -5: "TRD_ESTATE", -6: "TRD_EUNSUPPORTED"}


class TrdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class trd_sketch(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("sweep", C.c_int32), ("sizes", C.c_int32 * 8),
                ("idx", C.POINTER(C.c_void_p))]


class trd_fit_opts(C.Structure):
    _fields_ = [("max_sweeps", C.c_int32), ("tol", C.c_double), ("lambda_rel", C.c_double),
                ("sigma_mode", C.c_int32), ("sigma", C.c_double),
                ("sigma_given", C.POINTER(C.c_double)), ("q", C.c_double), ("c", C.c_double),
                ("shrink", C.c_double), ("sigma_min_rel", C.c_double), ("use_sketch", C.c_int32),
                ("sketch_sizes", C.c_int32 * 8), ("seed", C.c_uint64), ("precision", C.c_int32)]


class trd_fit_report(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("last_e", C.c_double), ("last_sigma", C.c_double),
                ("flags", C.c_uint32), ("e_hist", C.POINTER(C.c_double)),
                ("sigma_hist", C.POINTER(C.c_double)), ("eta_hist", C.POINTER(C.c_double))]


_lib = None


def load() -> C.CDLL:
    """Load libtrd.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_09044_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "trd_create": (i32, [P(vp), i32]),
        "trd_destroy": (None, [vp]),
        "trd_last_error": (C.c_char_p, [vp]),
        "trd_set_shape": (i32, [vp, i32, P(i64), P(C.c_int32), i32]),
        "trd_set_problem": (i32, [vp, i32, P(i64), P(C.c_int32), i32, vp, vp, vp]),
        "trd_problem_info": (i32, [vp, P(i64), P(C.c_size_t), P(C.c_int32)]),
        "trd_reconstruct": (i32, [vp, P(vp), vp, i64, vp, vp]),
        "trd_weights": (i32, [vp, i64, i32, dbl, vp, vp]),
        "trd_grad": (i32, [vp, P(vp), i32, dbl, P(trd_sketch), vp, vp, vp]),
        "trd_fgmc_gram": (i32, [vp, P(vp), i32, vp, vp]),
        "trd_step": (i32, [vp, P(vp), i32, dbl, dbl, P(trd_sketch), vp, vp, vp]),
        "trd_fit": (i32, [vp, P(vp), P(trd_fit_opts), P(trd_fit_report), vp]),
        "trd_loss_fwd": (i32, [vp, P(vp), dbl, vp, vp]),
        "trd_loss_bwd": (i32, [vp, P(vp), dbl, dbl, P(vp), vp]),
        "trd_sample_sketch": (i32, [C.c_uint64, i32, i32, i32, P(i64), P(C.c_int32), P(vp), vp]),
        "trd_sample_rows": (i32, [C.c_uint64, i32, i32, i32, P(i64), i64, vp, vp]),
        "trd_sample_leverage": (i32, [vp, P(vp), i32, C.c_uint64, i32, i64, dbl, vp, vp, vp]),
        "trd_workspace_bytes": (i32, [i32, i32, P(i64), P(C.c_int32), i32, i32, i64, P(C.c_size_t),
                                      P(C.c_size_t)]),
        "trd_sample_mask": (i32, [C.c_uint64, i32, P(i64), dbl, i32, dbl, vp, vp, vp, vp]),
        "trd_fgmc_gram_noalloc": (i32, [i32, P(i64), P(C.c_int32), i32, P(vp), i32, vp, vp]),
        "trd_set_precision": (i32, [vp, i32]),
        "trd_set_variant": (i32, [vp, i32, i32, i32]),
        "trd_profile": (i32, [vp, i32]),
        "trd_profile_read": (i32, [vp, P(i64), P(dbl), P(i64), P(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, ctx=None):
    if code != TRD_OK:
        msg = load().trd_last_error(ctx).decode(errors="replace")
        raise TrdError(code, msg)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _ptr_array(ts: Sequence[torch.Tensor]):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t).value
    return arr


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return TRD_F32
    if dt == torch.float64:
        return TRD_F64
    raise ValueError(f"unsupported dtype {dt}")


def make_sketch(sizes: Sequence[int], seed: int = 0, sweep: int = 0,
                idx: Optional[Sequence[Optional[torch.Tensor]]] = None):
    """trd_sketch; idx (optional) holds one int32 device tensor per mode (None for k)."""
    s = trd_sketch()
    s.seed = int(seed)
    s.sweep = int(sweep)
    for j, v in enumerate(sizes):
        s.sizes[j] = int(v)
    keep = None
    if idx is not None:
        arr = (C.c_void_p * 8)()
        for j, t in enumerate(idx):
            arr[j] = None if t is None else _ptr(t).value
        s.idx = C.cast(arr, C.POINTER(C.c_void_p))
        keep = arr
    return s, keep


def trd_weights(resid: torch.Tensor, sigma: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib = load()
    out = torch.empty_like(resid) if out is None else out
    _check(lib.trd_weights(_ptr(resid), resid.numel(), _dtype_code(resid.dtype), float(sigma),
                           _ptr(out), C.c_void_p(_stream())))
    return out


def trd_workspace_bytes(dims: Sequence[int], ranks: Sequence[int], n_obs: int,
                        dtype: torch.dtype = torch.float32, precision: str = "native",
                        device: int = 0) -> dict:
    """Device workspace of a problem of this shape before binding it: {'bound', 'typical'}
    (bytes; see include/trd.h)."""
    lib = load()
    N = len(dims)
    d = (C.c_int64 * N)(*[int(v) for v in dims])
    r = (C.c_int32 * N)(*[int(v) for v in ranks])
    b, t = C.c_size_t(), C.c_size_t()
    _check(lib.trd_workspace_bytes(int(device), N, d, r, _dtype_code(dtype), PRECISIONS[precision],
                                   int(n_obs), C.byref(b), C.byref(t)))
    return {"bound": b.value, "typical": t.value}


def trd_sample_mask(seed: int, dims: Sequence[int], rho: float, block: int = 0,
                    outlier_frac: float = 0.0, outliers: bool = False, uniforms: bool = False,
                    device="cuda"):
    """Observation mask (uint8, column-major flat), and optionally the outlier selection
    (uint8) and the per-entry uniforms (float64), drawn on the device (trd_sample_mask)."""
    lib = load()
    N = len(dims)
    n = math.prod(int(v) for v in dims)
    mask = torch.empty(n, dtype=torch.uint8, device=device)
    sel = torch.empty(n, dtype=torch.uint8, device=device) if outliers else None
    u = torch.empty(n, dtype=torch.float64, device=device) if uniforms else None
    d = (C.c_int64 * N)(*[int(v) for v in dims])
    _check(lib.trd_sample_mask(int(seed), N, d, float(rho), int(block), float(outlier_frac),
                               _ptr(mask), _ptr(sel), _ptr(u), C.c_void_p(_stream())))
    return mask, sel, u


def trd_fgmc_gram_noalloc(cores: Sequence[torch.Tensor], dims: Sequence[int], ranks: Sequence[int],
                          k: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """G^{!=k} of eq. 13 by the context-free entry point that allocates no device memory
    (its factors live in the library's fixed per-device scratch array)."""
    lib = load()
    N = len(dims)
    R = int(ranks[k]) * int(ranks[(k + 1) % N])
    dev = cores[(k + 1) % N].device
    out = torch.empty((R, R), dtype=torch.float64, device=dev) if out is None else out
    d = (C.c_int64 * N)(*[int(v) for v in dims])
    r = (C.c_int32 * N)(*[int(v) for v in ranks])
    _check(lib.trd_fgmc_gram_noalloc(N, d, r, _dtype_code(cores[(k + 1) % N].dtype),
                                     _ptr_array(cores), int(k), _ptr(out), C.c_void_p(_stream())))
    return out


def trd_sample_sketch(seed: int, t: int, k: int, dims: Sequence[int], sizes: Sequence[int],
                      device="cuda") -> list:
    lib = load()
    N = len(dims)
    outs = [torch.empty(int(dims[j]) if j == k else int(min(sizes[j], dims[j])), dtype=torch.int32,
                        device=device) for j in range(N)]
    d = (C.c_int64 * N)(*[int(v) for v in dims])
    s = (C.c_int32 * N)(*[int(v) for v in sizes])
    _check(lib.trd_sample_sketch(int(seed), int(t), int(k), N, d, s, _ptr_array(outs),
                                 C.c_void_p(_stream())))
    return outs


def trd_sample_rows(seed: int, t: int, k: int, dims: Sequence[int], J: int, device="cuda"):
    """The uniform row sample of update k in sweep t: (J,) int64 row indices of the
    subchain unfolding (see include/trd.h)."""
    lib = load()
    N = len(dims)
    out = torch.empty(int(J), dtype=torch.int64, device=device)
    d = (C.c_int64 * N)(*[int(v) for v in dims])
    _check(lib.trd_sample_rows(int(seed), int(t), int(k), N, d, int(J), C.c_void_p(out.data_ptr()),
                               C.c_void_p(_stream())))
    return out


class Problem:
    """One bound problem (trd_create + trd_set_problem).  Keeps X and mask alive."""

    def __init__(self, X: Optional[torch.Tensor], mask: Optional[torch.Tensor], dims: Sequence[int],
                 ranks: Sequence[int], device: Optional[int] = None, dtype: torch.dtype = torch.float32):
        """X/mask None binds only the shape (reconstruction and Gram only)."""
        lib = load()
        self.dims = [int(v) for v in dims]
        self.ranks = [int(v) for v in ranks]
        self.N = len(dims)
        d = (C.c_int64 * self.N)(*self.dims)
        r = (C.c_int32 * self.N)(*self.ranks)
        self._ctx = C.c_void_p()
        if X is None:
            self.dtype = dtype
            self.X = self.mask = None
            self.device = torch.device("cuda", device or 0)
            _check(lib.trd_create(C.byref(self._ctx), int(device or 0)))
            _check(lib.trd_set_shape(self._ctx, self.N, d, r, _dtype_code(dtype)), self._ctx)
            return
        if X.numel() != math.prod(dims) or mask.numel() != X.numel():
            raise ValueError("X / mask size does not match dims")
        if mask.dtype != torch.uint8:
            raise ValueError("mask must be uint8")
        self.dtype = X.dtype
        self.X = X.contiguous()
        self.mask = mask.contiguous()
        self.device = X.device
        dev = X.device.index if device is None else device
        _check(lib.trd_create(C.byref(self._ctx), int(dev or 0)))
        _check(lib.trd_set_problem(self._ctx, self.N, d, r, _dtype_code(X.dtype), _ptr(self.X),
                                   _ptr(self.mask), C.c_void_p(_stream())), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load().trd_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries
    def info(self):
        n = C.c_int64()
        ws = C.c_size_t()
        sp = (C.c_int32 * 8)()
        _check(load().trd_problem_info(self._ctx, C.byref(n), C.byref(ws), sp), self._ctx)
        return {"n_obs": n.value, "workspace_bytes": ws.value, "split": list(sp)[: self.N]}

    def core_numel(self, k: int) -> int:
        return self.ranks[k] * self.dims[k] * self.ranks[(k + 1) % self.N]

    # -- the calls of include/trd.h
    def reconstruct(self, cores, lin_idx: Optional[torch.Tensor] = None) -> torch.Tensor:
        n = lin_idx.numel() if lin_idx is not None else math.prod(self.dims)
        out = torch.empty(n, dtype=self.dtype, device=self.device)
        _check(load().trd_reconstruct(self._ctx, _ptr_array(cores), _ptr(lin_idx), n, _ptr(out),
                                      C.c_void_p(_stream())), self._ctx)
        return out

    def grad(self, cores, k: int, sigma: float, sketch=None):
        d = torch.empty(self.core_numel(k), dtype=self.dtype, device=self.device)
        stats = torch.zeros(3, dtype=torch.float64, device=self.device)
        sk = C.byref(sketch) if sketch is not None else None
        _check(load().trd_grad(self._ctx, _ptr_array(cores), int(k), float(sigma), sk, _ptr(d),
                               _ptr(stats), C.c_void_p(_stream())), self._ctx)
        return d, stats

    def fgmc_gram(self, cores, k: int) -> torch.Tensor:
        R = self.ranks[k] * self.ranks[(k + 1) % self.N]
        G = torch.empty(R * R, dtype=torch.float64, device=self.device)
        _check(load().trd_fgmc_gram(self._ctx, _ptr_array(cores), int(k), _ptr(G),
                                    C.c_void_p(_stream())), self._ctx)
        return G.view(R, R)

    def step(self, cores, k: int, sigma: float, lambda_rel: float = 1e-9, sketch=None):
        eta = torch.zeros(1, dtype=torch.float64, device=self.device)
        flags = torch.zeros(1, dtype=torch.int32, device=self.device)
        sk = C.byref(sketch) if sketch is not None else None
        _check(load().trd_step(self._ctx, _ptr_array(cores), int(k), float(sigma), float(lambda_rel),
                               sk, _ptr(eta), _ptr(flags), C.c_void_p(_stream())), self._ctx)
        return eta, flags

    def fit(self, cores, max_sweeps=30, tol=1e-3, lambda_rel=1e-9, sigma_mode="quantile",
            sigma=math.inf, sigma_given=None, q=0.5, c=5.0, shrink=0.5, sigma_min_rel=1e-6,
            sketch_sizes=None, seed=0, precision="native"):
        o = trd_fit_opts()
        o.max_sweeps = int(max_sweeps)
        o.tol = float(tol)
        o.lambda_rel = float(lambda_rel)
        o.sigma_mode = {"fixed": TRD_SIGMA_FIXED, "given": TRD_SIGMA_GIVEN,
                        "quantile": TRD_SIGMA_QUANTILE}[sigma_mode]
        o.sigma = float(sigma)
        given = None
        if sigma_given is not None:
            given = (C.c_double * len(sigma_given))(*[float(v) for v in sigma_given])
            o.sigma_given = C.cast(given, C.POINTER(C.c_double))
        o.q, o.c, o.shrink, o.sigma_min_rel = float(q), float(c), float(shrink), float(sigma_min_rel)
        o.use_sketch = 1 if sketch_sizes is not None else 0
        if sketch_sizes is not None:
            for j, v in enumerate(sketch_sizes):
                o.sketch_sizes[j] = int(v)
        o.seed = int(seed)
        o.precision = PRECISIONS[precision]
        rep = trd_fit_report()
        eh = (C.c_double * max_sweeps)()
        sh = (C.c_double * max_sweeps)()
        th = (C.c_double * (max_sweeps * self.N))()
        rep.e_hist = C.cast(eh, C.POINTER(C.c_double))
        rep.sigma_hist = C.cast(sh, C.POINTER(C.c_double))
        rep.eta_hist = C.cast(th, C.POINTER(C.c_double))
        code = load().trd_fit(self._ctx, _ptr_array(cores), C.byref(o), C.byref(rep),
                              C.c_void_p(_stream()))
        n = rep.sweeps
        out = {"sweeps": n, "last_e": rep.last_e, "last_sigma": rep.last_sigma, "flags": rep.flags,
               "e": list(eh)[:n], "sigma": list(sh)[:n],
               "eta": [list(th)[t * self.N:(t + 1) * self.N] for t in range(n)], "status": code}
        if code not in (TRD_OK, TRD_ENOTSPD):
            _check(code, self._ctx)
        return out

    def loss_fwd(self, cores, sigma: float) -> torch.Tensor:
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(load().trd_loss_fwd(self._ctx, _ptr_array(cores), float(sigma), _ptr(out),
                                   C.c_void_p(_stream())), self._ctx)
        return out

    def loss_bwd(self, cores, sigma: float, grad_scale: float = 1.0):
        grads = [torch.empty_like(c) for c in cores]
        _check(load().trd_loss_bwd(self._ctx, _ptr_array(cores), float(sigma), float(grad_scale),
                                   _ptr_array(grads), C.c_void_p(_stream())), self._ctx)
        return grads

    def set_precision(self, precision: str):
        code = PRECISIONS[precision]
        _check(load().trd_set_precision(self._ctx, code), self._ctx)

    def set_variant(self, direction: str = "scaled", gram: str = "global", sampling: str = "rsts"):
        """Update variants of the Sec. 6.1 ablations: direction 'scaled' | 'gradient',
        gram 'global' | 'local' (the sampled cores' Gram under a sketch), sampling 'rsts' |
        'rows' | 'leverage' (a sketch draws rows of the subchain unfolding instead: uniform, or
        by leverage with importance weights)."""
        _check(load().trd_set_variant(self._ctx, DIRECTIONS[direction], GRAMS[gram], SAMPLINGS[sampling]),
               self._ctx)

    def sample_leverage(self, cores, k: int, seed: int, t: int, J: int, lambda_rel: float = 1e-9):
        """The leverage-score row sample of update k in sweep t: (rows int64, weights FP64)."""
        dev = cores[0].device
        rows = torch.empty(int(J), dtype=torch.int64, device=dev)
        w = torch.empty(int(J), dtype=torch.float64, device=dev)
        _check(load().trd_sample_leverage(self._ctx, _ptr_array(cores), int(k), int(seed), int(t), int(J),
                                          float(lambda_rel), C.c_void_p(rows.data_ptr()),
                                          C.c_void_p(w.data_ptr()), C.c_void_p(_stream())), self._ctx)
        return rows, w

    def profile(self, enable: bool):
        _check(load().trd_profile(self._ctx, 1 if enable else 0), self._ctx)

    def profile_read(self):
        n, ms, sl, en = C.c_int64(), C.c_double(), C.c_int64(), C.c_int64()
        _check(load().trd_profile_read(self._ctx, C.byref(n), C.byref(ms), C.byref(sl), C.byref(en)),
               self._ctx)
        return {"launches": n.value, "total_ms": ms.value, "slots": sl.value, "entries": en.value}


def header_functions(header_path: Optional[str] = None) -> list:
    """Names of the functions declared in include/trd.h."""
    import re
    if header_path is None:
        header_path = os.path.join(os.path.dirname(_HERE), "include", "trd.h")
    txt = open(header_path).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(trd_\w+)\s*\(", txt, re.M)))
