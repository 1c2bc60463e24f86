"""Shared test plumbing: seeded inputs on host and device (no method arithmetic)."""
from __future__ import annotations

import math

import numpy as np

import synth


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def host_problem(dims, ranks, rho, seed, dtype=np.float32, outlier_frac=0.1, reconstruct=None,
                 mask_kind="bernoulli"):
    """(X (F-ordered, dtype-rounded, as float64), mask, starting cores rounded to dtype)."""
    w = synth.Workload("t", tuple(dims), tuple(ranks), rho, outlier_frac, "uniform_std", 10.0,
                       noise_var=1e-3, mask_kind=mask_kind)
    Zt, xstar, mask, X = synth.make_workload(w, seed, reconstruct)
    X = X.astype(dtype).astype(np.float64)
    Z0 = [z.astype(dtype).astype(np.float64) for z in synth.init_cores(dims, ranks, seed)]
    return X, mask, Z0, Zt, xstar


def device_problem(X, mask, dims, ranks, dtype):
    import torch
    import paper_2305_09044_amd as trd
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    Xd = torch.from_numpy(np.asarray(X, dtype=dtype).ravel(order="F").copy()).to("cuda")
    Pd = torch.from_numpy(np.asarray(mask, dtype=np.uint8).ravel(order="F").copy()).to("cuda")
    assert Xd.dtype == tdt
    return trd.Problem(Xd, Pd, dims, ranks)


def device_cores(Z, dtype):
    import torch
    return [torch.from_numpy(f).to("cuda") for f in synth.cores_to_flat(Z, dtype)]


def host_cores(cores, dims, ranks):
    return synth.flat_to_cores([c.detach().cpu().numpy() for c in cores], dims, ranks)


def unflatten_d(dflat, r, I, r2):
    """core-layout flat gradient -> (I x r*r2) unfolding with column a + b*r."""
    return np.asarray(dflat, dtype=np.float64).reshape(I, r2 * r)
