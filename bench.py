"""Benchmark: observed entries/s per AWRTRD core sweep on one MI355X, BF16 vs FP32.

A step is one sweep of Alg. 1 over all cores (subchain tables, fused
reconstruct+weight+gradient pass, FGMC Gram, scaled direction, line-search pass,
update, kernel-width quantile and convergence matrix), with inputs resident in HBM.
Default workload (the precision form): 60^5 tensor from TR rank 8 Gaussian cores
(7.8e8 entries, FP32 storage), 10% observed, 15% of the observed entries replaced by
outliers uniform in [-20 std, 20 std]; `value` is the BF16 matrix-core path
(--precision fp32 times the plain FP32 path instead).

The differentiation-form workload (--workload tr4_200_r10: 200^4, TR rank 10, 5 %
observed, 10 % outliers) times one step of the correntropy loss's forward and its
all-core backward through the torch.autograd.Function instead; `value` counts the observed
entries of every core's gradient per step.

Inputs are drawn on the device: the clean tensor by the library's reconstruction from
seeded Gaussian cores, the mask, outlier selection and outlier values by trd_sample_mask.

Prints one JSON line.  `equal_accuracy` fits both precisions from the same start and
reports the sweeps and time each needs to reach the BF16 recovery-error plateau, over
several seeds.  The roofline object covers the dominant kernel (the fused gradient pass),
timed with HIP events around each of its launches in the timed region, with its matrix-core
work beside it; cpu_baseline is the FP64 numpy oracle on a bounded sample of the same recipe.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "observed entries/sec per AWRTRD core sweep, BF16 vs FP32, at equal rel. error"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
PASS_SRC = os.path.join(ROOT, "paper_2305_09044_amd", "csrc", "kernels_pass.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grad_pass.json")
# workloads timed as the differentiation form (loss forward + all-core backward)
BACKWARD_WORKLOADS = ("tr4_200_r10",)
# default bounded samples of the CPU oracle (same recipe, smaller dims, every mode >= 2)
CPU_SAMPLES = {"tr5_60_r8": (30, 30, 30, 30, 30), "tr4_200_r10": (60, 60, 60, 60),
               "tr4_100_r5": (100, 100, 100, 12), "video_240x320x3x200_r8": (240, 320, 3, 20),
               "tr3_30_r3": (30, 30, 30)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(precision: str = "fp32") -> str:
    """Hash of the gradient pass's source and of the host code that plans its launches
    (grid, column groups, tables): the stored traffic is valid only for these sources."""
    src = PASS_SRC if precision == "fp32" else PASS_SRC.replace("kernels_pass", "kernels_tile")
    h = hashlib.sha256()
    for f in (src, os.path.join(os.path.dirname(src), "trd_api.cpp"),
              os.path.join(os.path.dirname(src), "trd_internal.h")):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def noise_seed(seed: int, stream: int) -> int:
    """Seed of the uniform stream `stream` (1, 2) of a workload's additive noise."""
    return (int(seed) ^ (0x4E4F495345000000 + stream)) & ((1 << 64) - 1)


def build_inputs(wname: str, seed: int, dims=None):
    """Seeded workload on the device: the clean tensor X* from the library's reconstruction
    of seeded Gaussian cores (synth), additive noise, then the mask, the outlier selection
    and the outlier values, every random number from the counter generator of
    trd_sample_mask.  Returns (workload, dims, X, mask, X*, true cores (host))."""
    import numpy as np
    import torch
    import synth
    import paper_2305_09044_amd as trd

    w = synth.WORKLOADS[wname]
    dims = tuple(dims or w.dims)
    std = w.core_std if w.core_std is not None else 1.0 / math.sqrt(w.ranks[0])
    cores_t = (synth.lowpass_cores(dims, w.ranks, seed, std) if w.lowpass
               else synth.gaussian_cores(dims, w.ranks, seed, std))
    npdt = np.float64 if w.dtype == "f64" else np.float32
    tdt = torch.float64 if w.dtype == "f64" else torch.float32
    shape = trd.Problem(None, None, dims, w.ranks, dtype=tdt)
    ct = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(cores_t, npdt)]
    xs = shape.reconstruct(ct)
    shape.close()
    del ct
    if w.normalise_max:  # keeps the exact TR rank: the first core scaled by the same factor
        mx = float(xs.abs().max())
        xs /= mx
        cores_t = [cores_t[0] / mx] + list(cores_t[1:])
    block = 16 if w.mask_kind == "block16" else 0
    want_out = w.outlier_frac > 0
    Pd, sel, u = trd.trd_sample_mask(seed, dims, w.rho, block, w.outlier_frac, outliers=want_out,
                                     uniforms=want_out)
    X = xs.clone()
    if w.noise_var > 0:
        # N(0, noise_var) by Box-Muller from two per-entry uniform streams of the same counter
        # generator (noise seeds derived from the workload seed), so that any entry's value
        # can be recomputed from the seed alone
        _, _, u1 = trd.trd_sample_mask(noise_seed(seed, 1), dims, 1.0, 0, 0.0, uniforms=True)
        _, _, u2 = trd.trd_sample_mask(noise_seed(seed, 2), dims, 1.0, 0, 0.0, uniforms=True)
        z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos((2.0 * math.pi) * u2)
        del u1, u2
        X += (z * math.sqrt(w.noise_var)).to(X.dtype)
        del z
    if want_out:
        selb = sel.bool()
        del sel
        if w.outlier_law == "uniform_std":
            sd = float(xs.double().std(unbiased=False))
            val = (2.0 * u[selb] - 1.0) * (w.outlier_scale * sd)
        elif w.outlier_law == "saltpepper":
            mx = float(xs.abs().max())
            val = torch.where(u[selb] < 0.5, -mx, mx)
        elif w.outlier_law == "uniform01":
            val = u[selb]
        else:
            raise ValueError(w.outlier_law)
        del u
        X[selb] = val.to(X.dtype)
        del val, selb
    torch.cuda.synchronize()
    return w, dims, X, Pd, xs, cores_t


def recovery_error(prob, cores, xstar_d, idx) -> float:
    """||Xhat - X*|| / ||X*|| over a fixed uniform sample of entries (measurement only)."""
    import torch
    xh = prob.reconstruct(cores, idx)
    xs = xstar_d[idx]
    num = torch.linalg.vector_norm((xh - xs).double())
    den = torch.linalg.vector_norm(xs.double())
    return float(num / den)


def equal_accuracy(prob, Z0_flat, xstar_d, sweeps, checkpoints, band=0.03, n_sample=1 << 20,
                   seed=0):
    """FP32 vs the BF16 forms, each fitted from the same start: recovery error after c
    sweeps for each checkpoint c (each run from scratch, so the timed c sweeps are exactly
    those of a c-sweep fit).  For a BF16 form f, its plateau e*_f is the median of its
    errors over the second half of the checkpoints: on its plateau the BF16 error wanders
    by about a percent from sweep to sweep (rounding of the direction) and may still drift
    by a few percent, so one checkpoint's error is a noisy estimate of the level.  The
    sweeps / time f and FP32 need to reach e*_f, i.e. an error within (1 + band) e*_f,
    give the speed-up at equal error.
    The recovery error is taken over a fixed uniform sample of n_sample entries (with
    2^20 entries its own relative sampling error is about 1e-3)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = xstar_d.numel()
    idx = torch.randint(0, n, (min(n_sample, n),), generator=g, dtype=torch.int64).cuda()
    res = {}
    for prec in ("native", "bf16", "bf16x3"):
        # one untimed sweep builds any layout this precision needs before the timed fits
        prob.fit([z.clone() for z in Z0_flat], max_sweeps=1, tol=0.0, precision=prec)
        rows = []
        for c in checkpoints:
            cores = [z.clone() for z in Z0_flat]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.fit(cores, max_sweeps=c, tol=0.0, precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows.append((c, dt, recovery_error(prob, cores, xstar_d, idx)))
        res[prec] = rows
    names = {"native": "fp32", "bf16": "bf16", "bf16x3": "bf16x3"}
    out = {"band": band, "sweeps_max": sweeps,
           "trace": {names[p]: [{"sweeps": c, "ms": round(dt * 1e3, 3), "rel_error": err}
                                for c, dt, err in rows] for p, rows in res.items()}}

    def first_hit(rows, target):
        return next((r for r in rows if r[2] <= target * (1 + band)), None)

    # common error levels: sweeps and time each precision needs to get there
    levels = {}
    for lv in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        row = {}
        for p, rows in res.items():
            h = next((r for r in rows if r[2] <= lv), None)
            row[names[p]] = None if h is None else {"sweeps": h[0], "ms": round(h[1] * 1e3, 3)}
        levels[f"{lv:.0e}"] = row
    out["levels"] = levels
    for form in ("bf16", "bf16x3"):
        e_star = statistics.median(r[2] for r in res[form][len(res[form]) // 2:])
        hf, h32 = first_hit(res[form], e_star), first_hit(res["native"], e_star)
        entry = {"target_rel_error": e_star,
                 "sweeps": hf[0] if hf else None, "ms": round(hf[1] * 1e3, 3) if hf else None,
                 "fp32_sweeps": h32[0] if h32 else None,
                 "fp32_ms": round(h32[1] * 1e3, 3) if h32 else None}
        if hf and h32:
            entry["speedup_vs_fp32"] = round(h32[1] / hf[1], 3)
        out[form] = entry
    return out


def equal_accuracy_seeds(wname, seeds, sweeps):
    """equal_accuracy over several seeds (inputs and start drawn from each seed): per BF16
    form the median and range of the speed-up at its own plateau, and per fixed error level
    the median speed-up over FP32."""
    import numpy as np
    import torch
    import synth
    import paper_2305_09044_amd as trd

    runs = []
    for s in seeds:
        w, dims, Xd, Pd, xs, _ = build_inputs(wname, s)
        prob = trd.Problem(Xd, Pd, dims, w.ranks)
        Z0 = synth.init_cores(dims, w.ranks, s)
        Z0_flat = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z0, np.float32)]
        r = equal_accuracy(prob, Z0_flat, xs, sweeps, list(range(1, sweeps + 1)), seed=s)
        r["seed"] = s
        runs.append(r)
        log(f"equal accuracy seed {s}:", json.dumps({k: v for k, v in r.items()
                                                     if k in ("bf16", "bf16x3")}))
        prob.close()
        del prob, Xd, Pd, xs, Z0_flat
        torch.cuda.empty_cache()
    summary = {"seeds": list(seeds)}
    for form in ("bf16", "bf16x3"):
        sp = [r[form].get("speedup_vs_fp32") for r in runs]
        sp = [v for v in sp if v is not None]
        summary[form] = {"speedup_median": statistics.median(sp) if sp else None,
                         "speedup_min": min(sp) if sp else None, "speedup_max": max(sp) if sp else None,
                         "target_rel_error_median": statistics.median(r[form]["target_rel_error"]
                                                                       for r in runs)}
    fixed = {}
    for lv in ("1e-02", "1e-03", "1e-04", "1e-05", "1e-06"):
        row = {}
        for form in ("bf16", "bf16x3"):
            ratios = []
            for r in runs:
                a, b = r["levels"][lv]["fp32"], r["levels"][lv][form]
                if a and b:
                    ratios.append(a["ms"] / b["ms"])
            row[form] = {"speedup_median": round(statistics.median(ratios), 3) if ratios else None,
                         "seeds_reached": len(ratios)}
        fixed[lv] = row
    summary["fixed_levels"] = fixed
    summary["per_seed"] = runs
    return summary


ABLATION_VARIANTS = (("method", "scaled", "global", "rsts"), ("gradient descent", "gradient", "global", "rsts"),
                     ("local scaled term", "scaled", "local", "rsts"),
                     ("uniform row sampling", "scaled", "global", "rows"),
                     ("leverage score sampling", "scaled", "global", "leverage"))


def ablation(prob, Z0_flat, xstar_d, dims, sizes, sweeps, seed=0, n_sample=1 << 20):
    """The ablations of Sec. 6.1 on the sketched path: the method, the plain gradient
    direction, the local scaled term (each with the same RStS sketches), uniform row
    sampling and leverage-score sampling (as many rows of the subchain unfolding, drawn
    i.i.d. uniformly or from the cores' leverage distributions), each fitted for
    `sweeps` sweeps from the same start, for several per-mode sample sizes s (J = s^(N-1)
    sampled rows per update); recovery error over a fixed uniform sample of entries, and
    the fit's time."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = xstar_d.numel()
    idx = torch.randint(0, n, (min(n_sample, n),), generator=g, dtype=torch.int64).cuda()
    rows = []
    for s in sizes:
        sk = [min(s, d) for d in dims]
        for name, direction, gram, sampling in ABLATION_VARIANTS:
            prob.set_variant(direction, gram, sampling)
            prob.fit([z.clone() for z in Z0_flat], max_sweeps=1, tol=0.0, sketch_sizes=sk, seed=seed)
            cores = [z.clone() for z in Z0_flat]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.fit(cores, max_sweeps=sweeps, tol=0.0, sketch_sizes=sk, seed=seed)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows.append({"variant": name, "s": s, "J": math.prod(sk[1:]), "ms": round(dt * 1e3, 3),
                         "rel_error": recovery_error(prob, cores, xstar_d, idx)})
            log(f"ablation {name} s={s}: {dt * 1e3:.1f} ms, rel. error {rows[-1]['rel_error']:.4g}")
    prob.set_variant("scaled", "global", "rsts")
    return {"sweeps": sweeps, "rows": rows}


def _host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    return model, cores


def _blas_threads(default):
    try:
        from threadpoolctl import threadpool_info
        n = [p["num_threads"] for p in threadpool_info() if p.get("user_api") == "blas"]
        return max(n) if n else default
    except Exception:
        return default


def cpu_baseline(wname: str, seed: int, sample_dims, backward: bool):
    """FP64 oracle on a bounded sample of the same recipe (same ranks, observed fraction and
    outlier law on smaller dims): one sweep with the quantile kernel width, or (the
    differentiation form) the loss and its all-core gradient at a perturbed point."""
    import numpy as np
    import synth
    from oracle import awrtrd as aw
    from oracle import tr

    from threadpoolctl import threadpool_limits

    model, cores = _host_cpu()
    w = synth.scaled(synth.WORKLOADS[wname], sample_dims)
    Zt, xstar, mask, X = synth.make_workload(w, seed, tr.reconstruct)
    X32 = X.astype(np.float32).astype(np.float64)
    nobs = int(mask.sum())
    N = len(sample_dims)
    with threadpool_limits(limits=cores, user_api="blas"):   # BLAS threads pinned to the cores
        threads = _blas_threads(cores)
        if backward:
            Z = synth.perturbed_cores(Zt, seed, rel=0.1)
            e = aw.residual_abs(X32, mask, Z)
            sigma = aw.quantile_sigma(e, 0.5, 5.0, 1e-6 * float(np.max(np.abs(X32[mask.astype(bool)]))))
            t0 = time.perf_counter()
            aw.loss(X32, mask, Z, sigma)
            aw.loss_grads(X32, mask, Z, sigma)
            what = "the loss and its gradient for every core"
        else:
            Z0 = synth.init_cores(sample_dims, w.ranks, seed)
            t0 = time.perf_counter()
            aw.fit(X32, mask, Z0, aw.FitOptions(max_sweeps=1, tol=0.0))
            what = "one sweep (quantile kernel width)"
        dt = time.perf_counter() - t0
    return {"value": N * nobs / dt, "unit": "observed entries/s", "cores": min(cores, threads),
            "kind": "oracle", "cpu_model": model,
            "sample": f"FP64 oracle, {what}, on the same recipe at {'x'.join(map(str, sample_dims))} "
                      f"(TR ranks {list(w.ranks)}, {nobs} observed entries, {dt:.2f} s, "
                      f"{min(cores, threads)} BLAS threads)"}


def mfma_object(prec: str, RR: int, K: int, split: bool, entries: float, total_entries: float,
                avg_ms: float):
    """Matrix-core work of one gradient-pass launch: the algorithmic products (2 RR flops for
    xhat and 2 RR for the gradient row factor per observed entry, RR = r_k r_s the contracted
    pair) and the products the dense 64 x 32 blocks issue (every position of a block, the
    contraction padded to K; three reconstruction products in the split form)."""
    if prec == "native":
        return None
    alg = entries * 4.0 * RR
    issued = total_entries * 2.0 * K * ((3 if split else 1) + 1)
    t = avg_ms / 1e3
    return {"unit": "TFLOP/s", "peak": BF16_PEAK_TFLOPS,
            "algorithmic": round(alg / t / 1e12, 2), "algorithmic_frac": round(alg / t / 1e12 / BF16_PEAK_TFLOPS, 4),
            "issued": round(issued / t / 1e12, 2), "issued_frac": round(issued / t / 1e12 / BF16_PEAK_TFLOPS, 4),
            "padding_factor": round(issued / alg, 2),
            "flop_per_entry": 4 * RR}


def sweep_bench(args, prob, w, dims, n_obs, Z0, xstar_d):
    """K timed sweeps (Alg. 1) of the bound problem."""
    import numpy as np
    import torch
    import synth

    npdt = np.float64 if w.dtype == "f64" else np.float32
    cores = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z0, npdt)]
    sk = list(w.sketch) if (args.sketch and w.sketch) else None
    prec = {"fp32": "native", "bf16": "bf16", "bf16x3": "bf16x3"}[args.precision]
    if sk is not None and prec != "native":  # RStS sketches run the native passes
        log("RStS path: native (fp32) passes")
        prec, args.precision = "native", "fp32"
    if args.warmup > 0:
        prob.fit(cores, max_sweeps=args.warmup, tol=0.0, sketch_sizes=sk, precision=prec)
    torch.cuda.synchronize()
    prob.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    rep = prob.fit(cores, max_sweeps=args.steps, tol=0.0, sketch_sizes=sk, seed=args.seed,
                   precision=prec)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = prob.profile_read()
    prob.profile(False)
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    elapsed = max(wall, gpu_s)
    assert rep["sweeps"] == args.steps, rep
    N = len(dims)
    # observed entries touched per sweep: all of them on the full path, the sketches' on RStS
    per_sweep = N * n_obs if sk is None else prof["entries"] / args.steps
    value = args.steps * per_sweep / elapsed
    log(f"timed {args.steps} sweeps: wall {wall * 1e3:.2f} ms, events {gpu_s * 1e3:.2f} ms, "
        f"sigma {rep['sigma'][-1]:.4g}, e {rep['e'][-1]:.3g}")
    return value, elapsed, prof, prec, sk


def backward_bench(args, prob, w, dims, n_obs, cores_t):
    """K timed steps of the differentiation form: the correntropy loss forward and its
    backward for every core through the torch.autograd.Function, at the true cores plus a
    N(0, 0.1/r) perturbation, with the kernel width of the quantile rule at that point."""
    import numpy as np
    import torch
    import synth
    import paper_2305_09044_amd as trd

    prec = {"fp32": "native", "bf16": "bf16", "bf16x3": "bf16x3"}[args.precision]
    Z = synth.perturbed_cores(cores_t, args.seed, rel=0.1)
    flat = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z, np.float32)]
    rep = prob.fit([c.clone() for c in flat], max_sweeps=1, tol=0.0, precision=prec)
    sigma = rep["sigma"][0]
    prob.set_precision(prec)
    cores = [c.clone().requires_grad_(True) for c in flat]

    def step():
        for c in cores:
            c.grad = None
        L = trd.correntropy_loss(prob, cores, sigma)
        L.backward()
        return L

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    prob.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        L = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = prob.profile_read()
    prob.profile(False)
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    elapsed = max(wall, gpu_s)
    N = len(dims)
    value = args.steps * N * n_obs / elapsed
    grads = [c.grad.detach().clone() for c in cores]
    # the same step in FP32 for the comparison (time and gradient difference)
    out = {"sigma": sigma, "loss": float(L.detach())}
    if prec != "native":
        prob.set_precision("native")
        for _ in range(max(args.warmup, 1)):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - t1) / args.steps
        g32 = [c.grad.detach() for c in cores]
        num = math.sqrt(sum(float(torch.sum((a.double() - b.double()) ** 2)) for a, b in zip(grads, g32)))
        den = math.sqrt(sum(float(torch.sum(b.double() ** 2)) for b in g32))
        out.update({"fp32_ms_per_step": round(t32 * 1e3, 4), "speedup_vs_fp32": round(t32 / (elapsed / args.steps), 3),
                    "grad_rel_diff_vs_fp32": num / den})
        prob.set_precision(prec)
    log(f"timed {args.steps} fwd+bwd steps: wall {wall * 1e3:.2f} ms, events {gpu_s * 1e3:.2f} ms, "
        f"sigma {sigma:.4g}; {json.dumps(out)}")
    return value, elapsed, prof, prec, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tr5_60_r8")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default=None,
                    help="dims of the oracle's bounded sample (default: the same recipe on smaller "
                         "dims, every mode kept)")
    ap.add_argument("--sketch", action="store_true", help="RStS path with the workload's sample sizes")
    ap.add_argument("--no-equal-accuracy", action="store_true",
                    help="skip the FP32-vs-BF16 time-to-equal-recovery-error comparison")
    ap.add_argument("--accuracy-sweeps", type=int, default=30)
    ap.add_argument("--accuracy-seeds", default="0,1,2,3,4",
                    help="seeds of the equal-accuracy comparison (inputs and start per seed)")
    ap.add_argument("--ablation", default=None,
                    help="comma-separated per-mode sample sizes: also run the Sec. 6.1 ablations "
                         "(method, gradient descent, local scaled term) on the RStS path")
    ap.add_argument("--ablation-sweeps", type=int, default=20)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "bf16x3"],
                    help="bf16: matrix-core passes with bf16 subchain tables (FP32 residuals); "
                         "bf16x3: the same with the reconstruction from split bf16 tables")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path runs on a single MI355X); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_09044_amd as trd

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst
    backward = args.workload in BACKWARD_WORKLOADS
    t_setup = time.perf_counter()
    w, dims, Xd, Pd, xstar_d, cores_t = build_inputs(args.workload, args.seed)
    t_inputs = time.perf_counter() - t_setup
    prob = trd.Problem(Xd, Pd, dims, w.ranks)
    info = prob.info()
    n_obs = info["n_obs"]
    import synth
    Z0 = synth.init_cores(dims, w.ranks, args.seed)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t_setup:.1f}s (inputs {t_inputs:.1f}s) n_obs={n_obs} "
        f"split={info['split']} workspace={info['workspace_bytes'] / 2**20:.0f} MiB")

    sk = None
    extra = {}
    if backward:
        value, elapsed, prof, prec, extra = backward_bench(args, prob, w, dims, n_obs, cores_t)
    else:
        value, elapsed, prof, prec, sk = sweep_bench(args, prob, w, dims, n_obs, Z0, xstar_d)

    # roofline of the fused gradient pass.  Algorithmic bytes per launch: every observed
    # entry is read once as a 4 B value and a 2 B position (in-tile column for the FP32
    # sliced-ELL pass, in-block position for the BF16 matrix-core pass); in a sweep the BF16
    # pass also writes the entry's weight (2 B, fp16) for the line search that follows, the
    # optional weight term of the per-entry accounting of the fused pass (a backward has no
    # line search and stores none).
    avg_ms = prof["total_ms"] / max(prof["launches"], 1)
    ent = prof["entries"] / max(prof["launches"], 1)
    bytes_per_entry = 4 + 2 + (2 if (prec != "native" and not backward) else 0)
    bytes_per_launch = ent * bytes_per_entry
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and sk is None:
        tf = json.load(open(TRAFFIC_FILE)).get(f"{args.workload}/{args.precision}", {})
        if tf.get("src_hash") == src_hash(args.precision):
            traffic = tf.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ("k_tpass<K,GradFast> (MFMA bf16 reconstruct+weight+gradient)" if prec != "native"
                       else "k_pass<float,RC,GradFast> (fused reconstruct+weight+gradient)"),
            "avg_launch_ms": round(avg_ms, 5), "launches": prof["launches"],
            "bytes_per_entry": bytes_per_entry, "bytes_per_launch": int(bytes_per_launch)}
    RR = w.ranks[0] * w.ranks[0]  # uniform ranks: r_k r_s of every contracted pair
    K = (RR + 31) // 32 * 32
    roof["mfma"] = mfma_object(prec, RR, K, prec == "bf16x3", ent, math.prod(dims), avg_ms)

    N = len(dims)
    cfg = {"workload": args.workload, "dims": list(dims), "tr_ranks": list(w.ranks),
           "observed_fraction": w.rho, "n_obs": n_obs, "precision": args.precision,
           "sketch_sizes": sk}
    if backward:
        cfg["path"] = ("differentiation form: correntropy loss forward + backward for all cores "
                       "(torch.autograd.Function), quantile kernel width at the evaluation point")
        metric = "observed entries/sec per all-core correntropy-loss forward+backward, BF16 vs FP32"
    else:
        cfg["path"] = (("SAWRTRD sweep (RStS sketches), FGMC, " if sk else "AWRTRD full sweep, FGMC, ")
                       + "quantile kernel width")
        metric = METRIC
    out = {"metric": metric, "value": value, "unit": "observed entries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if w.dtype == "f64" else ("f32" if prec == "native" else "bf16"),
           "data": "synthetic", "config": cfg, "roofline": roof}
    if backward:
        out["backward"] = extra
    if args.ablation:
        import numpy as np
        sizes = [int(v) for v in args.ablation.split(",")]
        npdt = np.float64 if w.dtype == "f64" else np.float32
        Z0_flat = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z0, npdt)]
        out["ablation"] = ablation(prob, Z0_flat, xstar_d, dims, sizes, args.ablation_sweeps,
                                   args.seed)
    prob.close()
    del prob, Xd, Pd, xstar_d
    torch.cuda.empty_cache()
    if not args.no_equal_accuracy and not backward and sk is None and w.dtype != "f64":
        seeds = [int(v) for v in args.accuracy_seeds.split(",")]
        out["equal_accuracy"] = equal_accuracy_seeds(args.workload, seeds, args.accuracy_sweeps)
        log("equal accuracy:", json.dumps({k: v for k, v in out["equal_accuracy"].items()
                                           if k not in ("per_seed",)}))
    if not args.no_cpu_baseline:
        sample = (tuple(int(v) for v in args.cpu_sample.split(",")) if args.cpu_sample
                  else CPU_SAMPLES.get(args.workload, tuple(min(d, 20) for d in dims)))
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed, sample, backward)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
