"""Benchmark: observed entries/s per AWRTRD core sweep on one MI355X.

A step is one sweep of Alg. 1 over all cores (sampling, subchain tables, fused
reconstruct+weight+gradient pass, FGMC Gram, scaled direction, line-search pass,
update, kernel-width quantile and convergence matrix), with inputs resident in HBM.
Default workload: 100^4 tensor of TR rank 5 (1e8 entries), 30% observed, N(0,1e-3)
noise, 20% of the observed entries replaced by +-max|X| salt and pepper, FP32.

Prints one JSON line.  The roofline object covers the dominant kernel (the fused
gradient pass), timed with HIP events around each of its launches in the timed
region; cpu_baseline is the FP64 numpy oracle on a bounded sample of the same recipe.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "observed entries/sec per AWRTRD core sweep, BF16 vs FP32, at equal rel. error"
HBM_PEAK_GBS = 8000.0
PASS_SRC = os.path.join(ROOT, "paper_2305_09044_amd", "csrc", "kernels_pass.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grad_pass_tr4_100_r5.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(precision: str = "fp32") -> str:
    src = PASS_SRC if precision == "fp32" else PASS_SRC.replace("kernels_pass", "kernels_tile")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def build_inputs(wname: str, seed: int, dims=None):
    """Seeded workload on the device: clean tensor from the library's own reconstruction,
    noise, outliers and mask from synth."""
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
    torch.cuda.synchronize()
    xstar = xs.cpu().numpy().astype(np.float64).reshape(dims, order="F")
    shape.close()
    del ct
    if w.normalise_max:
        mx = float(np.max(np.abs(xstar)))
        xstar /= mx
        xs /= mx
    mask = (synth.bernoulli_mask(dims, w.rho, seed) if w.mask_kind == "bernoulli"
            else synth.block_mask(dims, 16, 1.0 - w.rho, seed))
    X = synth.assemble(w, xstar, mask, seed)
    del xstar
    Xd = torch.from_numpy(X.astype(npdt).ravel(order="F")).cuda()
    Pd = torch.from_numpy(mask.ravel(order="F").copy()).cuda()
    del X
    return w, dims, Xd, Pd, mask, xs


def recovery_error(prob, cores, xstar_d) -> float:
    """||Xhat - X*||_F / ||X*||_F over every entry (measurement only)."""
    import torch
    xh = prob.reconstruct(cores)
    num = torch.linalg.vector_norm((xh - xstar_d).double())
    den = torch.linalg.vector_norm(xstar_d.double())
    return float(num / den)


def equal_accuracy(prob, Z0_flat, xstar_d, sweeps, checkpoints, band=0.03):
    """FP32 vs BF16 sweeps from the same start: recovery error after c sweeps for each
    checkpoint c (each run from scratch, so the timed c sweeps are exactly those of a
    c-sweep fit), the BF16 plateau e* = its error after the last checkpoint, and the
    sweeps / time each precision needs to reach e*.  On its plateau the BF16 error
    wanders by about a percent from sweep to sweep (rounding of the direction), so
    reaching e* means an error within (1 + band) e*."""
    import torch
    res = {}
    for prec in ("native", "bf16"):
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
            rows.append((c, dt, recovery_error(prob, cores, xstar_d)))
        res[prec] = rows
    e_star = res["bf16"][-1][2]
    out = {"target_rel_error": e_star, "band": band, "sweeps_max": sweeps}
    for prec, name in (("native", "fp32"), ("bf16", "bf16")):
        hit = next((r for r in res[prec] if r[2] <= e_star * (1 + band)), None)
        out[name] = {"trace": [{"sweeps": c, "ms": round(dt * 1e3, 3), "rel_error": err}
                               for c, dt, err in res[prec]],
                     "sweeps_to_target": hit[0] if hit else None,
                     "ms_to_target": round(hit[1] * 1e3, 3) if hit else None}
    if out["fp32"]["ms_to_target"] and out["bf16"]["ms_to_target"]:
        out["bf16_speedup_at_equal_error"] = round(out["fp32"]["ms_to_target"] /
                                                   out["bf16"]["ms_to_target"], 3)
    return out


def cpu_baseline(wname: str, seed: int, sample_dims):
    """FP64 oracle, one sweep (quantile kernel width), on a bounded sample of the recipe."""
    import numpy as np
    import synth
    from oracle import awrtrd as aw
    from oracle import tr

    w = synth.scaled(synth.WORKLOADS[wname], sample_dims)
    Zt, xstar, mask, X = synth.make_workload(w, seed, tr.reconstruct)
    Z0 = synth.init_cores(sample_dims, w.ranks, seed)
    X32 = X.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    aw.fit(X32, mask, Z0, aw.FitOptions(max_sweeps=1, tol=0.0))
    dt = time.perf_counter() - t0
    nobs = int(mask.sum())
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": len(sample_dims) * nobs / dt, "unit": "observed entries/s", "cores": min(cores, threads),
            "kind": "oracle",
            "sample": f"one FP64 sweep of the same recipe on a {'x'.join(map(str, sample_dims))} tensor "
                      f"({nobs} observed entries, {dt:.2f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tr4_100_r5")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default=None,
                    help="dims of the oracle's bounded sample (default: the workload with its last "
                         "mode cut so the sample has at most 2e7 entries)")
    ap.add_argument("--sketch", action="store_true", help="RStS path with the workload's sample sizes")
    ap.add_argument("--no-equal-accuracy", action="store_true",
                    help="skip the FP32-vs-BF16 time-to-equal-recovery-error comparison")
    ap.add_argument("--accuracy-sweeps", type=int, default=30)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="bf16: matrix-core passes with bf16 subchain tables (FP32 residuals)")
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
    t_setup = time.perf_counter()
    w, dims, Xd, Pd, mask_np, xstar_d = build_inputs(args.workload, args.seed)
    prob = trd.Problem(Xd, Pd, dims, w.ranks)
    info = prob.info()
    n_obs = info["n_obs"]
    import numpy as np
    import synth
    Z0 = synth.init_cores(dims, w.ranks, args.seed)
    npdt = np.float64 if w.dtype == "f64" else np.float32
    cores = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z0, npdt)]
    sk = list(w.sketch) if (args.sketch and w.sketch) else None
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t_setup:.1f}s n_obs={n_obs} split={info['split']} "
        f"workspace={info['workspace_bytes'] / 2**20:.0f} MiB")

    prec = "bf16" if args.precision == "bf16" else "native"
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

    # roofline of the fused gradient pass.  Algorithmic bytes per launch: FP32 sliced-ELL
    # passes read a 4 B value and a 2 B in-tile column per observed entry; the BF16
    # matrix-core passes read the 4 B value plus one mask bit per tensor position.
    avg_ms = prof["total_ms"] / max(prof["launches"], 1)
    ent = prof["entries"] / max(prof["launches"], 1)
    if prec == "bf16" and sk is None:
        bytes_per_launch = ent * 4 + math.prod(dims) / 8
    else:
        bytes_per_launch = ent * (4 + 2)
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE)).get(args.precision, {})
        if tf.get("src_hash") == src_hash(args.precision) and tf.get("workload") == args.workload \
                and sk is None:
            traffic = tf.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": ("k_tpass<K,GradFast> (MFMA bf16 reconstruct+weight+gradient)" if prec == "bf16"
                       else "k_pass<float,RC,GradFast> (fused reconstruct+weight+gradient)"),
            "avg_launch_ms": round(avg_ms, 5), "launches": prof["launches"],
            "bytes_per_launch": int(bytes_per_launch)}

    out = {"metric": METRIC, "value": value, "unit": "observed entries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if w.dtype == "f64" else ("bf16" if prec == "bf16" else "f32"),
           "data": "synthetic",
           "config": {"workload": args.workload, "dims": list(dims), "tr_ranks": list(w.ranks),
                      "observed_fraction": w.rho, "n_obs": n_obs, "path": "AWRTRD full sweep, FGMC, "
                      "quantile kernel width", "precision": args.precision},
           "roofline": roof}
    if not args.no_equal_accuracy and sk is None and w.dtype != "f64":
        C = args.accuracy_sweeps
        cps = sorted(set([1, 2, 3, 4, 6, 8, 10, 12, 15, 20, 25, C]) & set(range(1, C + 1)))
        Z0_flat = [torch.from_numpy(f).cuda() for f in synth.cores_to_flat(Z0, np.float32)]
        out["equal_accuracy"] = equal_accuracy(prob, Z0_flat, xstar_d, C, cps)
        log("equal accuracy:", json.dumps({k: v for k, v in out["equal_accuracy"].items()
                                           if k not in ("fp32", "bf16")}))
    if not args.no_cpu_baseline:
        if args.cpu_sample:
            sample = tuple(int(v) for v in args.cpu_sample.split(","))
        else:
            rest = math.prod(dims[:-1])
            sample = tuple(dims[:-1]) + (max(1, min(dims[-1], int(2e7 // rest))),)
        del prob, Xd, Pd, xstar_d
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed, sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
