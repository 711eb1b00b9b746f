"""Benchmark: plain batched partial evaluation of a whole population on one GPU.

Workload (clinical-shaped): 512x512x100 float32 CT-like volumes, 10x10x6-point
dual meshes (2430 tetrahedra each), population 512, all 600 single-point FOS
elements partial-evaluated in one launch per step (307,200 partial
evaluations, each re-evaluating every objective over the star of its point in
both grids).  Old terms come from the per-tetrahedron cache written by one
full evaluation before timing.  Inputs are synthetic and resident in HBM.

Prints one JSON line (rank 0).  ``--gpus`` above 1 is refused: this build
evaluates on a single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_SAMPLE = 8   # one streamed own voxel + one (amortised) gathered voxel, float32
KERNEL_SRC = os.path.join(ROOT, "paper_2202_11001_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_partial_clinical_traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, X, off, pts, cand, budget_s=20.0):
    """The FP64 oracle on a bounded sample: all FOS elements of the first
    solutions, until about budget_s of CPU time; partial evaluations/s."""
    from oracle import ref
    rp = ref.Problem(w.moving, w.fixed, w.mesh, w.spacing, w.tau, guid_moving=w.guid_moving,
                     corr_moving=w.corr_moving, guid_fixed=w.guid_fixed, corr_fixed=w.corr_fixed)
    F = len(off) - 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # probe: 64 elements of solution 0 (current terms recomputed by the oracle too: it has no cache,
    # so time the candidate side only by passing zero cached terms)
    zeros = np.zeros((1, rp.T, 3))
    nprobe = min(F, 64)
    t0 = time.perf_counter()
    rp.eval_partial(X[:1], off[:nprobe + 1], pts[:off[nprobe]], cand[:1, :off[nprobe]], tet_terms=zeros)
    dt = time.perf_counter() - t0
    per = dt / nprobe
    n = int(max(nprobe, min(F * len(X), budget_s / max(per, 1e-9))))
    ns = max(1, min(len(X), n // F))
    t0 = time.perf_counter()
    rp.eval_partial(X[:ns], off, pts, cand[:ns], tet_terms=np.zeros((ns, rp.T, 3)))
    dt = time.perf_counter() - t0
    return {"value": ns * F / dt, "unit": "partial_evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{ns} solution(s) x {F} single-point FOS elements of the same workload, FP64, "
                      f"{dt:.1f} s wall"}


def kernel_source_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings to bytes."""
    import torch
    n = 256 * 1024 * 1024  # float32 elements = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--small", action="store_true", help="64^3 workload (quick check)")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3: 2 steps, no warmup, no CPU leg")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the copy kernel of known size")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile:
        args.steps, args.warmup, args.no_cpu = 2, 0, True
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} not supported: this evaluator runs on one GPU "
              f"(solutions shard across GPUs without exchange, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = W.batched() if args.small else W.clinical()
    log(f"workload {w.name} generated in {time.perf_counter() - t0:.1f} s")
    gp = dsm.Problem.from_workload(w)
    S = w.S

    def reject(X):
        return gp.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0

    X = w.population(reject=reject)
    off, pts = w.fos()
    F = len(off) - 1
    cand = w.candidates(X, off, pts)
    Xd = torch.from_numpy(X).to(dev)
    offd, ptsd, candd = (torch.from_numpy(a).to(dev) for a in (off, pts, cand))
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=dev)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    out = (torch.empty((S, F, 3), dtype=torch.float64, device=dev), torch.empty((S, F, 3), dtype=torch.float64, device=dev),
           torch.empty((S, F), dtype=torch.int32, device=dev), torch.empty((S, F), dtype=torch.int32, device=dev))
    gp.eval_partial(Xd, offd, ptsd, candd, tet_terms_in=cache, out=out)
    torch.cuda.synchronize()
    samples = int(out[3].to(torch.int64).sum().item())
    nflag = int((out[2] != 0).sum().item())
    log(f"S={S} F={F} T={gp.T} samples/step={samples} (8VS={8 * gp.V * S}) flagged={nflag}")

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        gp.eval_partial(Xd, offd, ptsd, candd, tet_terms_in=cache, out=out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    gp.timing(args.steps)
    t_start = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        gp.eval_partial(Xd, offd, ptsd, candd, tet_terms_in=cache, out=out)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    sweep_ms = gp.timing_read()
    gp.timing(0)
    ms = float(np.mean(step_ms))
    kms = float(np.mean(sweep_ms))
    log(f"step ms: {['%.2f' % x for x in step_ms]}; sweep kernel ms: {['%.2f' % x for x in sweep_ms]}; "
        f"wall {wall:.3f} s")

    evals_per_s = S * F / (ms / 1e3)
    samples_per_s = samples / (ms / 1e3)
    achieved = samples * BYTES_PER_SAMPLE / (kms / 1e3) / 1e9
    traffic = measured_traffic()
    res = {
        "metric": "partial solution evals/s @512^2x100 (plain, batched)",
        "value": evals_per_s,
        "unit": "partial_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name + f", meshes {w.mesh}, population {S}, {F} single-point FOS elements per step",
                   "partial_evals_per_step": S * F, "voxel_samples_per_step": samples},
        "voxel_samples_per_s": samples_per_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep<1> (partial-evaluation voxel sweep)", "kernel_ms": kms,
                     "algorithmic_bytes_per_launch": samples * BYTES_PER_SAMPLE,
                     "kernel_source_sha256_16": kernel_source_hash()},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)...")
        res["cpu_baseline"] = cpu_baseline(w, X, off, pts, cand)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
