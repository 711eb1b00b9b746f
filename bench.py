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


def cpu_model():
    """The host CPU's model name."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, X, off, pts, cand, budget_s=20.0, budget_1core_s=8.0):
    """The FP64 oracle on a bounded sample: all FOS elements of the first
    solutions, until about budget_s of CPU time, on every host thread it
    uses; then a smaller sample of solution 0 on one thread.  Partial
    evaluations/s (the oracle has no term cache here: zero cached terms make
    it time the candidate side only)."""
    from oracle import ref
    rp = ref.Problem(w.moving, w.fixed, w.mesh, w.spacing, w.tau, guid_moving=w.guid_moving,
                     corr_moving=w.corr_moving, guid_fixed=w.guid_fixed, corr_fixed=w.corr_fixed)
    F = len(off) - 1
    threads = ref.lib().ref_max_threads()
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
    res = {"value": ns * F / dt, "unit": "partial_evals/s", "cores": threads, "kind": "oracle",
           "sample": f"{ns} solution(s) x {F} single-point FOS elements of the same workload, FP64, "
                     f"{dt:.1f} s wall", "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    prev = ref.set_threads(1)
    try:
        n1 = int(max(1, min(F, budget_1core_s / max(per * threads, 1e-9))))
        t0 = time.perf_counter()
        rp.eval_partial(X[:1], off[:n1 + 1], pts[:off[n1]], cand[:1, :off[n1]], tet_terms=zeros)
        dt1 = time.perf_counter() - t0
    finally:
        ref.set_threads(prev)
    res["one_core"] = {"value": n1 / dt1, "unit": "partial_evals/s", "cores": 1,
                       "sample": f"{n1} single-point FOS elements of solution 0, FP64, {dt1:.1f} s wall"}
    return res


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


def screened_step(gp, Xd, offd, ptsd, candd, cache, out, w, S, F, K=4, train_steps=500):
    """Times one surrogate-screened pass over all (solution, element) pairs: K
    candidates each, features + MLP forward + selection, then exact partial
    evaluation of the picks flagged for it.  The surrogate is first trained on
    the exact deltas of the plain step's candidates."""
    import torch
    from paper_2202_11001_amd import dsm
    old, new, flags, _ = out
    feats = dsm.Surrogate.features(gp, Xd, ptsd, candd.reshape(S, F, 1, 2, 3))
    ok = (flags == 0).reshape(-1)
    f_ok, o_ok, n_ok = feats[ok], old.reshape(-1, 3)[ok].contiguous(), new.reshape(-1, 3)[ok].contiguous()
    sur = dsm.Surrogate(seed=11, max_rows=S * F * K, max_batch=4096)
    sur.fit_scaling(f_ok, sur.pack(part_old=o_ok, part_new=n_ok)[2])  # raw deltas new - old
    fb, tg, _ = sur.pack(f_ok, o_ok, n_ok)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = sur.train(fb, tg, steps=train_steps, batch=4096)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del feats, f_ok, fb, tg
    candK = gp.sample_candidates(Xd, ptsd, K, w.sigma_cand, 77, 1)
    gp.eval_full(Xd, tet_terms=cache)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    stream = torch.cuda.current_stream()
    for rep in range(2):  # the second repetition is timed
        ev[0].record(stream)
        pick, run, pred, cpick = sur.screen(gp, Xd, ptsd, candK)
        ev[1].record(stream)
        gp.eval_partial(Xd, offd, ptsd, cpick, tet_terms_in=cache, out=out, mask=run)
        ev[2].record(stream)
        torch.cuda.synchronize()
    t_screen = ev[0].elapsed_time(ev[1])
    t_exact = ev[1].elapsed_time(ev[2])
    n_exact = int(run.sum().item())
    lo = losses.cpu().numpy()
    log(f"screened step: screen {t_screen:.2f} ms (K={K}), exact {t_exact:.2f} ms for {n_exact}/{S * F} picks; "
        f"training {train_steps} steps {t_train:.2f} s, loss {lo[:5].mean():.3f} -> {lo[-20:].mean():.3f}")
    return {"K": K, "ms_per_step": t_screen + t_exact, "screen_ms": t_screen, "exact_ms": t_exact,
            "exact_evals": n_exact, "pairs": S * F, "candidates_screened_per_s": S * F * K / ((t_screen + t_exact) / 1e3),
            "train_steps": train_steps, "train_s": t_train, "train_loss_first": float(lo[:5].mean()),
            "train_loss_last": float(lo[-20:].mean())}


def generation_timing(gp, Xd, n=3):
    """Milliseconds per plain optimiser generation (8 class steps: sample,
    evaluate, accept) run eagerly and replayed from a captured HIP graph."""
    import torch
    from paper_2202_11001_amd import optimizer as O
    res = {}
    for mode in ("eager", "graph"):
        opt = O.Optimiser(gp, Xd, sigma=1.0, seed=11, graph=mode == "graph")
        opt.generation()  # capture / warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            opt.generation()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        res[mode + "_ms"] = float(np.median(ts))
    return res


def surrogate_report(gp, opt, sur, K=4, seed=4242):
    """Held-out quality of the trained surrogate on the final screened
    population: K fresh candidates for every (solution, point) of one parity
    class, all evaluated exactly.  Reports RMSE, R^2 and sign agreement of the
    predicted deltas per objective, and the ablation trained pick vs random
    pick vs an untrained network's pick (mean standardised exact delta of the
    pick, fraction of picks accepted by the exact acceptance rule)."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import optimizer as O
    pts = opt.classes[0]
    F, S = pts.shape[0], opt.S
    off = torch.arange(F + 1, dtype=torch.int32, device=pts.device)
    candK = gp.sample_candidates(opt.X, pts, K, opt.sigma, seed, 1)
    true = torch.empty((S, F, K, 3), dtype=torch.float64, device=pts.device)
    ok = torch.ones((S, F), dtype=torch.bool, device=pts.device)
    for k in range(K):
        o, n, fl, _ = gp.eval_partial(opt.X, off, pts, candK[:, :, k].contiguous(), tet_terms_in=opt.cache)
        true[:, :, k] = n - o
        ok &= fl == 0
    pick, _, pred, _ = sur.screen(gp, opt.X, pts, candK)
    fresh = dsm.Surrogate(seed=99, max_rows=S * F * K, max_batch=1024)
    im, irs, om, ors = sur.scaling()
    fresh.set_scaling(im, irs, om, ors)
    pick0 = fresh.screen(gp, opt.X, pts, candK)[0]
    t = true[ok].reshape(-1, 3).cpu().numpy()
    p = pred[ok].reshape(-1, 3).to(torch.float64).cpu().numpy()
    res = {"candidates": int(t.shape[0]), "rmse": [], "r2": [], "sign_agreement_nonzero": [], "nonzero_fraction": []}
    for c in range(3):
        err = p[:, c] - t[:, c]
        var = float(np.var(t[:, c]))
        nz = t[:, c] != 0  # e.g. no guidance point in the star: the exact delta is 0
        res["rmse"].append(float(np.sqrt(np.mean(err ** 2))))
        res["r2"].append(float(1 - np.mean(err ** 2) / var) if var > 0 else None)
        res["sign_agreement_nonzero"].append(float(np.mean(np.sign(p[nz, c]) == np.sign(t[nz, c]))) if nz.any() else None)
        res["nonzero_fraction"].append(float(nz.mean()))
    tn = true.cpu().numpy()
    okn = ok.cpu().numpy()
    score = ((tn - om) * ors).sum(axis=-1)
    arch = np.asarray(opt.archive)
    objn = opt.obj.cpu().numpy()

    def accepted(d, s_idx):
        if np.all(d <= 0) and np.any(d < 0):
            return True
        if not np.any(d < 0):
            return False
        nv = objn[s_idx] + d
        return not np.any(np.all(arch <= nv, axis=1) & np.any(arch < nv, axis=1))

    rng = np.random.default_rng(seed)
    picks = {"trained": pick.cpu().numpy(), "untrained": pick0.cpu().numpy(),
             "random": rng.integers(0, K, size=(S, F))}
    ss = np.nonzero(okn)
    for name, pk in picks.items():
        sel = pk[ss]
        res[f"{name}_mean_std_delta"] = float(score[ss[0], ss[1], sel].mean())
        res[f"{name}_accept_rate"] = float(np.mean([accepted(tn[a, b, k], a) for a, b, k in zip(ss[0], ss[1], sel)]))
    return res


def surrogate_oracle_report(w, gp, opt, sur, n_sol=16, n_pts=64, K=4, seed=4343):
    """Held-out quality judged against the FP64 oracle: K fresh candidates for
    n_pts points of one parity class in n_sol solutions of the final screened
    population (n_sol * n_pts * K candidates); their exact deltas come from the
    oracle (which recomputes the current terms itself), the predictions from
    the surrogate.  Also reports how far the GPU's exact deltas are from the
    oracle's on the same candidates."""
    import torch
    from oracle import ref
    rp = ref.Problem(w.moving, w.fixed, w.mesh, w.spacing, w.tau, guid_moving=w.guid_moving,
                     corr_moving=w.corr_moving, guid_fixed=w.guid_fixed, corr_fixed=w.corr_fixed)
    rng = np.random.default_rng(seed)
    dev = opt.X.device
    pts_all = opt.classes[0].cpu().numpy()
    pts = np.sort(rng.choice(pts_all, size=min(n_pts, len(pts_all)), replace=False)).astype(np.int32)
    sols = np.sort(rng.choice(opt.S, size=n_sol, replace=False))
    Xd = opt.X[torch.from_numpy(sols).to(dev)].contiguous()
    ptsd = torch.from_numpy(pts).to(dev)
    F = len(pts)
    off = np.arange(F + 1, dtype=np.int32)
    offd = torch.from_numpy(off).to(dev)
    candK = gp.sample_candidates(Xd, ptsd, K, opt.sigma, seed, 1)          # [n_sol][F][K][2][3]
    _, _, pred, _ = sur.screen(gp, Xd, ptsd, candK)
    gpu = np.zeros((n_sol, F, K, 3))
    for k in range(K):
        o, n, fl, _ = gp.eval_partial(Xd, offd, ptsd, candK[:, :, k].contiguous())
        gpu[:, :, k] = (n - o).cpu().numpy()
    Xh, ch, predh = Xd.cpu().numpy(), candK.cpu().numpy(), pred.cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    true = np.zeros((n_sol, F, K, 3))
    ok = np.ones((n_sol, F), dtype=bool)
    for k in range(K):
        rold, rnew, rfl, _ = rp.eval_partial(Xh, off, pts, np.ascontiguousarray(ch[:, :, k]))
        true[:, :, k] = rnew - rold
        ok &= rfl == 0
    t_oracle = time.perf_counter() - t0
    t = true[ok].reshape(-1, 3)
    p = predh[ok].reshape(-1, 3)
    g = gpu[ok].reshape(-1, 3)
    res = {"candidates": int(t.shape[0]), "oracle_seconds": t_oracle, "rmse": [], "r2": [],
           "sign_agreement_nonzero": [], "nonzero_fraction": [],
           "gpu_vs_oracle_max_abs": [float(np.abs(g[:, c] - t[:, c]).max()) for c in range(3)]}
    for c in range(3):
        err = p[:, c] - t[:, c]
        var = float(np.var(t[:, c]))
        nz = t[:, c] != 0
        res["rmse"].append(float(np.sqrt(np.mean(err ** 2))))
        res["r2"].append(float(1 - np.mean(err ** 2) / var) if var > 0 else None)
        res["sign_agreement_nonzero"].append(float(np.mean(np.sign(p[nz, c]) == np.sign(t[nz, c]))) if nz.any() else None)
        res["nonzero_fraction"].append(float(nz.mean()))
    return res


def surrogate_run(gp, X, G, train_generations, name, w, seeds=(5, 6, 7)):
    """For each seed: a plain run of G generations vs a run whose first
    train_generations generations are plain (collecting exact deltas),
    followed by surrogate training and screened generations until 99 % of the
    plain run's final hypervolume; hypervolume of the elitist archive against a
    reference point fixed by the initial population.  Generations replay a
    captured HIP graph (the collecting ones run eagerly); the clock counts
    optimisation and training, not the hypervolume monitoring.  Reports every
    seed and the medians; the first seed's surrogate is scored on held-out
    candidates against the GPU's exact deltas and against the FP64 oracle."""
    import torch
    from paper_2202_11001_amd import optimizer as O
    Xd = torch.from_numpy(X).to("cuda:0")
    runs = []
    first = None
    for seed in seeds:
        log(f"seed {seed}: plain run, {G} generations")
        lp, op, _ = O.run(gp, Xd, G, sigma=1.0, seed=seed, log_every=10, graph=True)
        target = 0.99 * lp.hypervolume[-1]
        plain_reach = next(i for i, h in enumerate(lp.hypervolume) if h >= target)
        log(f"seed {seed}: screened run, {train_generations} plain generations, then screened, "
            f"until hv >= {target:.6g} or {G}")
        ls, os_, sur = O.run(gp, Xd, G, sigma=1.0, seed=seed, train_generations=train_generations, target_hv=target,
                             log_every=10, graph=True)
        reach = next((i for i, h in enumerate(ls.hypervolume) if h >= target), None)
        r = {"seed": seed, "target_hv": target,
             "plain": {"final_hv": lp.hypervolume[-1], "seconds": lp.seconds[-1],
                       "generations_to_target": plain_reach + 1, "seconds_to_target": lp.seconds[plain_reach],
                       "exact_to_target": int(sum(lp.exact_evals[:plain_reach + 1]))},
             "screened": {"final_hv": ls.hypervolume[-1], "seconds": ls.seconds[-1],
                          "generations_to_target": None if reach is None else reach + 1,
                          "seconds_to_target": None if reach is None else ls.seconds[reach],
                          "exact_to_target": None if reach is None else int(sum(ls.exact_evals[:reach + 1])),
                          "hv": ls.hypervolume, "t": ls.seconds, "exact": ls.exact_evals, "accepted": ls.accepted}}
        if reach is not None:
            r["speedup_to_target"] = lp.seconds[-1] / ls.seconds[reach]
            r["speedup_vs_plain_reaching_target"] = lp.seconds[plain_reach] / ls.seconds[reach]
        log(f"seed {seed}: plain {lp.seconds[-1]:.1f} s (target at {lp.seconds[plain_reach]:.1f} s), "
            f"screened {r['screened']['seconds_to_target']} s")
        runs.append(r)
        if first is None:
            first = (os_, sur)
    os_, sur = first
    quality = surrogate_report(gp, os_, sur)
    log(f"surrogate held-out quality (GPU exact deltas): {quality}")
    oracle_quality = surrogate_oracle_report(w, gp, os_, sur)
    log(f"surrogate held-out quality (FP64 oracle deltas): {oracle_quality}")
    med = lambda xs: float(np.median([x for x in xs if x is not None])) if any(x is not None for x in xs) else None
    res = {"workload": name, "generations": G, "train_generations": train_generations, "seeds": list(seeds),
           "median": {"plain_seconds": med([r["plain"]["seconds"] for r in runs]),
                      "plain_seconds_to_target": med([r["plain"]["seconds_to_target"] for r in runs]),
                      "screened_seconds_to_target": med([r["screened"]["seconds_to_target"] for r in runs]),
                      "speedup_to_target": med([r.get("speedup_to_target") for r in runs]),
                      "speedup_vs_plain_reaching_target": med([r.get("speedup_vs_plain_reaching_target")
                                                               for r in runs])},
           "runs": runs, "surrogate_quality": quality, "surrogate_quality_oracle": oracle_quality}
    print(json.dumps(res), flush=True)


def sampler_run(gp, X, G, name, w):
    """G generations with isotropic Gaussian candidates around the current
    position vs G generations whose candidates are drawn from per-point normal
    distributions estimated on the selected solutions (RV-GOMEA's partial
    changes; tau = 0.35, adaptive multipliers), for single-point elements and
    for the paper's FOS (one random tetrahedron per cube, its 4 points drawn
    jointly), each estimated sampler also with 5 clusters of the selection in
    objective space, and with 5 clusters plus the anticipated mean shift,
    forced improvements and the standard-deviation-ratio multiplier schedule;
    all eager from the same population; hypervolume of the elitist archive
    against a reference point fixed by the initial population."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import optimizer as O
    Xd = torch.from_numpy(X).to("cuda:0")
    gp4 = dsm.Problem.from_workload(w, max_fos_points=4)
    out = {"workload": name, "generations": G}
    for fos, prob in (("point", gp), ("tetrahedron", gp4)):
        for sampler, k, full in (("isotropic", 1, False), ("estimated", 1, False), ("estimated", 5, False),
                                 ("estimated", 5, True)):
            key = f"{fos}/{sampler}" + (f"/{k} clusters" if k > 1 else "") + ("/AMS+FI+SDR" if full else "")
            log(f"{key}: {G} generations")
            lg, opt, _ = O.run(prob, Xd, G, sigma=1.0, seed=5, log_every=10, sampler=sampler, fos=fos, clusters=k,
                               ams=full, forced_improvements=full, multiplier_schedule="sdr" if full else "simple")
            arch = np.asarray(opt.archive)
            pop = opt.obj.cpu().numpy()
            out[key] = {"final_hv": lg.hypervolume[-1], "seconds": lg.seconds[-1], "hv": lg.hypervolume,
                        "t": lg.seconds, "accepted": lg.accepted, "exact": lg.exact_evals,
                        "archive": lg.archive_size[-1],
                        "archive_inside_reference": float(np.mean(np.all(arch < opt.ref, axis=1))),
                        "population_objectives_over_reference_median": (np.median(pop, axis=0) / opt.ref).tolist()}
            if sampler == "estimated":
                m = torch.cat(opt.mult) if fos == "point" else opt.mult_cube
                out[key]["multiplier"] = {"min": float(m.min()), "median": float(m.median()), "max": float(m.max())}
    print(json.dumps(out), flush=True)


def phantom_run(G1=300, G2=600, S1=250, S2=500, clusters=1, ams=False, forced=False, single_objective=False,
                schedule="simple"):
    """Sec. 3's synthetic experiment on the seeded replica phantom (a cube with
    parabolic intrusions on every face and a shrinking central sphere, guidance
    on the sphere): the paper's multi-resolution scheme (6^3 grids, population
    250, 300 generations, then 11^3 grids seeded from the approximation set,
    population 500, 600 generations), with its FOS (one random tetrahedron per
    cube) and estimated distributions (optionally per cluster of the selection
    in objective space).  As in Fig. 2 the archived solution with
    the lowest guidance error is selected; its transformation (dsm_transform)
    gives the transformed source and the DVF, summarised against the phantom's
    known surfaces."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import optimizer as O
    from paper_2202_11001_amd import workloads as W
    dev = torch.device("cuda:0")
    wc = W.phantom(mesh=(6, 6, 6), S=S1)
    wf = W.phantom(mesh=(11, 11, 11), S=S2)
    gpc = dsm.Problem.from_workload(wc, max_fos_points=4)
    gpf = dsm.Problem.from_workload(wf, max_fos_points=4)
    X = wc.population(reject=lambda X: gpc.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0)
    res = {"workload": wf.name, "clusters": clusters, "ams": ams, "forced_improvements": forced,
           "single_objective_clusters": single_objective, "multiplier_schedule": schedule,
           "phantom": {"half": 15.0, "depth": 6.0, "r_source": 9.0, "r_target": 5.0,
                       "guidance_pairs": int(len(wf.guid_moving))}}

    def level(name, opt, G):
        t0 = time.perf_counter()
        t_opt, hv = 0.0, [(0, opt.hypervolume())]
        for g in range(G):
            t1 = time.perf_counter()
            opt.generation()
            torch.cuda.synchronize()
            t_opt += time.perf_counter() - t1
            if (g + 1) % 50 == 0 or g + 1 == G:
                hv.append((g + 1, opt.hypervolume()))
                log(f"{name} gen {g + 1}: hv {hv[-1][1]:.6g} archive {opt.n_arch} t {t_opt:.1f} s")
            elif (g + 1) % 25 == 0:
                log(f"{name} gen {g + 1}: archive {opt.n_arch} t {t_opt:.1f} s")
        return {"mesh": list(opt.p.mesh), "S": opt.S, "generations": G, "seconds": t_opt,
                "seconds_with_monitoring": time.perf_counter() - t0, "hv": hv, "archive": len(opt.archive)}

    opts = dict(keep_solutions=True, sampler="estimated", fos="tetrahedron", clusters=clusters,
                archive_capacity=1 << 16, ams=ams, forced_improvements=forced,
                single_objective_clusters=single_objective, multiplier_schedule=schedule)
    oc = O.Optimiser(gpc, torch.from_numpy(X).to(dev), seed=41, **opts)
    res["coarse"] = level("coarse", oc, G1)
    Xf, rejected = O.seed_finer(oc, gpf, S2, seed=42)
    res["seed"] = {"S": S2, "rejected_draws": rejected, "coarse_archive": len(oc.archive)}
    of = O.Optimiser(gpf, Xf, seed=43, **opts)
    res["fine"] = level("fine", of, G2)
    arch = np.asarray(of.archive)
    best = int(np.argmin(arch[:, 2]))
    Xb = of.arch_X_dev[best].contiguous()
    I = gpf.topology()["identity"]
    obj_id, _ = gpf.eval_full(torch.from_numpy(np.stack([I, I])[None]).to(dev))
    obj_b, fl_b = gpf.eval_full(Xb[None].contiguous())
    dvf, warped = gpf.transform(Xb, own=1)
    torch.cuda.synchronize()
    dvf, warped = dvf.cpu().numpy(), warped.cpu().numpy()
    src, tgt = wf.moving, wf.fixed

    def dice(a, b):
        return float(2.0 * np.sum(a & b) / max(1, np.sum(a) + np.sum(b)))

    o_id, o_b = obj_id.cpu().numpy()[0], obj_b.cpu().numpy()[0]
    c = (np.array(src.shape[::-1]) - 1) / 2.0
    probes = {}
    # ideal displacement at target surface points along the axes: the intruded
    # face centre (half - depth from the centre) maps to the source face (half),
    # the target sphere (r_target) to the source sphere (r_source)
    for name, rt, rs in (("face", 15.0 - 6.0, 15.0), ("sphere", 5.0, 9.0)):
        got = []
        for a in range(3):
            for sgn in (-1.0, 1.0):
                p = c.copy()
                p[a] += sgn * rt
                v = np.rint(p).astype(int)
                u = dvf[v[2], v[1], v[0]]
                got.append(float(sgn * u[a]))
        probes[name] = {"ideal_normal_mm": rs - rt, "found_normal_mm": got}
    mag = np.sqrt(np.sum(dvf ** 2, axis=-1))
    zs = 25
    step = 5
    sl = dvf[zs, ::step, ::step, :2]
    res["selected"] = {
        "archive_size": len(arch), "index": best, "fold_flags": int(fl_b.cpu().numpy()[0]),
        "objectives_identity": o_id.tolist(), "objectives_selected": o_b.tolist(),
        "guidance_rms_mm": {"identity": float(np.sqrt(o_id[2])), "selected": float(np.sqrt(o_b[2]))},
        "dice_cube": {"before": dice(src > 0.25, tgt > 0.25), "after": dice(warped > 0.25, tgt > 0.25)},
        "dice_sphere": {"before": dice(src > 0.75, tgt > 0.75), "after": dice(warped > 0.75, tgt > 0.75)},
        "mean_sq_diff": {"before": float(np.mean((src - tgt) ** 2)), "after": float(np.mean((warped - tgt) ** 2))},
        "dvf_mm": {"max": float(mag.max()), "mean_in_cube": float(mag[tgt > 0.25].mean())},
        "probes": probes,
        "dvf_slice": {"z": zs, "step": step, "ux_uy_mm": np.round(sl, 2).tolist()}}
    res["front"] = {"size": len(arch), "sim_range": [float(arch[:, 0].min()), float(arch[:, 0].max())],
                    "def_range": [float(arch[:, 1].min()), float(arch[:, 1].max())],
                    "guid_range": [float(arch[:, 2].min()), float(arch[:, 2].max())],
                    "by_guidance": arch[np.argsort(arch[:, 2])][np.linspace(0, len(arch) - 1, 12).astype(int)].tolist()}
    print(json.dumps(res), flush=True)


def transform_bench(reps=5):
    """The registration output (dsm_transform: DVF and transformed image, Sec.
    2.1 / Fig. 2) of one solution of the 512x512x100 clinical-shaped pair, both
    directions, timed with HIP events.  Algorithmic bytes per voxel: 16 written
    (3 DVF components and the transformed value, FP32) + 4 for the sampled
    voxel of the other image, as for the sweep."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.clinical()
    gp = dsm.Problem.from_workload(w, max_solutions=1, max_fos=1)
    X = w.population(reject=lambda X: gp.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0, S=1)
    X2 = torch.from_numpy(X[0]).to(dev)
    V = int(np.prod(w.fixed.shape))
    Dz, Dy, Dx = w.fixed.shape
    dvf = torch.empty((Dz, Dy, Dx, 3), dtype=torch.float32, device=dev)
    warped = torch.empty((Dz, Dy, Dx), dtype=torch.float32, device=dev)
    L = dsm.lib()
    out = {"workload": w.name, "voxels": V, "bytes_per_voxel": 20}
    for own in (1, 0):
        def call():
            dsm._check(L.dsm_transform(gp._h, own, dsm._dptr(X2), dsm._dptr(dvf), dsm._dptr(warped), None))
        call()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        for r in range(reps):
            ev[2 * r].record()
            call()
            ev[2 * r + 1].record()
        torch.cuda.synchronize()
        ms = float(np.mean([ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps)]))
        gbs = 20.0 * V / (ms / 1e3) / 1e9
        nan = int(torch.isnan(dvf).sum().item())
        log(f"transform own={own}: {ms:.3f} ms per call, {V / (ms / 1e3) / 1e9:.2f} G voxels/s, "
            f"{gbs:.0f} GB/s algorithmic, uncovered voxels {nan}")
        out["target" if own == 1 else "source"] = {"ms": ms, "voxels_per_s": V / (ms / 1e3), "algorithmic_GBps": gbs,
                                                   "roofline_frac": gbs / 8000.0, "uncovered": nan}
    print(json.dumps(out), flush=True)


def uneven_batch(steps=3, warmup=1):
    """Several registration problems of uneven size in one fused launch per
    pyramid level: the 12 problems of workloads.UNEVEN_PROBLEMS at the 2x
    box-averaged level and at full resolution (population handed off by
    x -> 2x + 0.5); per level, all single-point FOS elements of every
    solution.  Each problem's image row pitch, chunk and row order are
    autotuned first (the row order also on the whole batch).  Timed three
    ways: one dsm_eval_partial_batch call per level (job table uploaded per
    call), one dsm_batch_run per level (stored configuration), and one HIP
    graph holding both levels' runs (a whole two-level generation)."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import workloads as W
    dev = torch.device("cuda:0")
    n = len(W.UNEVEN_PROBLEMS)
    res = {"problems": n, "levels": []}
    handoff = {}
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))

    keep = []
    for level in (0, 1):
        t0 = time.perf_counter()
        ws = W.uneven(level=level)
        jobs = []
        for i, w in enumerate(ws):
            gp = dsm.Problem.from_workload(w)

            def reject(X, gp=gp):
                return gp.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0

            X = w.population(reject=reject) if level == 0 else W.upsample_population(handoff[i])
            if level == 0:
                handoff[i] = X
            off, pts = w.fos()
            cand = w.candidates(X, off, pts)
            Xd = torch.from_numpy(X).to(dev)
            offd, ptsd, cd = (torch.from_numpy(a).to(dev) for a in (off, pts, cand))
            cache = torch.empty((X.shape[0], gp.T, 3), dtype=torch.float64, device=dev)
            gp.eval_full(Xd, tet_terms=cache)
            gp.autotune_pitch(Xd, offd, ptsd, cd, tet_terms_in=cache)
            gp.autotune_chunk(Xd, offd, ptsd, cd, tet_terms_in=cache)
            gp.autotune_row_order(Xd, offd, ptsd, cd, tet_terms_in=cache)
            jobs.append(dict(problem=gp, X=Xd, fos_off=offd, fos_pts=ptsd, cand=cd, tet_terms_in=cache))
        log(f"uneven level {level}: {n} problems set up in {time.perf_counter() - t0:.1f} s")
        # A problem timed alone fills the GPU less than the fused launch does, so
        # the row orders are also compared on the whole stored batch: as tuned
        # per problem, all by slice, all by slice pair; the fastest is kept.
        tuned = [j["problem"].row_order for j in jobs]
        choice = {}
        for name, orders in (("per problem", tuned), ("by slice", [0] * n), ("by slice pair", [1] * n)):
            for j, o in zip(jobs, orders):
                j["problem"].set_row_order(o)
            trial = dsm.Batch(max_jobs=n)
            trial.set_jobs(jobs)
            choice[name] = (timed(trial.run), orders)
            del trial
        best_name = min(choice, key=lambda k: choice[k][0])
        for j, o in zip(jobs, choice[best_name][1]):
            j["problem"].set_row_order(o)
        log(f"uneven level {level}: row orders on the stored batch (ms) "
            f"{ {k: round(v[0], 3) for k, v in choice.items()} } -> {best_name}")
        batch = dsm.Batch(max_jobs=n)
        outs = batch.eval_partial(jobs)
        torch.cuda.synchronize()
        samples = int(sum(int(o[3].to(torch.int64).sum().item()) for o in outs))
        evals = sum(j["X"].shape[0] * (j["fos_off"].shape[0] - 1) for j in jobs)
        flagged = int(sum(int((o[2] != 0).sum().item()) for o in outs))
        ms = timed(lambda: batch.eval_partial(jobs))
        stored = dsm.Batch(max_jobs=n)
        stored.set_jobs(jobs)
        ms_run = timed(stored.run)
        log(f"uneven level {level}: {evals} partial evaluations, {samples} samples, {flagged} flagged, {ms:.2f} ms "
            f"per fused launch ({ms_run:.2f} ms from the stored configuration)")
        res["levels"].append({"level": level, "partial_evals": evals, "voxel_samples": samples, "ms": ms,
                              "ms_stored": ms_run,
                              "partial_evals_per_s": evals / (ms / 1e3), "voxel_samples_per_s": samples / (ms / 1e3),
                              "algorithmic_GBps": samples * BYTES_PER_SAMPLE / (ms_run / 1e3) / 1e9,
                              "roofline_frac": samples * BYTES_PER_SAMPLE / (ms_run / 1e3) / 1e9 / HBM_PEAK_GBS,
                              "part_chunks": [j["problem"].part_chunk for j in jobs],
                              "row_orders": [j["problem"].row_order for j in jobs],
                              "row_pitches": [j["problem"].pitch for j in jobs]})
        keep.append((batch, stored, jobs))
    # both levels in one captured graph
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for _, stored, _ in keep:
            stored.run()
    torch.cuda.synchronize()
    ms_graph = timed(graph.replay)
    log(f"uneven: both levels replayed from one HIP graph in {ms_graph:.2f} ms")
    tot_e = sum(l["partial_evals"] for l in res["levels"])
    tot_ms = sum(l["ms"] for l in res["levels"])
    res["total"] = {"partial_evals": tot_e, "voxel_samples": sum(l["voxel_samples"] for l in res["levels"]),
                    "ms": tot_ms, "ms_graph_both_levels": ms_graph, "partial_evals_per_s": tot_e / (tot_ms / 1e3),
                    "partial_evals_per_s_graph": tot_e / (ms_graph / 1e3)}
    print(json.dumps(res), flush=True)


def multires(G1, G2, S1=256, S2=512, coarse_mesh=(6, 6, 4)):
    """Sec. 2.4 multi-resolution run on the 512x512x100 pair: G1 generations on
    a coarse mesh (population S1), then a random sample of S2 solutions of its
    approximation set refined to 2n-1 points per axis and G2 generations there
    (the paper's scheme: 6^3 -> 11^3 grids, populations 250 -> 500).
    Generations replay captured HIP graphs."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import optimizer as O
    from paper_2202_11001_amd import workloads as W
    dev = torch.device("cuda:0")
    wc = W.clinical(mesh=coarse_mesh, S=S1)
    gpc = dsm.Problem.from_workload(wc)
    X = wc.population(reject=lambda X: gpc.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0)
    fine_mesh = tuple(2 * n - 1 for n in coarse_mesh)
    wf = W.clinical(mesh=fine_mesh, S=S2)
    gpf = dsm.Problem.from_workload(wf)
    t0 = time.perf_counter()
    oc = O.Optimiser(gpc, torch.from_numpy(X).to(dev), sigma=1.0, seed=21, graph=True, keep_solutions=True)
    hv_c = [oc.hypervolume()]
    for g in range(G1):
        oc.generation()
        hv_c.append(oc.hypervolume())
        if (g + 1) % 20 == 0:
            log(f"coarse {coarse_mesh} gen {g + 1}: hv {hv_c[-1]:.6g} archive {len(oc.archive)}")
    torch.cuda.synchronize()
    t_coarse = time.perf_counter() - t0
    t0 = time.perf_counter()
    Xf, rejected = O.seed_finer(oc, gpf, S2, seed=22)
    torch.cuda.synchronize()
    t_seed = time.perf_counter() - t0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    dsm.refine_population(coarse_mesh, oc.X)
    ev[1].record()
    torch.cuda.synchronize()
    refine_ms = ev[0].elapsed_time(ev[1])
    log(f"seeded {S2} refined solutions on {fine_mesh} ({rejected} draws rejected) in {t_seed:.2f} s; "
        f"refining {S1} solutions takes {refine_ms:.3f} ms")
    t0 = time.perf_counter()
    of = O.Optimiser(gpf, Xf, sigma=0.5, seed=23, graph=True)
    hv_f = [of.hypervolume()]
    for g in range(G2):
        of.generation()
        hv_f.append(of.hypervolume())
        if (g + 1) % 20 == 0:
            log(f"fine {fine_mesh} gen {g + 1}: hv {hv_f[-1]:.6g} archive {len(of.archive)}")
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    res = {"workload": wf.name, "coarse": {"mesh": coarse_mesh, "S": S1, "generations": G1, "seconds": t_coarse,
                                            "hv_first": hv_c[0], "hv_last": hv_c[-1], "archive": len(oc.archive)},
           "seed": {"S": S2, "rejected_draws": rejected, "seconds": t_seed, "refine_ms": refine_ms},
           "fine": {"mesh": fine_mesh, "S": S2, "generations": G2, "seconds": t_fine, "hv_first": hv_f[0],
                    "hv_last": hv_f[-1], "archive": len(of.archive)}}
    print(json.dumps(res), flush=True)


def tetrahedron_fos_step(steps=3, warmup=1):
    """Partial evaluation with the paper's FOS on the 512x512x100 pair: per
    cube one of its 6 tetrahedra, whose 4 points move together (in both
    grids); all 405 elements of all 512 solutions in one launch."""
    import torch
    from paper_2202_11001_amd import dsm
    from paper_2202_11001_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.clinical()
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    X = w.population(reject=lambda X: gp.fold_check(torch.from_numpy(X).to(dev)).cpu().numpy() != 0)
    top = gp.topology()
    n_cubes = gp.T // 6
    off, pts = W.tetrahedron_fos(top["tets"], n_cubes, seed=41)
    cand = w.candidates(X, off, pts)
    Xd = torch.from_numpy(X).to(dev)
    offd, ptsd, cd = (torch.from_numpy(a).to(dev) for a in (off, pts, cand))
    cache = torch.empty((w.S, gp.T, 3), dtype=torch.float64, device=dev)
    gp.eval_full(Xd, tet_terms=cache)
    out = gp.eval_partial(Xd, offd, ptsd, cd, tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    samples = int(out[3].to(torch.int64).sum().item())
    flagged = int((out[2] != 0).sum().item())
    for _ in range(warmup):
        gp.eval_partial(Xd, offd, ptsd, cd, tet_terms_in=cache, out=out)
    torch.cuda.synchronize()
    gp.timing(steps)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        gp.eval_partial(Xd, offd, ptsd, cd, tet_terms_in=cache, out=out)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
    kms = float(np.mean(gp.timing_read()))
    gp.timing(0)
    evals = w.S * n_cubes
    log(f"tetrahedron FOS: {evals} partial evaluations of 4-point elements, {samples} samples, {flagged} flagged, "
        f"{ms:.2f} ms per step (sweep {kms:.2f} ms)")
    print(json.dumps({"workload": w.name, "fos": "one tetrahedron per cube (4 points)", "partial_evals": evals,
                      "voxel_samples": samples, "flagged": flagged, "ms_per_step": ms, "sweep_ms": kms,
                      "partial_evals_per_s": evals / (ms / 1e3), "voxel_samples_per_s": samples / (ms / 1e3),
                      "algorithmic_GBps": samples * BYTES_PER_SAMPLE / (kms / 1e3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--small", action="store_true", help="64^3 workload (quick check)")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3: 2 steps, no warmup, no CPU leg")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the copy kernel of known size")
    ap.add_argument("--no-screen", action="store_true", help="skip the surrogate-screened step")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default image row pitch, chunk and row order")
    ap.add_argument("--part-chunk", type=int, default=0,
                    help="affected tetrahedra per workgroup (4..8) instead of autotuning it")
    ap.add_argument("--row-order", type=int, default=-1, choices=(-1, 0, 1),
                    help="row order of the sweep (0 by slice, 1 by slice pair; -1: autotuned)")
    ap.add_argument("--multires", type=int, nargs=2, default=None, metavar=("G1", "G2"),
                    help="multi-resolution run: G1 coarse then G2 fine generations (reported separately)")
    ap.add_argument("--tet-fos", action="store_true",
                    help="partial evaluation with the paper's one-tetrahedron-per-cube FOS (reported separately)")
    ap.add_argument("--transform", action="store_true",
                    help="DVF and transformed image of one 512x512x100 solution (reported separately)")
    ap.add_argument("--uneven", action="store_true",
                    help="12 problems of uneven size in one fused launch per pyramid level (reported separately)")
    ap.add_argument("--surrogate-run", type=int, default=0, metavar="G",
                    help="plain vs surrogate-screened optimiser runs of G generations (hypervolume protocol)")
    ap.add_argument("--train-generations", type=int, default=30)
    ap.add_argument("--sampler-run", type=int, default=0, metavar="G",
                    help="G generations with isotropic vs estimated-distribution candidates (reported separately)")
    ap.add_argument("--phantom", type=int, nargs=2, default=None, metavar=("G1", "G2"),
                    help="synthetic-phantom registration: G1 coarse then G2 fine generations (reported separately)")
    ap.add_argument("--clusters", type=int, default=1, help="clusters of the selection for --phantom")
    ap.add_argument("--ams", action="store_true", help="anticipated mean shift for --phantom")
    ap.add_argument("--forced", action="store_true", help="forced improvements for --phantom")
    ap.add_argument("--single-objective", action="store_true", help="single-objective clusters for --phantom")
    ap.add_argument("--sdr", action="store_true", help="standard-deviation-ratio multiplier schedule for --phantom")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.uneven:
        uneven_batch()
        return
    if args.transform:
        transform_bench()
        return
    if args.multires:
        multires(*args.multires)
        return
    if args.phantom:
        phantom_run(*args.phantom, clusters=args.clusters, ams=args.ams, forced=args.forced,
                    single_objective=args.single_objective, schedule="sdr" if args.sdr else "simple")
        return
    if args.tet_fos:
        tetrahedron_fos_step()
        return
    if args.profile:
        args.steps, args.warmup, args.no_cpu, args.no_screen = 2, 0, True, True
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} not supported: this evaluator runs on one GPU; a population "
              f"would shard by solutions across GPUs with no exchange during evaluation, which is not built",
              file=sys.stderr)
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
    if args.sampler_run:
        sampler_run(gp, X, args.sampler_run, w.name, w)
        return
    if args.surrogate_run:
        surrogate_run(gp, X, args.surrogate_run, args.train_generations, w.name, w)
        return
    off, pts = w.fos()
    F = len(off) - 1
    cand = w.candidates(X, off, pts)
    Xd = torch.from_numpy(X).to(dev)
    offd, ptsd, candd = (torch.from_numpy(a).to(dev) for a in (off, pts, cand))
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=dev)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    if not args.no_autotune and not args.profile:
        best, table = gp.autotune_pitch(Xd, offd, ptsd, candd, tet_terms_in=cache)
        log(f"image row pitch autotune (ms per step): {table} -> {best}")
        if not args.part_chunk:
            best, table = gp.autotune_chunk(Xd, offd, ptsd, candd, tet_terms_in=cache)
            log(f"affected tetrahedra per workgroup autotune (ms per step): {table} -> {best}")
        if args.row_order < 0:
            best, table = gp.autotune_row_order(Xd, offd, ptsd, candd, tet_terms_in=cache)
            log(f"row order autotune (0 by slice, 1 by slice pair; ms per step): {table} -> {best}")
    if args.part_chunk:
        gp.set_part_chunk(args.part_chunk)
    if args.row_order >= 0:
        gp.set_row_order(args.row_order)
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

    screened = None if args.no_screen else screened_step(gp, Xd, offd, ptsd, candd, cache, out, w, S, F)
    generation = None if args.profile else generation_timing(gp, Xd)
    if generation:
        log(f"optimiser generation ms: {generation}")

    evals_per_s = S * F / (ms / 1e3)
    samples_per_s = samples / (ms / 1e3)
    achieved = samples * BYTES_PER_SAMPLE / (kms / 1e3) / 1e9
    achieved_step = samples * BYTES_PER_SAMPLE / (ms / 1e3) / 1e9
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
        "tuning": {"image_row_pitch": gp.pitch, "part_chunk": gp.part_chunk, "row_order": gp.row_order},
        # "bound" names the roofline the fraction is taken against (HBM, on
        # algorithmic bytes); "limiter" is what the kernel's counters show
        # limits it: the vector-memory (texture) address and data path, with
        # HBM-side traffic a few percent of the algorithmic bytes because both
        # images stay in the caches.
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "limiter": "vector-memory gather path (texture address and data units busy 97-100 %)",
                     "frac_step": achieved_step / HBM_PEAK_GBS,
                     "hbm_measured_GBps": traffic / (kms / 1e3) / 1e9 if traffic else None,
                     "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source, scaled by a copy "
                                       "kernel (profiles/k_sweep_partial_clinical_traffic.txt); not re-measured "
                                       "in this run" if traffic else None,
                     "kernel": f"k_sweep<1, {gp.row_order}> (partial-evaluation voxel sweep)", "kernel_ms": kms,
                     "algorithmic_bytes_per_launch": samples * BYTES_PER_SAMPLE,
                     "kernel_source_sha256_16": kernel_source_hash()},
    }
    if screened is not None:
        res["screened"] = screened
    if generation is not None:
        res["generation"] = generation
    if not args.no_cpu:
        log("cpu baseline (oracle)...")
        res["cpu_baseline"] = cpu_baseline(w, X, off, pts, cand)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
