"""Shared helpers for the tests: build oracle and GPU problems from one seeded
workload and compare results to the parity bar."""
import numpy as np

from oracle import ref
from paper_2202_11001_amd import workloads as W

REL = 1e-5     # relative tolerance of every objective (FP32 sampling vs FP64 oracle)
ABS = 1e-7     # absolute floor for objectives that are (near) zero


def oracle_problem(w, **kw):
    return ref.Problem(w.moving, w.fixed, w.mesh, w.spacing, w.tau, guid_moving=w.guid_moving,
                       corr_moving=w.corr_moving, guid_fixed=w.guid_fixed, corr_fixed=w.corr_fixed, **kw)


def feasible_population(w, rp, S=None):
    return w.population(reject=lambda X: rp.fold_check(X)[0] != 0, S=S)


def assert_objectives_close(gpu, ref_, flags=None, rel=REL, abs_=ABS, what="objective"):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref_ = np.asarray(ref_, dtype=np.float64)
    ok = np.abs(gpu - ref_) <= rel * np.abs(ref_) + abs_
    if flags is not None:
        ok |= (np.asarray(flags) != 0)[..., None] if ok.ndim > np.asarray(flags).ndim else (np.asarray(flags) != 0)
    if not ok.all():
        bad = np.argwhere(~ok)[:5]
        msg = "; ".join(f"{tuple(b)}: gpu {gpu[tuple(b)]!r} ref {ref_[tuple(b)]!r}" for b in bad)
        raise AssertionError(f"{what}: {int((~ok).sum())} entries outside rel {rel} abs {abs_}: {msg}")


def assert_delta_close(gpu_old, gpu_new, ref_old, ref_new, flags, rel=REL, abs_=ABS):
    """Delta of a partial change within rel * (|old| + |new|)."""
    dg = np.asarray(gpu_new) - np.asarray(gpu_old)
    dr = np.asarray(ref_new) - np.asarray(ref_old)
    tol = rel * (np.abs(ref_old) + np.abs(ref_new)) + abs_
    ok = (np.abs(dg - dr) <= tol) | (np.asarray(flags) != 0)[..., None]
    if not ok.all():
        bad = np.argwhere(~ok)[:5]
        msg = "; ".join(f"{tuple(b)}: gpu {dg[tuple(b)]!r} ref {dr[tuple(b)]!r}" for b in bad)
        raise AssertionError(f"delta: {int((~ok).sum())} entries outside tolerance: {msg}")
