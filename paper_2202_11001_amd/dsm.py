"""Python binding of libdsm (``include/dsm.h``): argument marshalling only.

Every computation runs in the library's HIP kernels; this module converts
torch tensors to device pointers, allocates outputs with torch and passes the
current torch stream.  There is no fallback: if ``libdsm.so`` is missing the
import of the library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dsm.h")

OK, ERR_ARG, ERR_CAPACITY, ERR_DOMAIN, ERR_DEVICE, ERR_NOMEM, ERR_UNSUPPORTED = range(7)
FLAG_INV_MOVING, FLAG_INV_FIXED, FLAG_BORDER, FLAG_DOMAIN, FLAG_LATTICE, FLAG_NONFINITE, FLAG_BAD_FOS = (
    1, 2, 4, 8, 16, 32, 64)
FLAG_SKIPPED = 128


class DsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dsm status {status}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("spacing_mm", C.c_float * 3), ("moving", C.c_void_p),
                ("fixed", C.c_void_p), ("mesh", C.c_int32 * 3), ("empty_tau", C.c_float),
                ("n_guid_moving", C.c_int32), ("n_guid_fixed", C.c_int32), ("guid_moving", C.c_void_p),
                ("guid_fixed", C.c_void_p), ("corr_moving", C.c_void_p), ("corr_fixed", C.c_void_p),
                ("max_solutions", C.c_int32), ("max_fos", C.c_int32), ("max_fos_points", C.c_int32)]


class SurrogateDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("max_rows", C.c_int32), ("max_batch", C.c_int32)]


class PartialJob(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("S", C.c_int32), ("X", C.c_void_p), ("F", C.c_int32),
                ("fos_off", C.c_void_p), ("fos_pts", C.c_void_p), ("cand", C.c_void_p), ("mask", C.c_void_p),
                ("tet_terms_in", C.c_void_p), ("part_old", C.c_void_p), ("part_new", C.c_void_p),
                ("flags", C.c_void_p), ("tet_terms_new", C.c_void_p), ("voxel_count", C.c_void_p)]


class ProblemInfo(C.Structure):
    _fields_ = [("P", C.c_int32), ("T", C.c_int32), ("E", C.c_int32), ("max_star", C.c_int32),
                ("V", C.c_int64), ("max_affected", C.c_int32), ("norm", C.c_double * 3), ("pitch", C.c_int32)]


_lib = None


def lib():
    """Loads libdsm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() (the HIP path has no fallback)")
        L = C.CDLL(LIB_PATH)
        V, I = C.c_void_p, C.c_int32
        sig = {
            "dsm_status_string": ([I], C.c_char_p),
            "dsm_last_error": ([], C.c_char_p),
            "dsm_problem_create": ([V, V], I),
            "dsm_problem_destroy": ([V], I),
            "dsm_problem_query": ([V, V], I),
            "dsm_problem_topology": ([V, V, V, V, V], I),
            "dsm_mesh_topology": ([V, V, V, V, V, V, V], I),
            "dsm_fold_check": ([V, I, V, V, V, V], I),
            "dsm_eval_full": ([V, I, V, V, V, V, V], I),
            "dsm_eval_partial": ([V, I, V, I, V, V, V, V, V, V, V, V, V, V], I),
            "dsm_eval_partial_noalloc": ([V, I, V, I, V, V, V, V, V, V, V, V, V, V], I),
            "dsm_rasterize_owner": ([V, V, V, V, V], I),
            "dsm_transform": ([V, I, V, V, V, V], I),
            "dsm_problem_timing": ([V, I], I),
            "dsm_problem_timing_read": ([V, V, I, V], I),
            "dsm_eval_partial_masked": ([V, I, V, I, V, V, V, V, V, V, V, V, V, V, V], I),
            "dsm_sample_candidates": ([V, I, V, I, V, I, C.c_float, C.c_uint64, C.c_uint64, V, V, V], I),
            "dsm_estimate_distributions": ([V, I, V, I, V, I, V, V, V, V], I),
            "dsm_sample_estimated": ([V, I, V, I, V, I, V, V, V, I, V, V, V, C.c_double, C.c_uint64, C.c_uint64, V,
                                      V, V], I),
            "dsm_estimate_elements": ([V, I, V, I, V, I, V, V, V, V, V], I),
            "dsm_sample_elements": ([V, I, V, I, V, V, V, V, V, I, V, V, V, C.c_double, C.c_uint64, C.c_uint64, V,
                                     V, V], I),
            "dsm_cluster_objectives": ([I, V, I, V, I, V, V, V, V], I),
            "dsm_copy_from_donor": ([V, I, V, I, V, V, V, V], I),
            "dsm_improvement_ratio": ([I, I, V, V, V, I, V, V, V, I, V, V], I),
            "dsm_accept": ([V, I, V, I, V, V, V, V, V, V, V, V, I, V, V, V, V], I),
            "dsm_accept_elements": ([V, I, V, I, V, V, V, V, V, V, V, V, V, I, V, V, V, V], I),
            "dsm_batch_create": ([I, V], I),
            "dsm_batch_destroy": ([V], I),
            "dsm_eval_partial_batch": ([V, I, V, V], I),
            "dsm_batch_set_jobs": ([V, I, V], I),
            "dsm_archive_work_bytes": ([I, I, I], C.c_size_t),
            "dsm_archive_merge": ([I, V, V, I, V, I, V, V, V, V, V], I),
            "dsm_select": ([I, V, I, V, V, V], I),
            "dsm_avs_update": ([I, V, V, V, I, C.c_float, C.c_float, C.c_float, V], I),
            "dsm_mark_improved": ([I, I, V, V, V], I),
            "dsm_multiplier_step": ([I, I, I, V, V, V, C.c_float, C.c_float, C.c_float, V], I),
            "dsm_forced_work_bytes": ([V, I], C.c_size_t),
            "dsm_forced_replace": ([V, I, V, V, V, V, V, V, V, V, V], I),
            "dsm_batch_run": ([V, V], I),
            "dsm_problem_set_pitch": ([V, I], I),
            "dsm_refine_population": ([V, I, V, V, V], I),
            "dsm_autotune_pitch": ([V, I, V, I, V, V, V, V, I, V, V, V], I),
            "dsm_ams_shift": ([I, V, V, V, I, V], I),
            "dsm_single_objective_clusters": ([I, V, I, V, V, V], I),
            "dsm_draw_donors": ([I, V, I, V, V, V, V, V], I),
            "dsm_set_part_chunk": ([V, I], I),
            "dsm_get_part_chunk": ([V], I),
            "dsm_autotune_chunk": ([V, I, V, I, V, V, V, V, I, V, V, V], I),
            "dsm_set_row_order": ([V, I], I),
            "dsm_get_row_order": ([V], I),
            "dsm_autotune_row_order": ([V, I, V, I, V, V, V, V, V, V], I),
            "dsm_surrogate_create": ([V, V], I),
            "dsm_surrogate_destroy": ([V], I),
            "dsm_surrogate_last_error": ([], C.c_char_p),
            "dsm_surrogate_params": ([V, V, I], I),
            "dsm_surrogate_fit_scaling": ([V, I, V, V, V], I),
            "dsm_surrogate_get_scaling": ([V, V, V, V, V], I),
            "dsm_surrogate_set_scaling": ([V, V, V, V, V], I),
            "dsm_surrogate_features": ([V, I, V, I, V, I, V, V, V], I),
            "dsm_surrogate_pack": ([V, I, V, V, V, V, V, V, V], I),
            "dsm_surrogate_features_packed": ([V, V, I, V, I, V, I, V, V, V], I),
            "dsm_surrogate_forward": ([V, I, V, V, V], I),
            "dsm_surrogate_gradient": ([V, I, V, V, V, V, V], I),
            "dsm_surrogate_train": ([V, I, V, V, I, I, V, V], I),
            "dsm_surrogate_screen": ([V, V, I, V, I, V, I, V, V, I, V, V, V, V, V, V], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def header_symbols():
    """Names of the functions declared in include/dsm.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsm_[a-z_]+)\s*\(", txt)))


def _check(st):
    if st != OK:
        L = lib()
        raise DsmError(st, f"{L.dsm_status_string(st).decode()}: {L.dsm_last_error().decode()}")


def _np_ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def refine_population(mesh_coarse, Xc, out=None, stream=None):
    """Sec. 2.4 refinement of a device population Xc [S][2][Pc][3] to the mesh of
    2n-1 points per axis: [S][2][Pf][3] (``dsm_refine_population``)."""
    torch = _torch()
    m = np.ascontiguousarray(mesh_coarse, dtype=np.int32)
    S = Xc.shape[0]
    Pf = int(np.prod(2 * m - 1))
    if out is None:
        out = torch.empty((S, 2, Pf, 3), dtype=torch.float32, device=Xc.device)
    _check(lib().dsm_refine_population(_np_ptr(m), S, _dptr(Xc), _dptr(out), _stream(stream)))
    return out


def cluster_objectives(obj, sel, k, stream=None):
    """Balanced k-leader-means clustering of the selected solutions sel [n]
    int32 in objective space obj [S][3] float64 (``dsm_cluster_objectives``):
    (members [k][cmax] int32, assign [S] int32, means [k][3] float64)."""
    torch = _torch()
    if obj.dtype != torch.float64 or obj.dim() != 2 or obj.shape[1] != 3 or sel.dtype != torch.int32:
        raise ValueError("cluster_objectives: obj float64 [S][3] and sel int32 [n] expected")
    S, n = obj.shape[0], sel.shape[0]
    cmax = min(n, -(-2 * n // k)) if k > 0 else 0
    members = torch.empty((max(k, 0), cmax), dtype=torch.int32, device=obj.device)
    assign = torch.empty(S, dtype=torch.int32, device=obj.device)
    means = torch.empty((max(k, 0), 3), dtype=torch.float64, device=obj.device)
    _check(lib().dsm_cluster_objectives(S, _dptr(obj), n, _dptr(sel), int(k), _dptr(members) if cmax else None,
                                        _dptr(assign) if S else None, _dptr(means), _stream(stream)))
    return members, assign, means


def improvement_ratio(off, cand, accepted, mean, chol, cluster=None, stream=None):
    """Standard-deviation ratio of the accepted candidates per (cluster,
    element) (``dsm_improvement_ratio``): off int32 [F+1], cand [S][off[F]][2][3],
    accepted uint8 [S][F], mean float64 [C][F][n] and chol [C][F][n(n+1)/2]
    with n = 6 or 24; returns float64 [C][F] (-1: nothing accepted)."""
    torch = _torch()
    S, F = accepted.shape[0], off.shape[0] - 1
    n_vars = 6 if chol.shape[-1] == 21 else 24
    C = max(1, mean.numel() // max(1, F * n_vars))
    if (mean.dtype != torch.float64 or chol.dtype != torch.float64 or mean.numel() != C * F * n_vars
            or chol.numel() != C * F * n_vars * (n_vars + 1) // 2 or accepted.dtype != torch.uint8
            or accepted.numel() != S * F or off.dtype != torch.int32):
        raise ValueError("improvement_ratio: argument shapes or dtypes")
    if cluster is not None and (cluster.dtype != torch.int32 or cluster.numel() != S):
        raise ValueError("improvement_ratio: cluster int32 [S] expected")
    out = torch.empty((C, F), dtype=torch.float64, device=accepted.device)
    _check(lib().dsm_improvement_ratio(S, F, _dptr(off), _dptr(cand), _dptr(accepted), C, _dptr(cluster),
                                       _dptr(mean), _dptr(chol), n_vars, _dptr(out), _stream(stream)))
    return out


class Archive:
    """The elitist archive on the device (``dsm_archive_merge``): vectors
    float64 [capacity][3] in lexicographic order, +inf after the count; with
    row_floats > 0 a payload row per vector.  The count lives on the device
    (``n_dev``); ``n`` reads it."""

    def __init__(self, capacity, m_max, row_floats=0, device="cuda:0"):
        torch = _torch()
        self.capacity, self.m_max, self.row_floats = int(capacity), int(m_max), int(row_floats)
        self.vec = torch.full((self.capacity, 3), float("inf"), dtype=torch.float64, device=device)
        self.rows = torch.empty((self.capacity, self.row_floats), dtype=torch.float32, device=device) \
            if self.row_floats else None
        self.n_dev = torch.zeros(1, dtype=torch.int32, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        nbytes = lib().dsm_archive_work_bytes(self.capacity, self.m_max, self.row_floats)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=device)

    @property
    def n(self):
        return int(self.n_dev.item())

    def merge(self, points, rows=None, stream=None):
        """Merges points float64 [m][3] (m <= m_max), with payload rows [m][row_floats] if the archive has them."""
        torch = _torch()
        m = points.shape[0]
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3 or m > self.m_max:
            raise ValueError(f"archive merge: points float64 [m][3] with m <= {self.m_max} expected")
        if self.row_floats and (rows is None or rows.dtype != torch.float32 or rows.numel() != m * self.row_floats):
            raise ValueError(f"archive merge: rows float32 [m][{self.row_floats}] expected")
        _check(lib().dsm_archive_merge(self.capacity, _dptr(self.vec), _dptr(self.n_dev), m, _dptr(points),
                                       self.row_floats, _dptr(self.rows), _dptr(rows) if self.row_floats else None,
                                       _dptr(self.work), _dptr(self.overflow), _stream(stream)))


def select(obj, n_sel, dominated_by=None, stream=None):
    """Selection (``dsm_select``): int32 [n_sel] indices of obj float64 [S][3]
    with the fewest dominating members, ties by the normalised objective sum;
    dominated_by int32 [S] receives the counts if given."""
    torch = _torch()
    S = obj.shape[0]
    if obj.dtype != torch.float64 or obj.dim() != 2 or obj.shape[1] != 3 or not 0 <= n_sel <= S:
        raise ValueError("select: obj float64 [S][3] and 0 <= n_sel <= S expected")
    if dominated_by is not None and (dominated_by.dtype != torch.int32 or dominated_by.numel() != S):
        raise ValueError("select: dominated_by int32 [S] expected")
    sel = torch.empty(n_sel, dtype=torch.int32, device=obj.device)
    _check(lib().dsm_select(S, _dptr(obj), int(n_sel), _dptr(sel), _dptr(dominated_by), _stream(stream)))
    return sel


def avs_update(mult, nis, sdr, nis_max, eta=0.9, lo=0.05, hi=10.0, stream=None):
    """Adaptive variance scaling in place (``dsm_avs_update``): mult float32,
    nis int32 and sdr float64 of equal size; returns (mult, nis)."""
    torch = _torch()
    n = mult.numel()
    if (mult.dtype != torch.float32 or nis.dtype != torch.int32 or sdr.dtype != torch.float64 or nis.numel() != n
            or sdr.numel() != n or not (mult.is_contiguous() and nis.is_contiguous() and sdr.is_contiguous())):
        raise ValueError("avs_update: contiguous mult float32, nis int32, sdr float64 of equal size expected")
    _check(lib().dsm_avs_update(n, _dptr(mult), _dptr(nis), _dptr(sdr), int(nis_max), float(eta), float(lo), float(hi),
                                _stream(stream)))
    return mult, nis


def multiplier_step(accepted, mult, cluster=None, eta=0.9, lo=0.05, hi=10.0, stream=None):
    """The simple multiplier schedule in place (``dsm_multiplier_step``):
    accepted uint8 [S][F], mult float32 [k][F] (contiguous), cluster int32 [S]
    (needed when k > 1)."""
    torch = _torch()
    S, F = accepted.shape
    k = mult.shape[0]
    if (accepted.dtype != torch.uint8 or mult.dtype != torch.float32 or mult.dim() != 2 or mult.shape[1] != F
            or not mult.is_contiguous() or (k > 1 and (cluster is None or cluster.dtype != torch.int32
                                                       or cluster.numel() != S))):
        raise ValueError("multiplier_step: accepted uint8 [S][F], mult float32 [k][F], cluster int32 [S] expected")
    _check(lib().dsm_multiplier_step(k, F, S, _dptr(accepted), _dptr(cluster) if k > 1 else None, _dptr(mult),
                                     float(eta), float(lo), float(hi), _stream(stream)))
    return mult


def mark_improved(accepted, improved, stream=None):
    """improved uint8 [S] |= any(accepted uint8 [S][F], axis 1) (``dsm_mark_improved``)."""
    torch = _torch()
    S = improved.numel()
    if accepted.dtype != torch.uint8 or improved.dtype != torch.uint8 or accepted.shape[0] != S:
        raise ValueError("mark_improved: accepted uint8 [S][F], improved uint8 [S] expected")
    F = accepted.numel() // max(1, S)
    _check(lib().dsm_mark_improved(S, F, _dptr(accepted), _dptr(improved), _stream(stream)))


def ams_shift(mean, prev, shift=None, has_prev=True, stream=None):
    """Anticipated mean shift (``dsm_ams_shift``): shift = mean - prev, then
    prev = mean, all float64 of equal size (prev, shift contiguous, updated in
    place); with has_prev False only prev = mean.  Returns shift."""
    torch = _torch()
    n = mean.numel()
    if (mean.dtype != torch.float64 or prev.dtype != torch.float64 or prev.numel() != n or not mean.is_contiguous()
            or not prev.is_contiguous() or (has_prev and (shift is None or shift.dtype != torch.float64
                                                          or shift.numel() != n or not shift.is_contiguous()))):
        raise ValueError("ams_shift: contiguous float64 mean, prev (and shift) of equal size expected")
    _check(lib().dsm_ams_shift(n, _dptr(mean), _dptr(prev), _dptr(shift) if has_prev else None, int(bool(has_prev)),
                               _stream(stream)))
    return shift


def single_objective_clusters(means, assign, stream=None):
    """Objective of every solution's cluster, or -1 (``dsm_single_objective_clusters``):
    means float64 [k][3], assign int32 [S]; returns int32 [S]."""
    torch = _torch()
    k, S = means.shape[0], assign.numel()
    if means.dtype != torch.float64 or means.dim() != 2 or means.shape[1] != 3 or assign.dtype != torch.int32:
        raise ValueError("single_objective_clusters: means float64 [k][3], assign int32 [S] expected")
    so = torch.empty(S, dtype=torch.int32, device=assign.device)
    _check(lib().dsm_single_objective_clusters(k, _dptr(means.contiguous()), S, _dptr(assign), _dptr(so),
                                               _stream(stream)))
    return so


def draw_donors(nis, nis_max, dominated_by, u, n_forced=None, stream=None):
    """Forced-improvement donors (``dsm_draw_donors``): nis and dominated_by
    int32 [S], u float32 [S] uniform draws in [0, 1); returns donor int32 [S]
    (-1 = none); n_forced int32 [1] is increased by the number of donors."""
    torch = _torch()
    S = nis.numel()
    if (nis.dtype != torch.int32 or dominated_by.dtype != torch.int32 or dominated_by.numel() != S
            or u.dtype != torch.float32 or u.numel() != S):
        raise ValueError("draw_donors: nis, dominated_by int32 [S] and u float32 [S] expected")
    donor = torch.empty(S, dtype=torch.int32, device=nis.device)
    _check(lib().dsm_draw_donors(S, _dptr(nis), int(nis_max), _dptr(dominated_by), _dptr(u), _dptr(donor),
                                 _dptr(n_forced), _stream(stream)))
    return donor


def mesh_topology(mesh, dims=None):
    """Host-only topology: dict of counts, tets [T][4], star_off, star, identity [P][3]."""
    L = lib()
    m = np.ascontiguousarray(mesh, dtype=np.int32)
    d = np.ascontiguousarray(dims, dtype=np.int32) if dims is not None else None
    cnt = np.zeros(4, np.int32)
    _check(L.dsm_mesh_topology(_np_ptr(m), _np_ptr(d), _np_ptr(cnt), None, None, None, None))
    P, T, E, ms = (int(x) for x in cnt)
    tets = np.zeros((T, 4), np.int32)
    off = np.zeros(P + 1, np.int32)
    st = np.zeros(4 * T, np.int32)
    ident = np.zeros((P, 3), np.float32) if d is not None else None
    _check(L.dsm_mesh_topology(_np_ptr(m), _np_ptr(d), None, _np_ptr(tets), _np_ptr(off), _np_ptr(st),
                               _np_ptr(ident)))
    return dict(P=P, T=T, E=E, max_star=ms, tets=tets, star_off=off, star=st, identity=ident)


def _torch():
    import torch
    return torch


def _check_dist(mean, chol, mult, cluster, S, n_dist, n_var, n_tri):
    """Host-side shape and dtype checks of per-element distributions before a
    sampler launch reads them: mean float64 [n_dist][n_var], chol float64
    [n_dist][n_tri], mult float32 [n_dist], cluster int32 [S] or None."""
    torch = _torch()
    for name, t, dt, n in (("mean", mean, torch.float64, n_dist * n_var), ("chol", chol, torch.float64, n_dist * n_tri),
                           ("mult", mult, torch.float32, n_dist)):
        if t.dtype != dt or t.numel() != n:
            raise ValueError(f"{name}: expected {dt} with {n} elements, got {t.dtype} with {t.numel()}")
    if cluster is not None and (cluster.dtype != torch.int32 or cluster.numel() != S):
        raise ValueError(f"cluster: expected int32 [{S}]")


def _check_single_objective(so, S):
    torch = _torch()
    if so is not None and (so.dtype != torch.int32 or so.numel() != S):
        raise ValueError(f"single_objective: expected int32 [{S}]")


def _check_shift(shift, ams, S, P):
    """Host-side checks of the anticipated-mean-shift arguments: shift float64
    [P][6] with ams uint8 [S], or neither."""
    torch = _torch()
    if shift is None:
        return
    if shift.dtype != torch.float64 or shift.numel() != 6 * P:
        raise ValueError(f"shift: expected float64 [{P}][6]")
    if ams is None or ams.dtype != torch.uint8 or ams.numel() != S:
        raise ValueError(f"ams: expected uint8 [{S}] with a shift")


def _dptr(t):
    if t is None:
        return None
    torch = _torch()
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Problem:
    """A registration problem resident on the current GPU (``dsm_problem``)."""

    def __init__(self, moving, fixed, mesh, spacing=(1.0, 1.0, 1.0), tau=0.1, guid_moving=None, corr_moving=None,
                 guid_fixed=None, corr_fixed=None, max_solutions=1, max_fos=0, max_fos_points=1):
        L = lib()
        moving = np.ascontiguousarray(moving, dtype=np.float32)
        fixed = np.ascontiguousarray(fixed, dtype=np.float32)
        if moving.shape != fixed.shape or moving.ndim != 3:
            raise ValueError("moving and fixed must be equal-shape 3-D arrays")
        gm = np.ascontiguousarray(guid_moving if guid_moving is not None else np.zeros((0, 3)), np.float32)
        gf = np.ascontiguousarray(guid_fixed if guid_fixed is not None else np.zeros((0, 3)), np.float32)
        cm = np.ascontiguousarray(corr_moving if corr_moving is not None else np.arange(len(gm)), np.int32)
        cf = np.ascontiguousarray(corr_fixed if corr_fixed is not None else np.arange(len(gf)), np.int32)
        d = ProblemDesc()
        d.dims[:] = [moving.shape[2], moving.shape[1], moving.shape[0]]
        d.spacing_mm[:] = [float(x) for x in spacing]
        d.moving, d.fixed = moving.ctypes.data, fixed.ctypes.data
        d.mesh[:] = [int(x) for x in mesh]
        d.empty_tau = float(tau)
        d.n_guid_moving, d.n_guid_fixed = len(gm), len(gf)
        d.guid_moving, d.guid_fixed = _np_ptr(gm), _np_ptr(gf)
        d.corr_moving, d.corr_fixed = _np_ptr(cm), _np_ptr(cf)
        d.max_solutions, d.max_fos, d.max_fos_points = int(max_solutions), int(max_fos), int(max_fos_points)
        h = C.c_void_p()
        _check(L.dsm_problem_create(C.byref(d), C.byref(h)))
        self._h = h
        info = ProblemInfo()
        _check(L.dsm_problem_query(self._h, C.byref(info)))
        self.P, self.T, self.E, self.max_star = info.P, info.T, info.E, info.max_star
        self.V, self.max_affected = info.V, info.max_affected
        self.norm = tuple(info.norm)
        self.dims = tuple(d.dims)
        self.mesh = tuple(d.mesh)

    @classmethod
    def from_workload(cls, w, max_solutions=None, max_fos=None, max_fos_points=1):
        return cls(w.moving, w.fixed, w.mesh, w.spacing, w.tau, w.guid_moving, w.corr_moving, w.guid_fixed,
                   w.corr_fixed, max_solutions=max_solutions or w.S,
                   max_fos=w.P if max_fos is None else max_fos, max_fos_points=max_fos_points)

    def close(self):
        if getattr(self, "_h", None):
            lib().dsm_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def topology(self):
        tets = np.zeros((self.T, 4), np.int32)
        off = np.zeros(self.P + 1, np.int32)
        st = np.zeros(4 * self.T, np.int32)
        ident = np.zeros((self.P, 3), np.float32)
        _check(lib().dsm_problem_topology(self._h, _np_ptr(tets), _np_ptr(off), _np_ptr(st), _np_ptr(ident)))
        return dict(tets=tets, star_off=off, star=st, identity=ident)

    def fold_check(self, X, first_bad=False, stream=None):
        torch = _torch()
        S = X.shape[0]
        flags = torch.empty(S, dtype=torch.int32, device=X.device)
        fb = torch.empty(S, dtype=torch.int32, device=X.device) if first_bad else None
        _check(lib().dsm_fold_check(self._h, S, _dptr(X), _dptr(flags), _dptr(fb), _stream(stream)))
        return (flags, fb) if first_bad else flags

    def eval_full(self, X, tet_terms=None, stream=None):
        torch = _torch()
        S = X.shape[0]
        obj = torch.empty((S, 3), dtype=torch.float64, device=X.device)
        flags = torch.empty(S, dtype=torch.int32, device=X.device)
        _check(lib().dsm_eval_full(self._h, S, _dptr(X), _dptr(obj), _dptr(flags), _dptr(tet_terms),
                                   _stream(stream)))
        return obj, flags

    def eval_partial(self, X, fos_off, fos_pts, cand, tet_terms_in=None, tet_terms_new=None, voxel_count=False,
                     out=None, mask=None, stream=None):
        torch = _torch()
        S, F = X.shape[0], fos_off.shape[0] - 1
        if out is None:
            out = (torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                   torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                   torch.empty((S, F), dtype=torch.int32, device=X.device),
                   torch.empty((S, F), dtype=torch.int32, device=X.device) if voxel_count else None)
        old, new, flags, vc = out
        if mask is None:
            _check(lib().dsm_eval_partial(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                          _dptr(tet_terms_in), _dptr(old), _dptr(new), _dptr(flags),
                                          _dptr(tet_terms_new), _dptr(vc), _stream(stream)))
        else:
            _check(lib().dsm_eval_partial_masked(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                                 _dptr(mask), _dptr(tet_terms_in), _dptr(old), _dptr(new),
                                                 _dptr(flags), _dptr(tet_terms_new), _dptr(vc), _stream(stream)))
        return out

    def eval_partial_noalloc(self, X, fos_off, fos_pts, cand, tet_terms_in=None, tet_terms_new=None,
                             voxel_count=False, out=None, stream=None):
        """eval_partial through dsm_eval_partial_noalloc (workspace in the
        library's fixed per-device array; pass ``out`` to allocate nothing here
        either)."""
        torch = _torch()
        S, F = X.shape[0], fos_off.shape[0] - 1
        if out is None:
            out = (torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                   torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                   torch.empty((S, F), dtype=torch.int32, device=X.device),
                   torch.empty((S, F), dtype=torch.int32, device=X.device) if voxel_count else None)
        old, new, flags, vc = out
        _check(lib().dsm_eval_partial_noalloc(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                              _dptr(tet_terms_in), _dptr(old), _dptr(new), _dptr(flags),
                                              _dptr(tet_terms_new), _dptr(vc), _stream(stream)))
        return out

    def sample_candidates(self, X, pts, K, sigma, seed, counter, out=None, stream=None, counter_dev=None):
        """Candidates [S][F][K][2][3] (K > 1) or [S][F][2][3] (K == 1); the counter is
        counter + counter_dev[0] when a device counter (int64 [1]) is given."""
        torch = _torch()
        S, F = X.shape[0], pts.shape[0]
        if out is None:
            shape = (S, F, 2, 3) if K == 1 else (S, F, K, 2, 3)
            out = torch.empty(shape, dtype=torch.float32, device=X.device)
        _check(lib().dsm_sample_candidates(self._h, S, _dptr(X), F, _dptr(pts), int(K), float(sigma), int(seed),
                                           int(counter), _dptr(counter_dev), _dptr(out), _stream(stream)))
        return out

    def estimate_distributions(self, X, sel, pts, stream=None):
        """(mean [F][6], lower Cholesky factor [F][21]) float64 of the single
        points pts [F] over the selected solutions sel [n] (int32) of X."""
        torch = _torch()
        if sel.dtype != torch.int32 or X.dtype != torch.float32:
            raise ValueError("X float32 and sel int32 expected")
        F = pts.shape[0]
        mean = torch.empty((F, 6), dtype=torch.float64, device=X.device)
        chol = torch.empty((F, 21), dtype=torch.float64, device=X.device)
        _check(lib().dsm_estimate_distributions(self._h, X.shape[0], _dptr(X), sel.shape[0], _dptr(sel), F, _dptr(pts),
                                                _dptr(mean), _dptr(chol), _stream(stream)))
        return mean, chol

    def sample_estimated(self, X, pts, K, mean, chol, mult, seed, counter, out=None, stream=None, counter_dev=None,
                         cluster=None, shift=None, ams=None, delta=2.0):
        """Candidates [S][F][K][2][3] (K > 1) or [S][F][2][3] (K == 1) drawn from
        N(mean, mult * L L^T) on the free coordinates (mult float32 [F]); with
        ``cluster`` [S] int32, mean/chol/mult hold one distribution per cluster
        ([C][F][...]) and solution s uses cluster[s]; with ``shift`` [P][6]
        float64 and ``ams`` [S] uint8 the flagged solutions draw around
        mean + delta * mult * shift (anticipated mean shift)."""
        torch = _torch()
        S, F = X.shape[0], pts.shape[0]
        _check_shift(shift, ams, S, self.P)
        if out is None:
            shape = (S, F, 2, 3) if K == 1 else (S, F, K, 2, 3)
            out = torch.empty(shape, dtype=torch.float32, device=X.device)
        nc = max(1, mean.numel() // max(1, 6 * F))
        _check_dist(mean, chol, mult, cluster, S, nc * F, 6, 21)
        _check(lib().dsm_sample_estimated(self._h, S, _dptr(X), F, _dptr(pts), int(K), _dptr(mean), _dptr(chol),
                                          _dptr(mult), nc, _dptr(cluster), _dptr(shift), _dptr(ams), float(delta),
                                          int(seed), int(counter), _dptr(counter_dev), _dptr(out), _stream(stream)))
        return out

    def accept(self, X, pts, cand, part_old, part_new, flags, terms_cand, terms_cache, obj, archive=None,
               accepted=None, stream=None, single_objective=None):
        na = 0 if archive is None else archive.shape[0]
        _check_single_objective(single_objective, X.shape[0])
        _check(lib().dsm_accept(self._h, X.shape[0], _dptr(X), pts.shape[0], _dptr(pts), _dptr(cand),
                                _dptr(part_old), _dptr(part_new), _dptr(flags), _dptr(terms_cand), _dptr(terms_cache),
                                _dptr(obj), na, _dptr(archive), _dptr(single_objective), _dptr(accepted),
                                _stream(stream)))

    def estimate_elements(self, X, sel, off, pts, stream=None):
        """Joint distributions of elements of up to 4 points (CSR off, pts):
        (mean [F][24], lower Cholesky factor [F][300]) float64."""
        torch = _torch()
        if sel.dtype != torch.int32 or X.dtype != torch.float32:
            raise ValueError("X float32 and sel int32 expected")
        F = off.shape[0] - 1
        mean = torch.empty((F, 24), dtype=torch.float64, device=X.device)
        chol = torch.empty((F, 300), dtype=torch.float64, device=X.device)
        _check(lib().dsm_estimate_elements(self._h, X.shape[0], _dptr(X), sel.shape[0], _dptr(sel), F, _dptr(off),
                                           _dptr(pts), _dptr(mean), _dptr(chol), _stream(stream)))
        return mean, chol

    def sample_elements(self, X, off, pts, mean, chol, mult, seed, counter, out=None, stream=None, counter_dev=None,
                        cluster=None, shift=None, ams=None, delta=2.0):
        """Candidates [S][len(pts)][2][3] drawn from the elements' joint
        distributions; with ``cluster`` [S] int32 the distributions are per
        cluster ([C][F][...]) and solution s uses cluster[s]; ``shift``, ``ams``
        and ``delta`` as for sample_estimated."""
        torch = _torch()
        S, F = X.shape[0], off.shape[0] - 1
        _check_shift(shift, ams, S, self.P)
        if out is None:
            out = torch.empty((S, pts.shape[0], 2, 3), dtype=torch.float32, device=X.device)
        nc = max(1, mean.numel() // max(1, 24 * F))
        _check_dist(mean, chol, mult, cluster, S, nc * F, 24, 300)
        _check(lib().dsm_sample_elements(self._h, S, _dptr(X), F, _dptr(off), _dptr(pts), _dptr(mean), _dptr(chol),
                                         _dptr(mult), nc, _dptr(cluster), _dptr(shift), _dptr(ams), float(delta),
                                         int(seed), int(counter), _dptr(counter_dev), _dptr(out), _stream(stream)))
        return out

    def copy_from_donor(self, X, pts, donor, cand, stream=None):
        """Forced improvements: candidates cand [S][len(pts)][2][3] of the
        solutions with donor[s] >= 0 (int32 [S]) become the donor's current
        coordinates at pts (in place); returns cand."""
        torch = _torch()
        S, n = X.shape[0], pts.shape[0]
        if donor.dtype != torch.int32 or donor.numel() != S or pts.dtype != torch.int32 or cand.numel() != S * n * 6:
            raise ValueError("copy_from_donor: donor int32 [S], pts int32 [n], cand [S][n][2][3] expected")
        _check(lib().dsm_copy_from_donor(self._h, S, _dptr(X), n, _dptr(pts), _dptr(donor), _dptr(cand),
                                         _stream(stream)))
        return cand

    def forced_replace(self, X, obj, cache, donor, improved, nis, n_replaced=None, work=None, stream=None):
        """Forced-improvement replacement in place (``dsm_forced_replace``);
        work is allocated here if not given (pass it to allocate nothing)."""
        torch = _torch()
        S = X.shape[0]
        if (donor.dtype != torch.int32 or donor.numel() != S or improved.dtype != torch.uint8 or improved.numel() != S
                or nis.dtype != torch.int32 or nis.numel() != S or obj.dtype != torch.float64
                or cache.dtype != torch.float64 or cache.numel() != S * self.T * 3 or X.numel() != S * 6 * self.P):
            raise ValueError("forced_replace: argument shapes or dtypes")
        if work is None:
            work = torch.empty(lib().dsm_forced_work_bytes(self._h, S), dtype=torch.uint8, device=X.device)
        _check(lib().dsm_forced_replace(self._h, S, _dptr(X), _dptr(obj), _dptr(cache), _dptr(donor), _dptr(improved),
                                        _dptr(nis), _dptr(work), _dptr(n_replaced), _stream(stream)))

    def accept_elements(self, X, off, pts, cand, part_old, part_new, flags, terms_cand, terms_cache, obj, archive=None,
                        accepted=None, stream=None, single_objective=None):
        """accept for elements of several points (CSR off [F+1], pts), candidates
        in the partial-evaluation layout [S][off[F]][2][3]."""
        na = 0 if archive is None else archive.shape[0]
        _check_single_objective(single_objective, X.shape[0])
        _check(lib().dsm_accept_elements(self._h, X.shape[0], _dptr(X), off.shape[0] - 1, _dptr(off), _dptr(pts),
                                         _dptr(cand), _dptr(part_old), _dptr(part_new), _dptr(flags),
                                         _dptr(terms_cand), _dptr(terms_cache), _dptr(obj), na, _dptr(archive),
                                         _dptr(single_objective), _dptr(accepted), _stream(stream)))

    @property
    def pitch(self):
        """Row pitch (elements) of the device image layout."""
        info = ProblemInfo()
        _check(lib().dsm_problem_query(self._h, C.byref(info)))
        return int(info.pitch)

    def set_pitch(self, pitch):
        """Re-packs the device images with row pitch `pitch` (0 = default); synchronises."""
        _check(lib().dsm_problem_set_pitch(self._h, int(pitch)))

    def autotune_pitch(self, X, fos_off, fos_pts, cand, tet_terms_in=None, pitches=None):
        """Times the partial evaluation for each candidate pitch and keeps the
        fastest; returns (best pitch, {pitch: ms})."""
        S, F = X.shape[0], fos_off.shape[0] - 1
        pl = np.ascontiguousarray(pitches if pitches is not None else [], dtype=np.int32)
        n = len(pl) if pitches is not None else 6
        ms = np.zeros(n, np.float32)
        best = C.c_int32()
        _check(lib().dsm_autotune_pitch(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                        _dptr(tet_terms_in), len(pl) if pitches is not None else 0,
                                        _np_ptr(pl), _np_ptr(ms), C.byref(best)))
        if pitches is None:
            pl = self._default_pitch_candidates()
        return int(best.value), {int(p): float(t) for p, t in zip(pl, ms)}

    @property
    def part_chunk(self):
        """Affected tetrahedra per workgroup of a partial evaluation."""
        return int(lib().dsm_get_part_chunk(self._h))

    def set_part_chunk(self, chunk):
        """Sets the affected tetrahedra per workgroup of later partial evaluations (4..8)."""
        _check(lib().dsm_set_part_chunk(self._h, int(chunk)))

    def autotune_chunk(self, X, fos_off, fos_pts, cand, tet_terms_in=None, chunks=None):
        """Times the partial evaluation for each candidate chunk and keeps the
        fastest; returns (best chunk, {chunk: ms})."""
        S, F = X.shape[0], fos_off.shape[0] - 1
        cl = np.ascontiguousarray(chunks if chunks is not None else [], dtype=np.int32)
        n = len(cl) if chunks is not None else 5
        ms = np.zeros(n, np.float32)
        best = C.c_int32()
        _check(lib().dsm_autotune_chunk(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                        _dptr(tet_terms_in), len(cl) if chunks is not None else 0,
                                        _np_ptr(cl), _np_ptr(ms), C.byref(best)))
        if chunks is None:
            cl = list(range(4, 9))
        return int(best.value), {int(c): float(t) for c, t in zip(cl, ms)}

    ROWS_BY_SLICE, ROWS_BY_SLICE_PAIR = 0, 1

    @property
    def row_order(self):
        """Row order of the sweep: ROWS_BY_SLICE (0) or ROWS_BY_SLICE_PAIR (1)."""
        return int(lib().dsm_get_row_order(self._h))

    def set_row_order(self, order):
        """Sets the row order of later evaluations (0 by slice, 1 by slice pair)."""
        _check(lib().dsm_set_row_order(self._h, int(order)))

    def autotune_row_order(self, X, fos_off, fos_pts, cand, tet_terms_in=None):
        """Times the partial evaluation with each row order and keeps the
        faster; returns (best order, {order: ms})."""
        S, F = X.shape[0], fos_off.shape[0] - 1
        ms = np.zeros(2, np.float32)
        best = C.c_int32()
        _check(lib().dsm_autotune_row_order(self._h, S, _dptr(X), F, _dptr(fos_off), _dptr(fos_pts), _dptr(cand),
                                            _dptr(tet_terms_in), _np_ptr(ms), C.byref(best)))
        return int(best.value), {0: float(ms[0]), 1: float(ms[1])}

    def _default_pitch_candidates(self):
        Dx = self.dims[0]
        d0 = Dx + 2 + ((8 - (Dx + 2) % 16) + 16) % 16
        return [d0 + k for k in (0, 4, 8, 16, 24, 56)]

    def timing(self, capacity):
        """Record the sweep kernel's duration in the next `capacity` evaluation calls."""
        _check(lib().dsm_problem_timing(self._h, int(capacity)))

    def timing_read(self, max_n=4096):
        ms = np.zeros(max_n, np.float32)
        n = C.c_int32()
        _check(lib().dsm_problem_timing_read(self._h, _np_ptr(ms), int(max_n), C.byref(n)))
        return ms[:n.value].astype(np.float64)

    def transform(self, X2, own=1, dvf=True, warped=True, stream=None):
        """(dvf [Dz][Dy][Dx][3] or None, warped [Dz][Dy][Dx] or None) of one
        solution X2 [2][P][3] f32 on the device (``dsm_transform``)."""
        torch = _torch()
        Dx, Dy, Dz = self.dims
        d = torch.empty((Dz, Dy, Dx, 3), dtype=torch.float32, device=X2.device) if dvf else None
        w = torch.empty((Dz, Dy, Dx), dtype=torch.float32, device=X2.device) if warped else None
        _check(lib().dsm_transform(self._h, int(own), _dptr(X2), _dptr(d) if d is not None else None,
                                   _dptr(w) if w is not None else None, _stream(stream)))
        return d, w

    def rasterize_owner(self, Xgrid, stream=None):
        torch = _torch()
        Dx, Dy, Dz = self.dims
        owner = torch.empty((Dz, Dy, Dx), dtype=torch.int32, device=Xgrid.device)
        overlap = torch.empty(1, dtype=torch.int32, device=Xgrid.device)
        _check(lib().dsm_rasterize_owner(self._h, _dptr(Xgrid), _dptr(owner), _dptr(overlap), _stream(stream)))
        return owner, overlap


SUR_FEATURES, SUR_OUTPUTS, SUR_NPARAMS = 192, 3, 43280


def _scheck(st):
    if st != OK:
        L = lib()
        raise DsmError(st, f"{L.dsm_status_string(st).decode()}: {L.dsm_surrogate_last_error().decode()}")


class Surrogate:
    """Candidate-screening MLP on the current GPU (``dsm_surrogate``)."""

    def __init__(self, seed=0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, max_rows=1 << 16, max_batch=4096):
        d = SurrogateDesc(seed=seed, lr=lr, beta1=beta1, beta2=beta2, eps=eps, max_rows=max_rows, max_batch=max_batch)
        h = C.c_void_p()
        _scheck(lib().dsm_surrogate_create(C.byref(d), C.byref(h)))
        self._h = h
        self.max_rows, self.max_batch = max_rows, max_batch

    def close(self):
        if getattr(self, "_h", None):
            lib().dsm_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, new=None):
        if new is not None:
            a = np.ascontiguousarray(new, dtype=np.float32)
            assert a.size == SUR_NPARAMS
            _scheck(lib().dsm_surrogate_params(self._h, _np_ptr(a), 1))
            return a
        a = np.zeros(SUR_NPARAMS, np.float32)
        _scheck(lib().dsm_surrogate_params(self._h, _np_ptr(a), 0))
        return a

    def fit_scaling(self, feats, deltas, stream=None):
        _scheck(lib().dsm_surrogate_fit_scaling(self._h, feats.shape[0], _dptr(feats), _dptr(deltas), _stream(stream)))

    def scaling(self):
        im, ir = np.zeros(SUR_FEATURES, np.float32), np.zeros(SUR_FEATURES, np.float32)
        om, orr = np.zeros(SUR_OUTPUTS, np.float32), np.zeros(SUR_OUTPUTS, np.float32)
        _scheck(lib().dsm_surrogate_get_scaling(self._h, _np_ptr(im), _np_ptr(ir), _np_ptr(om), _np_ptr(orr)))
        return im, ir, om, orr

    def set_scaling(self, in_mean, in_rstd, out_mean, out_rstd):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (in_mean, in_rstd, out_mean, out_rstd)]
        _scheck(lib().dsm_surrogate_set_scaling(self._h, *[_np_ptr(a) for a in arrs]))

    @staticmethod
    def features(problem, X, pts, cand, stream=None):
        """Raw features [S*F*K][192] of candidates cand [S][F][K][2][3]."""
        torch = _torch()
        S, F, K = cand.shape[:3]
        out = torch.empty((S * F * K, SUR_FEATURES), dtype=torch.float32, device=X.device)
        _scheck(lib().dsm_surrogate_features(problem._h, S, _dptr(X), F, _dptr(pts), K, _dptr(cand), _dptr(out),
                                             _stream(stream)))
        return out

    def features_packed(self, problem, X, pts, cand, stream=None):
        """Standardised BF16 feature rows (as int16) [S*F*K][192] of candidates
        cand [S][F][K][2][3], computed and packed in one kernel."""
        torch = _torch()
        S, F, K = cand.shape[:3]
        out = torch.empty((S * F * K, SUR_FEATURES), dtype=torch.int16, device=X.device)
        _scheck(lib().dsm_surrogate_features_packed(self._h, problem._h, S, _dptr(X), F, _dptr(pts), K, _dptr(cand),
                                                    _dptr(out), _stream(stream)))
        return out

    def pack(self, feats=None, part_old=None, part_new=None, stream=None):
        """(bf16 feature rows as int16, standardised targets, raw deltas)."""
        torch = _torch()
        N = feats.shape[0] if feats is not None else part_old.shape[0]
        dev = (feats if feats is not None else part_old).device
        fb = torch.empty((N, SUR_FEATURES), dtype=torch.int16, device=dev) if feats is not None else None
        tg = torch.empty((N, SUR_OUTPUTS), dtype=torch.float32, device=dev) if part_old is not None else None
        raw = torch.empty((N, SUR_OUTPUTS), dtype=torch.float32, device=dev) if part_old is not None else None
        _scheck(lib().dsm_surrogate_pack(self._h, N, _dptr(feats), _dptr(fb), _dptr(part_old), _dptr(part_new),
                                         _dptr(tg), _dptr(raw), _stream(stream)))
        return fb, tg, raw

    def forward(self, feats_bf16, stream=None):
        torch = _torch()
        N = feats_bf16.shape[0]
        out = torch.empty((N, SUR_OUTPUTS), dtype=torch.float32, device=feats_bf16.device)
        _scheck(lib().dsm_surrogate_forward(self._h, N, _dptr(feats_bf16), _dptr(out), _stream(stream)))
        return out

    def gradient(self, feats_bf16, targets, stream=None):
        torch = _torch()
        g = torch.empty(SUR_NPARAMS, dtype=torch.float32, device=targets.device)
        loss = torch.empty(1, dtype=torch.float32, device=targets.device)
        _scheck(lib().dsm_surrogate_gradient(self._h, feats_bf16.shape[0], _dptr(feats_bf16), _dptr(targets), _dptr(g),
                                             _dptr(loss), _stream(stream)))
        return g, loss

    def train(self, feats_bf16, targets, steps, batch, stream=None):
        torch = _torch()
        loss = torch.empty(max(steps, 1), dtype=torch.float32, device=targets.device)
        _scheck(lib().dsm_surrogate_train(self._h, feats_bf16.shape[0], _dptr(feats_bf16), _dptr(targets), int(steps),
                                          int(batch), _dptr(loss), _stream(stream)))
        return loss[:steps]

    def screen(self, problem, X, pts, cand, obj=None, archive=None, stream=None):
        """(pick [S][F], run_exact [S][F] uint8, raw predictions [S][F][K][3], picked candidates [S][F][2][3])."""
        torch = _torch()
        S, F, K = cand.shape[:3]
        pred = torch.empty((S, F, K, SUR_OUTPUTS), dtype=torch.float32, device=X.device)
        pick = torch.empty((S, F), dtype=torch.int32, device=X.device)
        run = torch.empty((S, F), dtype=torch.uint8, device=X.device)
        cp = torch.empty((S, F, 2, 3), dtype=torch.float32, device=X.device)
        na = 0 if archive is None else archive.shape[0]
        _scheck(lib().dsm_surrogate_screen(self._h, problem._h, S, _dptr(X), F, _dptr(pts), K, _dptr(cand), _dptr(obj),
                                           na, _dptr(archive), _dptr(pred), _dptr(pick), _dptr(run), _dptr(cp),
                                           _stream(stream)))
        return pick, run, pred, cp


class Batch:
    """Partial evaluation of several problems in one fused launch (``dsm_batch``)."""

    def __init__(self, max_jobs=16):
        h = C.c_void_p()
        _check(lib().dsm_batch_create(int(max_jobs), C.byref(h)))
        self._h = h
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            lib().dsm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_jobs(self, jobs):
        """Stores a configuration for run() (dsm_batch_set_jobs; synchronises the
        device): jobs as for eval_partial; returns the output tensors
        (part_old, part_new, flags, voxel_count) per job, which every run()
        overwrites.  The job tensors must stay alive and keep their storage."""
        arr, outs = self._table(jobs)
        self._set_keep = (arr, jobs, outs)
        _check(lib().dsm_batch_set_jobs(self._h, len(jobs), arr))
        return outs

    def run(self, stream=None):
        """Enqueues the stored configuration (dsm_batch_run): capture-safe."""
        _check(lib().dsm_batch_run(self._h, _stream(stream)))

    def _table(self, jobs):
        torch = _torch()
        arr = (PartialJob * len(jobs))()
        outs = []
        for j, d in enumerate(jobs):
            X = d["X"]
            S, F = X.shape[0], d["fos_off"].shape[0] - 1
            o = (torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                 torch.empty((S, F, 3), dtype=torch.float64, device=X.device),
                 torch.empty((S, F), dtype=torch.int32, device=X.device),
                 torch.empty((S, F), dtype=torch.int32, device=X.device))
            outs.append(o)
            arr[j] = PartialJob(d["problem"]._h.value, S, X.data_ptr(), F, d["fos_off"].data_ptr(),
                                d["fos_pts"].data_ptr(), d["cand"].data_ptr(),
                                d["mask"].data_ptr() if d.get("mask") is not None else None,
                                d["tet_terms_in"].data_ptr() if d.get("tet_terms_in") is not None else None,
                                o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), None, o[3].data_ptr())
        return arr, outs

    def eval_partial(self, jobs, stream=None):
        """jobs: list of dicts (problem, X, fos_off, fos_pts, cand, [tet_terms_in, mask]); returns a list of
        (part_old, part_new, flags, voxel_count) per job."""
        arr, outs = self._table(jobs)
        self._keep = (arr, jobs, outs)
        _check(lib().dsm_eval_partial_batch(self._h, len(jobs), arr, _stream(stream)))
        return outs
