"""ctypes binding of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product library never does.  It
shares no code with the GPU library (it does not import the package).

Every function takes and returns host numpy arrays.  Grid 0 is the source
("moving") grid on the source image, grid 1 the target ("fixed") grid on the
target image; coordinates are float32 voxel units on the 1/128-voxel lattice.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.environ.get("DSM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

FLAG_INV_MOVING = 1
FLAG_INV_FIXED = 2
FLAG_BORDER = 4
FLAG_DOMAIN = 8
FLAG_LATTICE = 16
FLAG_NONFINITE = 32


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.ref_create.restype = P
        L.ref_create.argtypes = [P, P, P, P, P, C.c_double, C.c_int, P, P, C.c_int, P, P, C.c_int, C.c_int]
        L.ref_destroy.argtypes = [P]
        for name, args in {
            "ref_counts": [P, P], "ref_tets": [P, P], "ref_edges": [P, P, P], "ref_star": [P, P, P],
            "ref_identity": [P, P], "ref_owner_bruteforce": [P, P, P, P],
            "ref_fold_check": [P, C.c_int, P, P, P],
            "ref_eval_full": [P, C.c_int, P, P, P, P, P],
            "ref_eval_partial": [P, C.c_int, P, C.c_int, P, P, P, P, P, P, P, P],
            "ref_tet_terms": [P, P, C.c_int, P], "ref_normalisers": [P, P],
        }.items():
            getattr(L, name).argtypes = args
            getattr(L, name).restype = None
        L.ref_orient3d.restype = C.c_double
        L.ref_orient3d.argtypes = [P, P, P, P]
        L.ref_inside.restype = C.c_int
        L.ref_inside.argtypes = [P, P]
        L.ref_tet_voxels.restype = C.c_int
        L.ref_tet_voxels.argtypes = [P, P, C.c_int, P, C.c_int]
        L.ref_trilinear.restype = C.c_double
        L.ref_trilinear.argtypes = [P, C.c_int, P, C.c_int]
        L.ref_refine.restype = None
        L.ref_refine.argtypes = [P, C.c_int, P, P]
        L.ref_transform.restype = None
        L.ref_transform.argtypes = [P, C.c_int, P, P, P]
        L.ref_literal_fold_check.restype = None
        L.ref_literal_fold_check.argtypes = [P, C.c_int, P, P]
        L.ref_set_threads.restype = None
        L.ref_set_threads.argtypes = [C.c_int]
        L.ref_max_threads.restype = C.c_int
        L.ref_max_threads.argtypes = []
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def refine(mesh_coarse, Xc):
    """Sec. 2.4 grid refinement of a population Xc [S][2][Pc][3] on a mesh of
    mesh_coarse points per axis -> [S][2][Pf][3] on 2n-1 points per axis."""
    nc = np.ascontiguousarray(mesh_coarse, dtype=np.int32)
    Xc = np.ascontiguousarray(Xc, dtype=np.float32)
    S = Xc.shape[0]
    Pf = int(np.prod(2 * nc - 1))
    Xf = np.zeros((S, 2, Pf, 3), np.float32)
    lib().ref_refine(_p(nc), S, _p(Xc), _p(Xf))
    return Xf


def orient3d(a, b, c, d) -> float:
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d)]
    return lib().ref_orient3d(*[_p(x) for x in arrs])


def set_threads(n):
    """Threads of the oracle's parallel loops (OpenMP); returns the previous maximum."""
    L = lib()
    prev = L.ref_max_threads()
    L.ref_set_threads(int(n))
    return prev


class Problem:
    """One registration problem: two images of equal dims, two coupled meshes of
    ``mesh`` points per axis, optional guidance point sets."""

    def __init__(self, moving, fixed, mesh, spacing=(1.0, 1.0, 1.0), tau=0.1,
                 guid_moving=None, corr_moving=None, guid_fixed=None, corr_fixed=None,
                 hard_threshold=False, abs_deformation=False):
        moving = np.ascontiguousarray(moving, dtype=np.float32)
        fixed = np.ascontiguousarray(fixed, dtype=np.float32)
        assert moving.shape == fixed.shape and moving.ndim == 3
        self.shape = moving.shape  # (Dz, Dy, Dx)
        self.dims = np.array([moving.shape[2], moving.shape[1], moving.shape[0]], dtype=np.int32)
        self.mesh = np.array(mesh, dtype=np.int32)
        self.spacing = np.array(spacing, dtype=np.float64)
        gm = np.ascontiguousarray(guid_moving if guid_moving is not None else np.zeros((0, 3)), dtype=np.float32)
        gf = np.ascontiguousarray(guid_fixed if guid_fixed is not None else np.zeros((0, 3)), dtype=np.float32)
        cm = np.ascontiguousarray(corr_moving if corr_moving is not None else np.arange(len(gm)), dtype=np.int32)
        cf = np.ascontiguousarray(corr_fixed if corr_fixed is not None else np.arange(len(gf)), dtype=np.int32)
        self._keep = (moving, fixed, gm, gf, cm, cf)
        self._h = lib().ref_create(_p(self.dims), _p(self.spacing), _p(moving), _p(fixed), _p(self.mesh),
                                   float(tau), len(gm), _p(gm), _p(cm), len(gf), _p(gf), _p(cf),
                                   int(hard_threshold), int(abs_deformation))
        cnt = np.zeros(4, dtype=np.int32)
        lib().ref_counts(self._h, _p(cnt))
        self.P, self.T, self.E, self.max_star = (int(x) for x in cnt)
        self.V = int(np.prod(self.dims))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ref_destroy(self._h)
            self._h = None

    # ---- topology
    def tets(self):
        out = np.zeros((self.T, 4), dtype=np.int32)
        lib().ref_tets(self._h, _p(out))
        return out

    def edges(self):
        e = np.zeros((self.E, 2), dtype=np.int32)
        k = np.zeros(self.E, dtype=np.int32)
        lib().ref_edges(self._h, _p(e), _p(k))
        return e, k

    def star(self):
        off = np.zeros(self.P + 1, dtype=np.int32)
        st = np.zeros(4 * self.T, dtype=np.int32)
        lib().ref_star(self._h, _p(off), _p(st))
        return off, st

    def identity(self):
        X = np.zeros((self.P, 3), dtype=np.float32)
        lib().ref_identity(self._h, _p(X))
        return X

    def normalisers(self):
        out = np.zeros(3)
        lib().ref_normalisers(self._h, _p(out))
        return out

    # ---- rasterisation
    def owner_bruteforce(self, Xg):
        Xg = np.ascontiguousarray(Xg, dtype=np.float32)
        owner = np.zeros(self.V, dtype=np.int32)
        count = np.zeros(self.V, dtype=np.int32)
        lib().ref_owner_bruteforce(self._h, _p(Xg), _p(owner), _p(count))
        return owner.reshape(self.shape), count.reshape(self.shape)

    def tet_voxels(self, Xg, t):
        Xg = np.ascontiguousarray(Xg, dtype=np.float32)
        n = lib().ref_tet_voxels(self._h, _p(Xg), int(t), None, 0)
        out = np.zeros(max(n, 1), dtype=np.int64)
        lib().ref_tet_voxels(self._h, _p(Xg), int(t), _p(out), n)
        return out[:n]

    def trilinear(self, grid, x, mask=False):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().ref_trilinear(self._h, int(grid), _p(x), int(mask))

    def transform(self, own, X2):
        """Sec. 2.1 / Fig. 2: (dvf [Dz][Dy][Dx][3], warped [Dz][Dy][Dx]) of one
        solution X2 [2][P][3]: where each voxel of image `own` maps to in the
        other image (displacement in voxel units), and the other image sampled
        there (own = 1: the transformed source on the target grid)."""
        X2 = np.ascontiguousarray(X2, dtype=np.float32)
        dvf = np.zeros((self.V, 3))
        warped = np.zeros(self.V)
        lib().ref_transform(self._h, int(own), _p(X2), _p(dvf), _p(warped))
        return dvf.reshape(self.shape + (3,)), warped.reshape(self.shape)

    # ---- objectives and constraints
    def fold_check(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        S = X.shape[0]
        flags = np.zeros(S, dtype=np.uint32)
        fb = np.zeros(S, dtype=np.int32)
        lib().ref_fold_check(self._h, S, _p(X), _p(flags), _p(fb))
        return flags, fb

    def literal_fold_check(self, X):
        """Sec. 2.3.4 as stated (points inside the surface / polygon of their
        surrounding faces, by ray casting): violating points per [S][grid]."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.zeros((X.shape[0], 2), np.int32)
        lib().ref_literal_fold_check(self._h, X.shape[0], _p(X), _p(out))
        return out

    def eval_full(self, X, want_terms=False):
        X = np.ascontiguousarray(X, dtype=np.float32)
        S = X.shape[0]
        obj = np.zeros((S, 3))
        flags = np.zeros(S, dtype=np.uint32)
        terms = np.zeros((S, self.T, 3)) if want_terms else None
        nvox = np.zeros(S, dtype=np.int64)
        lib().ref_eval_full(self._h, S, _p(X), _p(obj), _p(flags), _p(terms), _p(nvox))
        return (obj, flags, terms, nvox) if want_terms else (obj, flags)

    def eval_partial(self, X, fos_off, fos_pts, cand, tet_terms=None):
        X = np.ascontiguousarray(X, dtype=np.float32)
        fos_off = np.ascontiguousarray(fos_off, dtype=np.int32)
        fos_pts = np.ascontiguousarray(fos_pts, dtype=np.int32)
        cand = np.ascontiguousarray(cand, dtype=np.float32)
        S, F = X.shape[0], len(fos_off) - 1
        assert cand.shape == (S, int(fos_off[-1]), 2, 3)
        tt = np.ascontiguousarray(tet_terms, dtype=np.float64) if tet_terms is not None else None
        old = np.zeros((S, F, 3))
        new = np.zeros((S, F, 3))
        flags = np.zeros((S, F), dtype=np.uint32)
        nvox = np.zeros((S, F), dtype=np.int64)
        lib().ref_eval_partial(self._h, S, _p(X), F, _p(fos_off), _p(fos_pts), _p(cand), _p(tt),
                               _p(old), _p(new), _p(flags), _p(nvox))
        return old, new, flags, nvox

    def tet_terms(self, X2, t):
        X2 = np.ascontiguousarray(X2, dtype=np.float32)
        out = np.zeros(3)
        lib().ref_tet_terms(self._h, _p(X2), int(t), _p(out))
        return out
