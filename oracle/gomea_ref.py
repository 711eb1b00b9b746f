"""FP64 reference of the distribution estimation used for RV-GOMEA-style
partial changes of single-point elements.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).  Shares no
code with the GPU library.

RV-GOMEA, on which the paper's optimisation (Sec. 2.2) builds, draws the
variables of a FOS element from a normal distribution estimated on selected
solutions.  For a single grid point the variables are its 6 coordinates
(source x y z, target x y z); coordinates of border points pinned to the box
(grid index 0 or n-1 on that axis) are not variables.  The estimate is the
sample mean and the maximum-likelihood covariance (divisor n) of the free
coordinates; the sampler uses the lower Cholesky factor, computed here from its
definition (L L^T = C, L lower triangular with a non-negative diagonal), with a
zero column where the pivot is not positive (rank-deficient selections).
"""
from __future__ import annotations

import numpy as np


def free_axes(p, mesh):
    """Bool [6]: which of point p's 6 coordinates are variables (not pinned)."""
    nx, ny, nz = (int(n) for n in mesh)
    idx = (p % nx, (p // nx) % ny, p // (nx * ny))
    n = (nx, ny, nz)
    return np.array([0 < idx[c % 3] < n[c % 3] - 1 for c in range(6)])


def coordinates(X, sel, p):
    """[n][6] coordinates of point p in the solutions sel of X [S][2][P][3]
    (indices outside [0, S) skipped)."""
    S = X.shape[0]
    rows = [np.concatenate([X[s, 0, p], X[s, 1, p]]).astype(np.float64) for s in sel if 0 <= s < S]
    return np.array(rows).reshape(-1, 6)


def cholesky_semidefinite(C):
    """Lower L with L L^T = C for symmetric positive semi-definite C; a column
    whose pivot is not positive is set to zero."""
    n = C.shape[0]
    L = np.zeros_like(C)
    for r in range(n):
        for c in range(r + 1):
            v = C[r, c] - sum(L[r, t] * L[c, t] for t in range(c))
            if c == r:
                L[r, r] = np.sqrt(v) if v > 0.0 else 0.0
            else:
                L[r, c] = v / L[c, c] if L[c, c] > 0.0 else 0.0
    return L


def estimate(X, sel, pts, mesh):
    """(mean [F][6], covariance [F][6][6], Cholesky factor [F][6][6]) for the
    single points pts over the solutions sel of X."""
    F = len(pts)
    mean = np.zeros((F, 6))
    cov = np.zeros((F, 6, 6))
    chol = np.zeros((F, 6, 6))
    for f, p in enumerate(pts):
        P = X.shape[2]
        if not 0 <= p < P:
            continue
        x = coordinates(X, sel, p)
        if len(x) == 0:
            continue
        m = x.mean(axis=0)
        d = (x - m) * free_axes(p, mesh)
        C = d.T @ d / len(x)
        mean[f], cov[f], chol[f] = m, C, cholesky_semidefinite(C)
    return mean, cov, chol


def packed_lower(L):
    """The entries of a lower-triangular n x n matrix, row r holding columns
    0..r (21 for n = 6, 300 for n = 24)."""
    return np.concatenate([L[r, :r + 1] for r in range(L.shape[0])])


MAX_POINTS = 4
MAX_VARS = 6 * MAX_POINTS


def estimate_elements(X, sel, off, pts, mesh):
    """Joint distributions of elements of up to 4 points (CSR off, pts): the
    variables of element f are its points' coordinates in order, 6 per point.
    Returns (mean [F][24], covariance [F][24][24], Cholesky factor [F][24][24]),
    zero for variables beyond 6 x (number of points), for pinned coordinates,
    and for elements with no point, more than 4, or an invalid point."""
    F = len(off) - 1
    P = X.shape[2]
    mean = np.zeros((F, MAX_VARS))
    cov = np.zeros((F, MAX_VARS, MAX_VARS))
    chol = np.zeros((F, MAX_VARS, MAX_VARS))
    for f in range(F):
        ps = list(pts[off[f]:off[f + 1]])
        if not 1 <= len(ps) <= MAX_POINTS or any(not 0 <= p < P for p in ps):
            continue
        xs = [coordinates(X, sel, p) for p in ps]
        if len(xs[0]) == 0:
            continue
        x = np.concatenate(xs, axis=1)  # [n][6 * len(ps)]
        free = np.concatenate([free_axes(p, mesh) for p in ps])
        nv = x.shape[1]
        m = x.mean(axis=0)
        d = (x - m) * free
        C = d.T @ d / len(x)
        mean[f, :nv], cov[f, :nv, :nv], chol[f, :nv, :nv] = m, C, cholesky_semidefinite(C)
    return mean, cov, chol
