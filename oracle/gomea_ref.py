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


# --------------------------------------------------------------------- clustering
#
# The paper builds on MO-RV-GOMEA (Sec. 2.2), which clusters the selected
# solutions in objective space each generation and estimates one distribution
# per cluster and FOS element; every solution draws from the cluster nearest
# to it.  The clustering is balanced k-leader-means, read here as:
#   1. objectives normalised per objective to [0, 1] over the selection (a zero
#      range divides by 1);
#   2. k leaders by farthest-first traversal: the first is the selected solution
#      with the largest normalised first objective, each next one the selected
#      solution farthest (squared Euclidean distance) from its nearest leader;
#   3. k-means from the leaders: assign every selected solution to its nearest
#      mean, recompute each mean as the average of its solutions (kept if none),
#      until no assignment changes (at most 50 rounds);
#   4. cluster j = the c = min(n, ceil(2 n / k)) selected solutions nearest to
#      mean j, nearest first (clusters may overlap);
#   5. every population member is assigned to the nearest mean.
# Ties go to the lower selection position / cluster index.  Sums run in
# selection order, one addition at a time, so that a parallel implementation
# that keeps this order reproduces every bit.

MAX_CLUSTERS = 16
MAX_CLUSTER_SELECTION = 1024


def _d2(a, b):
    d0, d1, d2 = a[0] - b[0], a[1] - b[1], a[2] - b[2]
    return d0 * d0 + d1 * d1 + d2 * d2


def cluster(obj, sel, k):
    """(members [k][c] selection indices into the population, assign [S],
    means [k][3] normalised) for objectives obj [S][3] and selection sel
    (indices outside [0, S) dropped).  With fewer than k valid selected
    solutions every output is -1 (means NaN)."""
    obj = np.asarray(obj, dtype=np.float64)
    S = obj.shape[0]
    idx = [int(s) for s in sel if 0 <= s < S]
    n = len(idx)
    c = min(n, -(-2 * n // k)) if k > 0 else 0
    if k < 1 or n < k:
        return np.full((max(k, 0), max(c, 0)), -1, np.int32), np.full(S, -1, np.int32), np.full((max(k, 0), 3), np.nan)
    lo = [min(obj[s, o] for s in idx) for o in range(3)]
    hi = [max(obj[s, o] for s in idx) for o in range(3)]
    rng = [hi[o] - lo[o] if hi[o] - lo[o] > 0 else 1.0 for o in range(3)]
    norm = lambda s: [(obj[s, o] - lo[o]) / rng[o] for o in range(3)]
    Y = [norm(s) for s in idx]
    # farthest-first leaders
    first = 0
    for i in range(1, n):
        if Y[i][0] > Y[first][0]:
            first = i
    leaders = [first]
    near = [_d2(Y[i], Y[first]) for i in range(n)]
    while len(leaders) < k:
        far = 0
        for i in range(1, n):
            if near[i] > near[far]:
                far = i
        leaders.append(far)
        near = [min(near[i], _d2(Y[i], Y[far])) for i in range(n)]
    means = [list(Y[l]) for l in leaders]

    def nearest(y):
        best, bd = 0, _d2(y, means[0])
        for j in range(1, k):
            d = _d2(y, means[j])
            if d < bd:
                best, bd = j, d
        return best

    lab = [-1] * n
    for _ in range(50):
        new = [nearest(Y[i]) for i in range(n)]
        if new == lab:
            break
        lab = new
        for j in range(k):
            acc, cnt = [0.0, 0.0, 0.0], 0
            for i in range(n):
                if lab[i] == j:
                    for o in range(3):
                        acc[o] += Y[i][o]
                    cnt += 1
            if cnt:
                means[j] = [acc[o] / cnt for o in range(3)]
    members = np.zeros((k, c), np.int32)
    for j in range(k):
        d = [_d2(Y[i], means[j]) for i in range(n)]
        order = sorted(range(n), key=lambda i: (d[i], i))
        members[j] = [idx[i] for i in order[:c]]
    assign = np.array([nearest(norm(s)) for s in range(S)], np.int32)
    return members, assign, np.array(means)


def cluster_size(n_sel, k):
    """Members per cluster, c = min(n, ceil(2 n / k))."""
    return min(n_sel, -(-2 * n_sel // k))


# --------------------------------------------------------------------- variance scaling
#
# AMaLGaM's adaptive variance scaling, as used by RV-GOMEA: after a generation,
# the standard-deviation ratio of a distribution is the largest, over its
# variables, distance between the mean of the improving (accepted) samples and
# the distribution mean, in units of that variable's standard deviation.

def standard_deviation_ratio(samples, mean, cov):
    """Largest |mean(samples)_v - mean_v| / sqrt(cov_vv) over variables with
    positive variance; -1 for no sample.  samples [n][V], mean [V], cov [V][V]."""
    samples = np.asarray(samples, dtype=np.float64).reshape(-1, len(mean))
    if len(samples) == 0:
        return -1.0
    d = np.abs(samples.mean(axis=0) - np.asarray(mean, dtype=np.float64))
    var = np.diag(np.asarray(cov, dtype=np.float64))
    ok = var > 0
    return float((d[ok] / np.sqrt(var[ok])).max()) if ok.any() else 0.0
