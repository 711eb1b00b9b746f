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


# ---------------------------------------------------------------------------
# Generation bookkeeping of the multi-objective optimiser (Sec. 2.2, Sec. 2.4)
# written from the definitions, one solution at a time.

def dominates(a, b):
    """a Pareto-dominates b (minimisation): no worse in every objective, better in one."""
    return all(x <= y for x, y in zip(a, b)) and any(x < y for x, y in zip(a, b))


def archive_merge(archive, points, archive_rows=None, point_rows=None):
    """The elitist archive (the approximation set of Sec. 2.4) after adding
    `points`: of archive rows then points, in that order, a vector is kept iff
    no vector of either dominates it and no earlier vector equals it; the kept
    vectors are returned in lexicographic order, with their payload rows (e.g.
    solutions) if given.  Returns (vectors [k][3], rows [k][...] or None)."""
    vecs = [tuple(float(v) for v in r) for r in np.asarray(archive, np.float64).reshape(-1, 3)]
    vecs += [tuple(float(v) for v in r) for r in np.asarray(points, np.float64).reshape(-1, 3)]
    rows = None
    if archive_rows is not None:
        rows = list(np.asarray(archive_rows)) + list(np.asarray(point_rows))
    kept = []
    for i, v in enumerate(vecs):
        if any(dominates(u, v) for u in vecs):
            continue
        if any(vecs[j] == v for j in range(i)):
            continue
        kept.append(i)
    kept.sort(key=lambda i: vecs[i])  # tuples compare lexicographically
    out = np.array([vecs[i] for i in kept], np.float64).reshape(-1, 3)
    return out, (None if rows is None else np.array([rows[i] for i in kept]))


def select(obj, n_sel):
    """Selection: the n_sel solutions with the fewest population members
    dominating them; ties by the smallest sum, in objective order, of the
    objectives normalised to the population's range (divisor at least 1e-300),
    then by index.  Returns (indices [n_sel], dominated-by counts [S])."""
    obj = np.asarray(obj, np.float64)
    S = len(obj)
    count = np.array([sum(1 for j in range(S) if dominates(obj[j], obj[i])) for i in range(S)])
    lo = [min(obj[:, c]) for c in range(3)]
    hi = [max(obj[:, c]) for c in range(3)]
    key = []
    for i in range(S):
        nrm = 0.0
        for c in range(3):
            nrm = nrm + (obj[i, c] - lo[c]) / max(hi[c] - lo[c], 1e-300)
        key.append((count[i] * 4.0 + nrm, i))
    order = [i for _, i in sorted(key)]
    return np.array(order[:n_sel], np.int64), count


def avs_update(mult, nis, sdr, nis_max, eta=0.9, lo=0.05, hi=10.0):
    """AMaLGaM's adaptive variance scaling step per distribution, in float32:
    after an improvement (sdr >= 0) the multiplier is at least 1 and is divided
    by eta if sdr > 1, and the no-improvement stretch restarts; without one the
    stretch grows while the multiplier is at most 1, the multiplier is
    multiplied by eta if it is above 1 or the stretch reached nis_max, and is
    reset to 1 if it fell below 1 while the stretch is short; the result is
    clamped to [lo, hi].  Returns (mult float32, nis int32)."""
    f32 = np.float32
    out_c = np.zeros(len(mult), np.float32)
    out_n = np.zeros(len(mult), np.int32)
    for i, (c, n, r) in enumerate(zip(np.asarray(mult, np.float32), np.asarray(nis), np.asarray(sdr, np.float64))):
        c = f32(c)
        if r >= 0:
            c1 = f32(1.0) if c < 1 else c
            if r > 1:
                c1 = f32(c1 / f32(eta))
            n1 = 0
        else:
            n1 = int(n) + 1 if c <= 1 else int(n)
            c1 = c
            if c > 1 or n1 >= nis_max:
                c1 = f32(c * f32(eta))
            if c1 < 1 and n1 < nis_max:
                c1 = f32(1.0)
        out_c[i] = min(max(c1, f32(lo)), f32(hi))
        out_n[i] = n1
    return out_c, out_n


def forced_replace(X, obj, cache, donor, improved, nis):
    """Forced improvements at the end of a generation: the no-improvement
    stretch of a solution restarts if it accepted a change and grows otherwise;
    a solution that had a donor (donor >= 0) and accepted nothing takes the
    donor's coordinates, objectives and per-tetrahedron terms as they were
    before this step; every solution that had a donor restarts its stretch.
    Returns new (X, obj, cache, nis, number replaced)."""
    X2, obj2, cache2, nis2 = X.copy(), obj.copy(), cache.copy(), np.asarray(nis).copy()
    replaced = 0
    for s in range(len(X)):
        nis2[s] = 0 if improved[s] else nis2[s] + 1
        d = int(donor[s])
        if d >= 0:
            if not improved[s]:
                X2[s], obj2[s], cache2[s] = X[d], obj[d], cache[d]
                replaced += 1
            nis2[s] = 0
    return X2, obj2, cache2, nis2, replaced


def multiplier_step(accepted, mult, cluster=None, eta=0.9, lo=0.05, hi=10.0):
    """The simple multiplier schedule, float32: for each cluster j and element
    f the multiplier is divided by eta (at most hi) if a solution of cluster j
    (every solution without clusters) had element f accepted, else multiplied
    by eta (at least lo)."""
    acc = np.asarray(accepted)
    out = np.asarray(mult, np.float32).copy()
    k, F = out.shape
    for j in range(k):
        for f in range(F):
            hit = any(acc[s, f] and (cluster is None or cluster[s] == j) for s in range(acc.shape[0]))
            c = np.float32(out[j, f])
            out[j, f] = min(np.float32(c / np.float32(eta)), np.float32(hi)) if hit else \
                max(np.float32(c * np.float32(eta)), np.float32(lo))
    return out


def ams_shift(mean, prev):
    """RV-GOMEA's anticipated mean shift: the change of the selection's mean of
    every variable since the previous generation (mean - prev)."""
    return np.asarray(mean, np.float64) - np.asarray(prev, np.float64)


def single_objective_clusters(means, assign):
    """MO-RV-GOMEA's single-objective clusters: objective o = 0, 1, 2 (while
    o < k) takes, of the k clusters not yet taken, the one whose mean in o is
    lowest (the lowest index among equal means); returns, for every solution,
    the objective of its cluster assign[s], or -1 if that cluster has none."""
    means = np.asarray(means, np.float64)
    k = len(means)
    of_cluster = [-1] * k
    for o in range(min(3, k)):
        best = None
        for j in range(k):
            if of_cluster[j] < 0 and (best is None or means[j, o] < means[best, o]):
                best = j
        of_cluster[best] = o
    return np.array([of_cluster[a] if 0 <= a < k else -1 for a in assign], np.int32)


def draw_donors(nis, nis_max, dominated_by, u):
    """RV-GOMEA's forced-improvement donors: a solution whose no-improvement
    stretch exceeds nis_max gets a donor drawn from the solutions no member
    dominates, taken in ascending order: entry min(floor(u[s] n), n - 1) of the
    n of them, with the caller's uniform draw u[s] in [0, 1) (the product in
    float32); the others get -1."""
    nd = np.nonzero(np.asarray(dominated_by) == 0)[0]
    n = len(nd)
    donor = np.full(len(nis), -1, np.int32)
    for s in range(len(nis)):
        if nis[s] > nis_max and n > 0:
            i = int(np.floor(np.float32(u[s]) * np.float32(n)))
            donor[s] = nd[min(max(i, 0), n - 1)]
    return donor
