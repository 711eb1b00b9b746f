"""Pins of the distribution-estimation reference (oracle/gomea_ref.py) against
hand-computed values, numpy's Cholesky and the defining identities."""
import numpy as np

from oracle import gomea_ref as G

MESH = (4, 4, 3)
P = 48
INTERIOR = 1 + 4 * (1 + 4 * 1)  # (1, 1, 1)
CORNER = 0
FACE = 1 + 4 * 1  # (1, 1, 0): z pinned


def _population(S, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(10.0, 2.0, size=(S, 2, P, 3)).astype(np.float32)


def test_free_axes():
    assert G.free_axes(INTERIOR, MESH).all()
    assert not G.free_axes(CORNER, MESH).any()
    assert list(G.free_axes(FACE, MESH)) == [True, True, False, True, True, False]


def test_hand_computed_mean_and_covariance():
    X = np.zeros((3, 2, P, 3), dtype=np.float32)
    X[:, 0, INTERIOR, 0] = [0.0, 1.0, 2.0]   # source x: mean 1, variance 2/3
    X[:, 1, INTERIOR, 2] = [4.0, 4.0, 7.0]   # target z: mean 5, variance 2
    mean, cov, chol = G.estimate(X, [0, 1, 2], [INTERIOR], MESH)
    assert np.allclose(mean[0], [1, 0, 0, 0, 0, 5])
    want = np.zeros((6, 6))
    want[0, 0] = 2.0 / 3.0
    want[5, 5] = 2.0
    want[0, 5] = want[5, 0] = ((-1) * (-1) + 0 * (-1) + 1 * 2) / 3.0  # = 1
    assert np.allclose(cov[0], want)
    L = chol[0]
    assert np.allclose(L @ L.T, want)
    assert np.allclose(L[0, 0], np.sqrt(2.0 / 3.0)) and np.allclose(L[5, 0], 1.0 / np.sqrt(2.0 / 3.0))


def test_positive_definite_case_matches_numpy_cholesky():
    X = _population(40, seed=1)
    mean, cov, chol = G.estimate(X, list(range(0, 40, 2)), [INTERIOR], MESH)
    x = np.array([np.concatenate([X[s, 0, INTERIOR], X[s, 1, INTERIOR]]) for s in range(0, 40, 2)], dtype=np.float64)
    assert np.allclose(mean[0], x.mean(axis=0))
    assert np.allclose(cov[0], np.cov(x.T, bias=True))
    assert np.allclose(chol[0], np.linalg.cholesky(np.cov(x.T, bias=True)))


def test_rank_deficient_and_pinned():
    X = _population(10, seed=2)
    # 3 solutions: rank <= 2 covariance; the factor still reproduces it
    _, cov, chol = G.estimate(X, [1, 4, 7], [INTERIOR], MESH)
    assert np.allclose(chol[0] @ chol[0].T, cov[0], atol=1e-12)
    assert np.all(np.triu(chol[0], 1) == 0)
    # identical solutions: zero covariance and factor
    Y = np.repeat(X[:1], 4, axis=0)
    mean, cov, chol = G.estimate(Y, [0, 1, 2, 3], [INTERIOR], MESH)
    assert np.allclose(mean[0], np.concatenate([X[0, 0, INTERIOR], X[0, 1, INTERIOR]]))
    assert np.all(cov[0] == 0) and np.all(chol[0] == 0)
    # a face point: the pinned z rows and columns are zero
    _, cov, chol = G.estimate(X, list(range(10)), [FACE], MESH)
    for c in (2, 5):
        assert np.all(cov[0][c] == 0) and np.all(cov[0][:, c] == 0) and np.all(chol[0][:, c] == 0)
    assert np.allclose(chol[0] @ chol[0].T, cov[0])


def test_out_of_range_selection_is_skipped():
    X = _population(6, seed=3)
    a = G.estimate(X, [0, 2, 4], [INTERIOR], MESH)
    b = G.estimate(X, [0, -1, 2, 6, 4, 99], [INTERIOR], MESH)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_packed_lower_layout():
    L = np.tril(np.arange(36, dtype=float).reshape(6, 6))
    packed = G.packed_lower(L)
    assert len(packed) == 21
    assert packed[0] == L[0, 0] and list(packed[1:3]) == [L[1, 0], L[1, 1]] and packed[20] == L[5, 5]


def test_elements_reduce_to_points_and_are_joint():
    X = _population(60, seed=5)
    sel = list(range(0, 60, 2)) + list(range(1, 20, 2))  # 40 solutions: more than the 24 variables
    # a one-point element equals the per-point estimate in the first 6 variables
    pm, pc, pl = G.estimate(X, sel, [INTERIOR], MESH)
    em, ec, el = G.estimate_elements(X, sel, np.array([0, 1]), np.array([INTERIOR]), MESH)
    assert np.allclose(em[0, :6], pm[0]) and np.allclose(ec[0, :6, :6], pc[0]) and np.allclose(el[0, :6, :6], pl[0])
    assert np.all(em[0, 6:] == 0) and np.all(el[0, 6:] == 0)
    # a 4-point element: the diagonal blocks are the per-point covariances, the
    # off-diagonal blocks the cross-covariances; numpy's covariance and factor
    pts = np.array([INTERIOR, INTERIOR + 1, FACE, INTERIOR + 4])
    em, ec, el = G.estimate_elements(X, sel, np.array([0, 4]), pts, MESH)
    x = np.concatenate([G.coordinates(X, sel, p) for p in pts], axis=1)
    free = np.concatenate([G.free_axes(p, MESH) for p in pts])
    want = np.cov((x * free).T, bias=True)
    assert np.allclose(ec[0], want)
    for k, p in enumerate(pts):
        assert np.allclose(ec[0, 6 * k:6 * k + 6, 6 * k:6 * k + 6], G.estimate(X, sel, [p], MESH)[1][0])
    assert np.allclose(el[0] @ el[0].T, ec[0], atol=1e-10)
    fr = np.nonzero(free)[0]
    assert np.allclose(el[0][np.ix_(fr, fr)], np.linalg.cholesky(want[np.ix_(fr, fr)]))
    # rejected elements: 5 points, an invalid point, no point
    em, ec, el = G.estimate_elements(X, sel, np.array([0, 5, 6, 6]), np.array([1, 2, 3, 4, 5, -1]), MESH)
    assert np.all(em == 0) and np.all(el == 0)


# ---------------------------------------------------------------- clustering

def test_cluster_hand_computed():
    # first objective 0, 2, 4, 8 -> normalised 0, .25, .5, 1 (exact); leaders 3 then 0;
    # .5 is equally far from both leaders and joins cluster 0; means .75 and .125
    obj = np.zeros((4, 3))
    obj[:, 0] = [0, 2, 4, 8]
    members, assign, means = G.cluster(obj, [0, 1, 2, 3], 2)
    assert np.array_equal(assign, [1, 1, 0, 0])
    assert np.allclose(means, [[0.75, 0, 0], [0.125, 0, 0]], rtol=0, atol=0)
    # c = min(4, ceil(2 * 4 / 2)) = 4; equal distances keep selection order
    assert members.tolist() == [[2, 3, 1, 0], [0, 1, 2, 3]]


def _blobs(seed=0, n=20):
    rng = np.random.default_rng(seed)
    centres = np.array([[0, 0, 10], [10, 0, 0], [0, 10, 0]], float)
    obj = np.concatenate([c + rng.normal(0, 0.5, (n, 3)) for c in centres])
    return obj, np.repeat(np.arange(3), n)


def test_cluster_separated_blobs():
    obj, label = _blobs()
    members, assign, means = G.cluster(obj, np.arange(60), 3)
    assert members.shape == (3, 40)
    # every cluster is one blob (plus the 20 nearest others), every solution joins its blob's cluster
    for j in range(3):
        blob = label[members[j, 0]]
        assert set(np.nonzero(label == blob)[0]) <= set(members[j].tolist())
        assert np.all(assign[label == blob] == j)
    lo, hi = obj.min(axis=0), obj.max(axis=0)
    for j in range(3):
        blob = label[members[j, 0]]
        assert np.allclose(means[j], ((obj[label == blob] - lo) / (hi - lo)).mean(axis=0), atol=1e-12)


def test_cluster_invariants_random():
    rng = np.random.default_rng(4)
    obj = rng.uniform(0, 1, (90, 3)) ** np.array([1.0, 2.0, 0.5])
    sel = rng.choice(90, 40, replace=False)
    k = 4
    members, assign, means = G.cluster(obj, sel, k)
    c = G.cluster_size(40, k)
    assert members.shape == (k, c) == (4, 20)
    lo, hi = obj[sel].min(axis=0), obj[sel].max(axis=0)
    Y = (obj - lo) / (hi - lo)
    d = ((Y[:, None, :] - means[None]) ** 2).sum(axis=2)  # [S][k]
    assert np.array_equal(assign, d.argmin(axis=1))
    # k-means fixed point: each mean is the average of the selected solutions nearest to it
    near = d[sel].argmin(axis=1)
    for j in range(k):
        assert np.allclose(means[j], Y[sel][near == j].mean(axis=0), atol=1e-12)
        # cluster j: the c selected solutions nearest to mean j, nearest first
        order = sel[np.argsort(d[sel, j], kind="stable")]
        assert np.array_equal(members[j], order[:c])
    # one cluster: every selected solution, nearest to the centroid first
    m1, a1, mu1 = G.cluster(obj, sel, 1)
    assert m1.shape == (1, 40) and set(m1[0].tolist()) == set(sel.tolist()) and np.all(a1 == 0)
    assert np.allclose(mu1[0], Y[sel].mean(axis=0), atol=1e-12)


def test_cluster_edge_cases():
    obj, _ = _blobs(n=4)
    a = G.cluster(obj, [0, 5, 9], 2)
    b = G.cluster(obj, [-1, 0, 12, 5, 99, 9], 2)  # out-of-range indices are dropped
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    m, asg, mu = G.cluster(obj, [0, 5, -3], 3)  # 2 valid < k
    assert np.all(m == -1) and np.all(asg == -1) and np.all(np.isnan(mu))
    # identical objectives: zero ranges divide by 1, every solution ties to the first cluster
    m, asg, mu = G.cluster(np.ones((6, 3)), np.arange(6), 2)
    assert np.all(asg == 0) and m[0].tolist() == [0, 1, 2, 3, 4, 5]


def test_standard_deviation_ratio():
    # mean of the samples (2, 0, 5) against (0, 0, 5): 2 / sqrt(4) = 1 on the first
    # variable, 0 on the second, the third has zero variance (pinned) and is skipped
    cov = np.diag([4.0, 1.0, 0.0])
    assert G.standard_deviation_ratio([[1, 0, 5], [3, 0, 5]], [0, 0, 5], cov) == 1.0
    assert G.standard_deviation_ratio([[0, 3, 9]], [0, 0, 5], cov) == 3.0
    assert G.standard_deviation_ratio([[-4, 0.5, 5]], [0, 0, 5], cov) == 2.0  # a shift below the mean counts too
    assert G.standard_deviation_ratio(np.zeros((0, 3)), [0, 0, 5], cov) == -1.0
