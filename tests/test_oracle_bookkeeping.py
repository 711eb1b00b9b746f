"""Pins of the oracle's generation bookkeeping (oracle/gomea_ref.py): the
elitist archive (the approximation set, Sec. 2.4), the selection, the adaptive
multiplier step and the forced-improvement replacement (RV-GOMEA, Sec. 2.2),
against hand-computed cases and characterisations that do not use the
oracle's own code."""
import numpy as np
import pytest

from oracle import gomea_ref as G


def test_archive_merge_hand_case():
    arch = np.array([[1, 5, 5], [2, 2, 6], [4, 1, 9]], float)
    pts = np.array([[1, 5, 5],   # equal to an archive row: the archived one stays
                    [2, 2, 5],   # dominates archive row (2, 2, 6)
                    [3, 3, 3],
                    [0, 9, 9],
                    [3, 3, 3],   # duplicate of an earlier point
                    [5, 5, 9]], float)  # dominated by (2, 2, 5)
    vec, rows = G.archive_merge(arch, pts, np.array([10, 20, 30]), np.array([1, 2, 3, 4, 5, 6]))
    np.testing.assert_array_equal(vec, [[0, 9, 9], [1, 5, 5], [2, 2, 5], [3, 3, 3], [4, 1, 9]])
    np.testing.assert_array_equal(rows, [4, 10, 2, 3, 30])


def _insert_one_by_one(vectors):
    """The classic elitist-archive update, one vector at a time: a vector
    dominated by or equal to a member is rejected; otherwise it enters and the
    members it dominates leave."""
    arch = []
    for v in map(tuple, vectors):
        if any(all(a <= b for a, b in zip(m, v)) for m in arch):
            continue  # dominated by or equal to a member
        arch = [m for m in arch if not (all(a <= b for a, b in zip(v, m)) and any(a < b for a, b in zip(v, m)))]
        arch.append(v)
    return sorted(arch)


@pytest.mark.parametrize("seed", range(4))
def test_archive_merge_equals_incremental_insertion(seed):
    rng = np.random.default_rng(seed)
    # small integer objectives: many ties and duplicates
    pts = rng.integers(0, 6, (120, 3)).astype(float)
    vec, _ = G.archive_merge(np.zeros((0, 3)), pts)
    assert [tuple(r) for r in vec] == _insert_one_by_one(pts)
    # merging in rounds gives the same set (associativity) and is idempotent
    a = np.zeros((0, 3))
    for part in np.array_split(pts, 5):
        a, _ = G.archive_merge(a, part)
    np.testing.assert_array_equal(a, vec)
    again, _ = G.archive_merge(vec, vec)
    np.testing.assert_array_equal(again, vec)
    # sorted lexicographically and distinct
    assert all(tuple(vec[i]) < tuple(vec[i + 1]) for i in range(len(vec) - 1))


def test_select_hand_case():
    obj = np.array([[1, 1, 1], [2, 2, 2], [0, 5, 5], [2, 2, 2], [3, 0, 9]], float)
    # dominated-by counts: only (1, 1, 1) dominates the two (2, 2, 2) rows
    # normalised sums (ranges 3, 5, 8 from lows 0, 0, 1): 0.533, 1.192, 1.5, 1.192, 2.0
    sel, count = G.select(obj, 5)
    np.testing.assert_array_equal(count, [0, 1, 0, 1, 0])
    np.testing.assert_array_equal(sel, [0, 2, 4, 1, 3])  # equal keys by index
    np.testing.assert_array_equal(G.select(obj, 3)[0], [0, 2, 4])


def test_select_counts_decide_first():
    """Any solution dominated by fewer members comes first, whatever its sum."""
    rng = np.random.default_rng(3)
    obj = rng.uniform(0, 1, (60, 3))
    sel, count = G.select(obj, 60)
    assert np.all(np.diff(count[sel]) >= 0)
    assert sorted(sel.tolist()) == list(range(60))


@pytest.mark.parametrize("c,nis,sdr,want_c,want_nis", [
    (0.5, 7, 2.0, np.float32(1.0) / np.float32(0.9), 0),   # improvement, ratio above 1: at least 1, then / eta
    (0.5, 7, 0.5, 1.0, 0),                                  # improvement, ratio at most 1: at least 1
    (3.0, 7, 0.5, 3.0, 0),                                  # improvement keeps a multiplier above 1
    (9.5, 0, 2.0, 10.0, 0),                                 # clamped to the upper bound
    (2.0, 3, -1.0, np.float32(2.0) * np.float32(0.9), 3),  # no improvement, above 1: shrink, stretch kept
    (0.5, 3, -1.0, 1.0, 4),                                 # below 1 with a short stretch: back to 1
    (1.0, 9, -1.0, np.float32(0.9), 10),                    # the stretch reaches its limit: shrink below 1
    (0.06, 20, -1.0, np.float32(0.06) * np.float32(0.9), 21),
    (0.05, 20, -1.0, 0.05, 21),                             # clamped to the lower bound
])
def test_avs_update_cases(c, nis, sdr, want_c, want_nis):
    mc, mn = G.avs_update(np.array([c], np.float32), np.array([nis], np.int32), np.array([sdr]), 10)
    assert mc[0] == np.float32(want_c)
    assert mn[0] == want_nis


def test_forced_replace_with_a_chain_of_donors():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(4, 2, 5, 3)).astype(np.float32)
    obj = rng.normal(size=(4, 3))
    cache = rng.normal(size=(4, 7, 3))
    donor = np.array([-1, 2, 3, -1])
    improved = np.array([0, 0, 0, 1])
    X2, o2, c2, nis2, n = G.forced_replace(X, obj, cache, donor, improved, np.array([5, 5, 5, 5]))
    assert n == 2
    np.testing.assert_array_equal(X2[0], X[0])
    np.testing.assert_array_equal(X2[1], X[2])   # the donor's values from before the step
    np.testing.assert_array_equal(X2[2], X[3])
    np.testing.assert_array_equal(o2[1], obj[2])
    np.testing.assert_array_equal(c2[2], cache[3])
    np.testing.assert_array_equal(X2[3], X[3])
    np.testing.assert_array_equal(nis2, [6, 0, 0, 0])


def test_multiplier_step_hand_case():
    acc = np.array([[1, 0, 0],
                    [0, 0, 1],
                    [0, 0, 0]], np.uint8)
    cluster = np.array([0, 1, 1])
    mult = np.array([[1.0, 0.055, 9.5], [2.0, 1.0, 1.0]], np.float32)
    out = G.multiplier_step(acc, mult, cluster)
    f = np.float32
    # cluster 0 (solution 0) hit element 0; cluster 1 (solutions 1, 2) hit element 2
    # (0.055 * 0.9 = 0.0495 is raised to the lower bound 0.05)
    np.testing.assert_array_equal(out, np.array([[f(1.0) / f(0.9), 0.05, f(9.5) * f(0.9)],
                                                 [f(2.0) * f(0.9), f(1.0) * f(0.9), f(1.0) / f(0.9)]], np.float32))
    # without clusters a hit anywhere counts; the bounds hold
    out1 = G.multiplier_step(acc, np.array([[9.5, 0.05, 0.5]], np.float32))
    np.testing.assert_array_equal(out1, np.array([[10.0, 0.05, f(0.5) / f(0.9)]], np.float32))


def test_ams_shift_hand_case():
    np.testing.assert_array_equal(G.ams_shift([1.5, 2.0, -1.0], [1.0, 3.0, -1.0]), [0.5, -1.0, 0.0])


def test_single_objective_clusters_hand_case():
    means = np.array([[0.5, 0.2, 0.9],
                      [0.1, 0.8, 0.3],
                      [0.1, 0.1, 0.1],   # ties cluster 1 in objective 0: the lower index wins
                      [0.7, 0.7, 0.0]])
    # objective 0 -> cluster 1; objective 1 -> cluster 2 (0.1 < 0.2 < 0.7); objective 2 -> cluster 3 (0.0 < 0.9)
    np.testing.assert_array_equal(G.single_objective_clusters(means, [0, 1, 2, 3, 1, -1]), [-1, 0, 1, 2, 0, -1])
    # two clusters: objective 0 takes cluster 1, objective 1 the remaining cluster 0, objective 2 none
    np.testing.assert_array_equal(G.single_objective_clusters(means[:2], [0, 1, 1]), [1, 0, 0])
    # one cluster: it optimises objective 0
    np.testing.assert_array_equal(G.single_objective_clusters(means[:1], [0, 0]), [0, 0])


def test_draw_donors_hand_case():
    dominated_by = np.array([0, 2, 0, 1, 0])          # non-dominated: 0, 2, 4
    nis = np.array([5, 0, 7, 9, 1])                   # stretches above 4: solutions 0, 2, 3
    u = np.array([0.0, 0.5, 0.34, 0.999, 0.2], np.float32)
    # floor(0 * 3) = 0, floor(1.02) = 1, floor(2.997) = 2
    np.testing.assert_array_equal(G.draw_donors(nis, 4, dominated_by, u), [0, -1, 2, 4, -1])
    # nobody flagged
    np.testing.assert_array_equal(G.draw_donors(nis, 9, dominated_by, u), [-1] * 5)


def test_draw_donors_are_uniform_over_the_non_dominated():
    """Every flagged solution gets a non-dominated member, and draws spread
    evenly over [0, 1) give every such member the same share."""
    rng = np.random.default_rng(4)
    S = 40
    dominated_by = rng.integers(0, 3, S)
    nd = np.nonzero(dominated_by == 0)[0]
    hits = np.zeros(S, int)
    for r in range(500):
        u = ((np.arange(S) + r * S) / (500.0 * S)).astype(np.float32)  # 20,000 draws on an even grid of [0, 1)
        d = G.draw_donors(np.ones(S, int), 0, dominated_by, u)
        assert np.all(np.isin(d, nd))
        np.add.at(hits, d, 1)
    share = hits[nd]
    assert share.sum() == 500 * S and share.max() - share.min() <= 1
