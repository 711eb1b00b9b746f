"""Host-side pieces of the optimiser harness: parity classes (independent
partial changes, Sec. 2.2), non-dominated filtering, exact 3-D hypervolume."""
import itertools

import numpy as np

from oracle import ref
from paper_2202_11001_amd import optimizer as O


def test_parity_classes_have_disjoint_stars():
    z = np.zeros((20, 20, 20), np.float32)
    for mesh in [(3, 3, 3), (5, 4, 3), (10, 10, 6)]:
        rp = ref.Problem(z, z, mesh)
        off, st = rp.star()
        classes = O.parity_classes(mesh)
        assert sorted(np.concatenate(classes).tolist()) == list(range(rp.P))
        for c in classes:
            seen = set()
            for p in c:
                s = set(st[off[p]:off[p + 1]].tolist())
                assert not (s & seen)
                seen |= s


def test_nondominated():
    pts = np.array([[1, 2, 3], [2, 1, 3], [2, 2, 4], [1, 2, 3], [0, 5, 5], [3, 3, 3]], float)
    nd = O.nondominated(pts)
    assert {tuple(r) for r in nd} == {(1, 2, 3), (2, 1, 3), (0, 5, 5)}


def _hv_bruteforce(pts, ref_):
    """Exact union volume by inclusion-exclusion over all subsets (small sets)."""
    pts = np.asarray(pts, float)
    total = 0.0
    for k in range(1, len(pts) + 1):
        for sub in itertools.combinations(range(len(pts)), k):
            corner = pts[list(sub)].max(axis=0)
            total += (-1) ** (k + 1) * np.prod(np.maximum(ref_ - corner, 0))
    return total


def test_hypervolume_exact():
    ref_ = np.array([10.0, 10.0, 10.0])
    assert O.hypervolume([[1, 2, 3]], ref_) == 9 * 8 * 7
    rng = np.random.default_rng(0)
    for n in (2, 3, 5, 8):
        pts = rng.uniform(0, 10, (n, 3))
        assert O.hypervolume(pts, ref_) == __import__("pytest").approx(_hv_bruteforce(pts, ref_), rel=1e-12)
    # points outside the reference box contribute nothing
    assert O.hypervolume([[11, 1, 1]], ref_) == 0.0


def test_merge_archive_equals_filtering_the_union():
    rng = np.random.default_rng(5)
    arch = O.nondominated(rng.random((300, 3)))
    for _ in range(5):
        new = np.round(rng.random((64, 3)), 2)
        new[:4] = arch[:4]  # duplicates of archive rows
        merged = O.merge_archive(arch, new)
        np.testing.assert_array_equal(merged, O.nondominated(np.concatenate([arch, new])))
        arch = merged
