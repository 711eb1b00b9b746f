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


def test_merge_archive_with_payload_matches_plain_merge():
    rng = np.random.default_rng(9)
    pts = np.round(rng.random((200, 3)), 2)
    pay = np.arange(200)[:, None].astype(np.float64)
    arch, ap = O.merge_archive_with(np.zeros((0, 3)), None, pts[:80], pay[:80])
    arch, ap = O.merge_archive_with(arch, ap, pts[80:], pay[80:])
    np.testing.assert_array_equal(arch, O.nondominated(pts))
    for row, p in zip(arch, ap[:, 0].astype(int)):
        np.testing.assert_array_equal(pts[p], row)  # every kept row carries its own payload


def test_device_merge_payload_matches_host_merge():
    """merge_archive_device (run here on CPU tensors) carries each row's solution
    exactly as the host merge does, over several generations with duplicates."""
    import torch
    rng = np.random.default_rng(11)
    cap = 512
    arch = torch.full((cap, 3), float("inf"), dtype=torch.float64)
    arch_X = torch.zeros((cap, 2, 3), dtype=torch.float32)
    n, h_arch, h_pay = 0, np.zeros((0, 3)), None
    for g in range(6):
        new = np.round(rng.random((64, 3)), 2)
        if n:
            new[:3] = arch[:3].numpy()  # duplicates of archived rows: the archived payload is kept
        new_X = rng.random((64, 2, 3)).astype(np.float32)
        n = O.merge_archive_device(arch, n, torch.from_numpy(new), arch_X, torch.from_numpy(new_X))
        h_arch, h_pay = O.merge_archive_with(h_arch, h_pay, new, new_X)
        np.testing.assert_array_equal(arch[:n].numpy(), h_arch)
        np.testing.assert_array_equal(arch_X[:n].numpy(), h_pay)
        assert torch.all(torch.isinf(arch[n:]))


def test_avs_update_rule():
    """AMaLGaM's variance-scaling step, case by case (run on CPU tensors)."""
    import torch
    c = torch.tensor([0.5, 1.0, 2.0, 2.0, 1.0, 1.0, 0.8], dtype=torch.float32)
    nis = torch.tensor([3, 3, 0, 5, 2, 9, 9], dtype=torch.int32)
    sdr = torch.tensor([2.0, 0.5, 1.5, -1.0, -1.0, -1.0, -1.0], dtype=torch.float64)
    c1, n1 = O.avs_update(c, nis, sdr, nis_max=10)
    want = [1.0 / 0.9,   # improved, c < 1 -> 1, sdr > 1 -> grows
            1.0,         # improved, sdr <= 1: at least 1
            2.0 / 0.9,   # improved far from the mean: grows
            1.8,         # no improvement, c > 1: shrinks, stretch unchanged
            1.0,         # no improvement, c <= 1, short stretch: stays 1, stretch + 1
            0.9,         # no improvement, stretch reaches the maximum: shrinks below 1
            0.72]        # c < 1 and the stretch past the maximum: keeps shrinking
    assert np.allclose(c1.numpy(), want, rtol=1e-6)
    assert n1.tolist() == [0, 0, 0, 5, 3, 10, 10]
