"""GPU parity of the generation bookkeeping kernels against the oracle
(oracle/gomea_ref.py): the elitist archive bit for bit (vectors, order, count
and payload rows, over several merges, with ties and duplicates, and the
capacity overflow), the selection's indices and dominated-by counts, the
adaptive multiplier step, and the forced-improvement replacement."""
import sys

import numpy as np
import pytest

from oracle import gomea_ref as G
from paper_2202_11001_amd import optimizer as O
from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-bookkeeping] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("kind", ["integers", "reals"])
def test_archive_merge_rounds_match_oracle(kind):
    rng = np.random.default_rng(0 if kind == "integers" else 1)
    A = dsm.Archive(capacity=4096, m_max=80, row_floats=5)
    ref_vec, ref_rows = np.zeros((0, 3)), np.zeros((0, 5), np.float32)
    for r in range(8):
        m = int(rng.integers(1, 81))
        if kind == "integers":
            pts = rng.integers(0, 8, (m, 3)).astype(np.float64)   # many ties and duplicates
        else:
            pts = rng.uniform(0, 1, (m, 3)) + 0.01 * r
        rows = rng.normal(size=(m, 5)).astype(np.float32)
        A.merge(_t(pts), _t(rows))
        ref_vec, ref_rows = G.archive_merge(ref_vec, pts, ref_rows, rows)
        torch.cuda.synchronize()
        n = A.n
        _say(f"{kind} round {r}: {m} points -> {n} archived")
        assert n == len(ref_vec)
        v = A.vec.cpu().numpy()
        np.testing.assert_array_equal(v[:n], ref_vec)
        assert np.all(v[n:] == np.inf)
        np.testing.assert_array_equal(A.rows[:n].cpu().numpy(), ref_rows)
        assert int(A.overflow.item()) == 0


def test_archive_merge_large_equals_host_merge():
    """A population-sized stream of points into a large archive, against the
    host merge of the optimiser harness."""
    rng = np.random.default_rng(5)
    A = dsm.Archive(capacity=1 << 14, m_max=512)
    host = np.zeros((0, 3))
    for r in range(6):
        # points near a front so that the archive grows to thousands of rows
        u = rng.uniform(0, 1, (512, 2))
        pts = np.stack([u[:, 0], u[:, 1], 1.0 - u.sum(1) / 2 + rng.uniform(0, 0.02, 512)], 1)
        A.merge(_t(pts))
        host = O.merge_archive(host, pts)
    torch.cuda.synchronize()
    assert A.n == len(host) > 1000
    np.testing.assert_array_equal(A.vec[:A.n].cpu().numpy(), host)


def test_archive_overflow_leaves_archive_unchanged():
    A = dsm.Archive(capacity=8, m_max=16)
    pts = np.stack([np.arange(6.0), 5 - np.arange(6.0), np.zeros(6)], 1)  # 6 mutually non-dominated
    A.merge(_t(pts))
    torch.cuda.synchronize()
    before = A.vec.cpu().numpy().copy()
    more = np.stack([np.arange(6.0) + 0.5, 5 - np.arange(6.0), np.zeros(6)], 1)  # 6 more, all kept: 12 > 8
    more[:, 1] -= 0.25
    A.merge(_t(more))
    torch.cuda.synchronize()
    assert int(A.overflow.item()) == 1 and A.n == 6
    np.testing.assert_array_equal(A.vec.cpu().numpy(), before)


@pytest.mark.parametrize("kind", ["integers", "reals"])
def test_select_matches_oracle(kind):
    rng = np.random.default_rng(7)
    S = 512
    obj = rng.integers(0, 5, (S, 3)).astype(np.float64) if kind == "integers" else rng.uniform(0, 2, (S, 3))
    n_sel = 179
    cnt = torch.empty(S, dtype=torch.int32, device=DEV)
    sel = dsm.select(_t(obj), n_sel, dominated_by=cnt)
    torch.cuda.synchronize()
    rsel, rcnt = G.select(obj, n_sel)
    np.testing.assert_array_equal(cnt.cpu().numpy(), rcnt)
    np.testing.assert_array_equal(sel.cpu().numpy(), rsel)


def test_avs_update_matches_oracle():
    rng = np.random.default_rng(9)
    n = 5000
    mult = rng.choice([0.05, 0.5, 0.9, 1.0, 1.5, 9.5], n).astype(np.float32) * rng.uniform(0.9, 1.1, n).astype(np.float32)
    nis = rng.integers(0, 40, n).astype(np.int32)
    sdr = np.where(rng.uniform(size=n) < 0.5, -1.0, rng.uniform(0, 3, n))
    m_d, n_d = _t(mult), _t(nis)
    dsm.avs_update(m_d, n_d, _t(sdr), 31)
    torch.cuda.synchronize()
    rm, rn = G.avs_update(mult, nis, sdr, 31)
    np.testing.assert_array_equal(m_d.cpu().numpy(), rm)
    np.testing.assert_array_equal(n_d.cpu().numpy(), rn)


def test_forced_replace_matches_oracle():
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S = X.shape[0]
    gp = dsm.Problem.from_workload(w, max_solutions=S)
    rng = np.random.default_rng(2)
    obj = rng.normal(size=(S, 3))
    cache = rng.normal(size=(S, gp.T, 3))
    donor = np.full(S, -1, np.int32)
    donor[[1, 2, 5, 9]] = [2, 3, 0, 9]     # a chain 1 <- 2 <- 3 and a self-donor
    acc = [rng.integers(0, 2, (S, 4)).astype(np.uint8) * (rng.uniform(size=(S, 1)) < 0.3) for _ in range(3)]
    acc[0][[1, 2, 5, 9]] = 0
    acc[1][[1, 2, 5, 9]] = 0
    acc[2][[1, 2, 9]] = 0
    acc[2][5, 0] = 1                          # solution 5 had a donor but improved
    improved = np.zeros(S, np.uint8)
    imp_d = _t(improved)
    for a in acc:
        dsm.mark_improved(_t(a), imp_d)
    nis = rng.integers(0, 6, S).astype(np.int32)
    Xd, od, cd, nd = _t(X), _t(obj), _t(cache), _t(nis)
    nrep = torch.zeros(1, dtype=torch.int32, device=DEV)
    gp.forced_replace(Xd, od, cd, _t(donor), imp_d, nd, n_replaced=nrep)
    torch.cuda.synchronize()
    imp_ref = np.any(np.concatenate(acc, axis=1) != 0, axis=1).astype(np.uint8)
    np.testing.assert_array_equal(imp_d.cpu().numpy(), imp_ref)
    rX, ro, rc, rn, k = G.forced_replace(X, obj, cache, donor, imp_ref, nis)
    assert int(nrep.item()) == k == 3
    np.testing.assert_array_equal(Xd.cpu().numpy(), rX)
    np.testing.assert_array_equal(od.cpu().numpy(), ro)
    np.testing.assert_array_equal(cd.cpu().numpy(), rc)
    np.testing.assert_array_equal(nd.cpu().numpy(), rn)


@pytest.mark.parametrize("k", [1, 5])
def test_multiplier_step_matches_oracle(k):
    rng = np.random.default_rng(11 + k)
    S, F = 512, 75
    acc = (rng.uniform(size=(S, F)) < 0.004).astype(np.uint8)
    cluster = rng.integers(0, k, S).astype(np.int32)
    mult = rng.choice([0.05, 0.3, 1.0, 9.9], (k, F)).astype(np.float32)
    md = _t(mult)
    dsm.multiplier_step(_t(acc), md, cluster=_t(cluster) if k > 1 else None)
    torch.cuda.synchronize()
    want = G.multiplier_step(acc, mult, cluster if k > 1 else None)
    np.testing.assert_array_equal(md.cpu().numpy(), want)


@pytest.mark.parametrize("has_prev", [True, False])
def test_ams_shift_matches_oracle(has_prev):
    rng = np.random.default_rng(21)
    mean = rng.normal(size=(600, 6)) * 50
    prev = rng.normal(size=(600, 6)) * 50
    shift0 = rng.normal(size=(600, 6))
    m, p, sh = _t(mean), _t(prev), _t(shift0)
    dsm.ams_shift(m, p, sh, has_prev=has_prev)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p.cpu().numpy(), mean)
    np.testing.assert_array_equal(sh.cpu().numpy(), G.ams_shift(mean, prev) if has_prev else shift0)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 16])
def test_single_objective_clusters_matches_oracle(k):
    rng = np.random.default_rng(30 + k)
    means = rng.integers(0, 4, (k, 3)).astype(np.float64) / 4.0  # many ties
    assign = rng.integers(-1, k, 700).astype(np.int32)
    so = dsm.single_objective_clusters(_t(means), _t(assign))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(so.cpu().numpy(), G.single_objective_clusters(means, assign))


@pytest.mark.parametrize("S", [7, 512, 3000])
def test_draw_donors_matches_oracle(S):
    rng = np.random.default_rng(S)
    obj = rng.integers(0, 6, (S, 3)).astype(np.float64)
    cnt = torch.empty(S, dtype=torch.int32, device=DEV)
    dsm.select(_t(obj), 0, dominated_by=cnt)
    nis = rng.integers(0, 8, S).astype(np.int32)
    u = rng.random(S).astype(np.float32)
    n_forced = torch.full((1,), 5, dtype=torch.int32, device=DEV)
    donor = dsm.draw_donors(_t(nis), 4, cnt, _t(u), n_forced=n_forced)
    torch.cuda.synchronize()
    want = G.draw_donors(nis, 4, cnt.cpu().numpy(), u)
    np.testing.assert_array_equal(donor.cpu().numpy(), want)
    assert int(n_forced.item()) == 5 + int((want >= 0).sum()) and (want >= 0).sum() > 0
