"""GPU clustering in objective space (dsm_cluster_objectives) bit for bit
against the FP64 reference oracle/gomea_ref.cluster, per-cluster sampling,
the anticipated mean shift, forced improvements, and optimiser runs that use
them."""
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
    print(f"[gpu-cluster] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _check(obj, sel, k):
    obj = np.asarray(obj, dtype=np.float64)
    sel = np.asarray(sel, dtype=np.int32)
    _say(f"S {len(obj)} n_sel {len(sel)} k {k}")
    m, a, mu = dsm.cluster_objectives(_t(obj), _t(sel), k)
    rm, ra, rmu = G.cluster(obj, sel, k)
    m, a, mu = m.cpu().numpy(), a.cpu().numpy(), mu.cpu().numpy()
    cmax = min(len(sel), -(-2 * len(sel) // k))
    want = np.full((k, cmax), -1, np.int32)
    want[:, :rm.shape[1]] = rm
    np.testing.assert_array_equal(m, want)
    np.testing.assert_array_equal(a, ra)
    np.testing.assert_array_equal(mu, rmu)  # same operations in the same order: equal bits (NaN == NaN here)


def test_cluster_matches_reference_random():
    rng = np.random.default_rng(1)
    for S, n, k in ((500, 175, 5), (90, 40, 4), (37, 13, 13), (64, 64, 1), (3000, 1024, 16),
                    (256, 90, 7)):
        obj = rng.uniform(0, 1, (S, 3)) * np.array([0.1, 5.0, 30.0]) + np.array([0.02, 0.0, 1.0])
        sel = rng.choice(S, n, replace=False)
        _check(obj, sel, k)


def test_cluster_matches_reference_ties_and_edges():
    rng = np.random.default_rng(2)
    # integer-valued objectives: many exact ties in distances and leaders
    obj = rng.integers(0, 3, (64, 3)).astype(np.float64)
    _check(obj, np.arange(64), 5)
    _check(obj, rng.permutation(64)[:30], 3)
    # identical objectives (zero ranges), one constant objective
    _check(np.ones((10, 3)), np.arange(10), 2)
    o = rng.uniform(0, 1, (50, 3))
    o[:, 1] = 7.0
    _check(o, np.arange(0, 50, 2), 4)
    # out-of-range indices dropped (trailing member slots -1), fewer valid than k, empty selection
    _check(o, np.array([0, -1, 3, 50, 9, 12, 99, 20]), 2)
    _check(o, np.array([4, -2, 60]), 3)
    _check(o, np.zeros(0, np.int32), 2)
    # separated blobs
    centres = np.array([[0, 0, 10], [10, 0, 0], [0, 10, 0]], float)
    blobs = np.concatenate([c + rng.normal(0, 0.5, (20, 3)) for c in centres])
    _check(blobs, np.arange(60), 3)
    with pytest.raises(dsm.DsmError):
        dsm.cluster_objectives(_t(o), _t(np.arange(10, dtype=np.int32)), 17)
    with pytest.raises(dsm.DsmError):
        dsm.cluster_objectives(_t(np.zeros((2000, 3))), _t(np.arange(1025, dtype=np.int32)), 4)


def test_sampling_per_cluster():
    """Zero covariance: every candidate is its cluster's mean (snapped); an
    out-of-range cluster gives NaN."""
    w = W.batched()
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    I = gp.topology()["identity"]
    S = 8
    X = _t(np.repeat(np.stack([I, I])[None], S, axis=0))
    p = 1 + 5 * (2 + 5 * 2)  # interior point
    pts = _t(np.array([p], np.int32))
    base = np.concatenate([I[p], I[p]]).astype(np.float64)
    mean = np.stack([base + 1.0, base - 2.0, base + 0.5])[:, None, :]  # [3][1][6]
    chol = np.zeros((3, 1, 21))
    mult = np.ones((3, 1), np.float32)
    cl = np.array([0, 1, 2, 1, 0, 2, 2, 3], np.int32)  # the last one is out of range
    cand = gp.sample_estimated(X, pts, 1, _t(mean), _t(chol), _t(mult), 5, 1, cluster=_t(cl)).cpu().numpy()
    for s in range(S - 1):
        np.testing.assert_array_equal(cand[s, 0].reshape(6), mean[cl[s], 0].astype(np.float32))
    assert np.all(np.isnan(cand[S - 1]))
    # joint 4-point elements
    ps = np.array([p, p + 1, p + 5, p + 25], np.int32)
    off = _t(np.array([0, 4], np.int32))
    mu = np.stack([np.concatenate([np.concatenate([I[q], I[q]]) for q in ps]).astype(np.float64) + d
                   for d in (1.0, -1.0, 0.25)])
    cand = gp.sample_elements(X, off, _t(ps), _t(mu[:, None, :]), _t(np.zeros((3, 1, 300))), _t(mult), 5, 1,
                              cluster=_t(cl)).cpu().numpy()
    for s in range(S - 1):
        np.testing.assert_array_equal(cand[s].reshape(24), mu[cl[s]].astype(np.float32))
    assert np.all(np.isnan(cand[S - 1]))


@pytest.mark.parametrize("fos", ["point", "tetrahedron"])
def test_optimiser_with_clusters(fos):
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4 if fos == "tetrahedron" else 1)
    _say(f"6 generations, {fos} FOS, 4 clusters")
    log, opt, _ = O.run(gp, _t(X), 6, seed=3, sampler="estimated", fos=fos, clusters=4)
    assert log.hypervolume[-1] > log.hypervolume[0] and sum(log.accepted) > 0
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    obj, flags = gp.eval_full(opt.X)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    a = opt._assign.cpu().numpy()
    assert a.shape == (opt.S,) and a.min() >= 0 and a.max() < 4
    with pytest.raises(ValueError):
        O.Optimiser(gp, _t(X), clusters=2)  # clusters need the estimated sampler


def test_anticipated_mean_shift_sampling():
    """Zero covariance: a flagged solution's candidate is mean + delta * mult *
    shift on the free coordinates, an unflagged one the mean; pinned coordinates
    keep the solution's value."""
    w = W.batched()
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    I = gp.topology()["identity"]
    S = 6
    X = _t(np.repeat(np.stack([I, I])[None], S, axis=0))
    p = 1 + 5 * (2 + 5 * 2)          # interior
    q = 2 + 5 * (2 + 5 * 0)          # face point: z pinned in both grids
    rng = np.random.default_rng(6)
    shift = np.zeros((gp.P, 6))
    shift[[p, q, p + 1, p + 5]] = rng.integers(-64, 65, (4, 6)) / 64.0  # lattice-exact after 2 * mult * shift
    ams = np.array([1, 0, 1, 0, 1, 0], np.uint8)
    free = lambda r: np.array([0 < (r % 5) < 4, 0 < (r // 5) % 5 < 4, 0 < r // 25 < 4] * 2)
    # single points
    pts = np.array([p, q], np.int32)
    mean = np.stack([np.concatenate([I[r], I[r]]) for r in pts]).astype(np.float64)
    mult = np.array([1.0, 0.5], np.float32)
    cand = gp.sample_estimated(X, _t(pts), 1, _t(mean), _t(np.zeros((2, 21))), _t(mult), 5, 1,
                               shift=_t(shift), ams=_t(ams), delta=2.0).cpu().numpy()
    for s in range(S):
        for f, r in enumerate(pts):
            want = mean[f] + (2.0 * mult[f] * shift[r] * free(r) if ams[s] else 0.0)
            np.testing.assert_array_equal(cand[s, f].reshape(6), want.astype(np.float32))
    # a 4-point element
    ps = np.array([p, p + 1, p + 5, q], np.int32)
    mu = np.concatenate([np.concatenate([I[r], I[r]]) for r in ps]).astype(np.float64)
    m1 = np.array([0.5], np.float32)
    cand = gp.sample_elements(X, _t(np.array([0, 4], np.int32)), _t(ps), _t(mu[None]), _t(np.zeros((1, 300))),
                              _t(m1), 5, 1, shift=_t(shift), ams=_t(ams), delta=2.0).cpu().numpy()
    for s in range(S):
        want = mu + (2.0 * 0.5 * np.concatenate([shift[r] * free(r) for r in ps]) if ams[s] else 0.0)
        np.testing.assert_array_equal(cand[s].reshape(24), want.astype(np.float32))
    with pytest.raises(ValueError):
        gp.sample_estimated(X, _t(pts), 1, _t(mean), _t(np.zeros((2, 21))), _t(mult), 5, 1, shift=_t(shift))


@pytest.mark.parametrize("fos", ["point", "tetrahedron"])
def test_optimiser_with_anticipated_mean_shift(fos):
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4 if fos == "tetrahedron" else 1)
    _say(f"6 generations, {fos} FOS, anticipated mean shift, 3 clusters")
    log, opt, _ = O.run(gp, _t(X), 6, seed=4, sampler="estimated", fos=fos, clusters=3, ams=True)
    assert log.hypervolume[-1] > log.hypervolume[0] and sum(log.accepted) > 0
    assert opt._shift is not None and opt._shift.shape == (gp.P, 6)
    assert int(opt._ams.sum()) == opt.S // 2
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    obj, flags = gp.eval_full(opt.X)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    with pytest.raises(ValueError):
        O.Optimiser(gp, _t(X), ams=True)  # the shift needs the estimated sampler


def test_copy_from_donor():
    w = W.batched()
    gp = dsm.Problem.from_workload(w)
    rng = np.random.default_rng(12)
    S, P = 6, gp.P
    X = rng.uniform(0, 60, (S, 2, P, 3)).astype(np.float32)
    pts = np.array([3, 17, -1, 60, P, 99], np.int32)  # two invalid points stay unchanged
    donor = np.array([-1, 3, 0, -1, 5, 2], np.int32)
    cand0 = rng.uniform(0, 60, (S, len(pts), 2, 3)).astype(np.float32)
    cand = gp.copy_from_donor(_t(X), _t(pts), _t(donor), _t(cand0)).cpu().numpy()
    for s in range(S):
        for k, p in enumerate(pts):
            if donor[s] >= 0 and 0 <= p < P:
                np.testing.assert_array_equal(cand[s, k], X[donor[s], :, p, :])
            else:
                np.testing.assert_array_equal(cand[s, k], cand0[s, k])


@pytest.mark.parametrize("fos,sampler,sigma", [("point", "isotropic", 40.0), ("tetrahedron", "estimated", 1.0)])
def test_optimiser_with_forced_improvements(fos, sampler, sigma):
    """Forced often (nis_max 0; with sigma 40 nearly every isotropic candidate
    folds, so solutions stagnate and get donors): replaced solutions carry their
    donors' objectives and term cache, which equal a fresh full evaluation."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4 if fos == "tetrahedron" else 1)
    _say(f"6 generations, {fos} FOS, {sampler}, sigma {sigma}, forced improvements")
    log, opt, _ = O.run(gp, _t(X), 6, sigma=sigma, seed=5, sampler=sampler, fos=fos, forced_improvements=True,
                        nis_max=0)
    assert log.hypervolume[-1] >= log.hypervolume[0]
    if sigma > 10:
        assert opt.fi_forced > 0  # (copies from non-dominated donors are nearly always accepted)
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    fresh = torch.empty_like(opt.cache)
    obj, flags = gp.eval_full(opt.X, tet_terms=fresh)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(opt.cache.cpu().numpy(), fresh.cpu().numpy(), rtol=1e-5, atol=1e-9)
    assert opt.nis.min().item() >= 0
    with pytest.raises(ValueError):
        O.Optimiser(gp, _t(X), forced_improvements=True, graph=True)


def test_forced_solution_without_improvement_takes_its_donor():
    """The replacement step: forced solutions that accepted nothing become
    their donors (coordinates, objectives, term cache); improved ones stay."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w)
    opt = O.Optimiser(gp, _t(X), forced_improvements=True)
    S = opt.S
    donor = np.full(S, -1, np.int32)
    donor[[0, 5, 9]] = [7, 7, 0]  # 9's donor is 0, itself replaced in the same step: the old 0 is copied
    opt._donor, opt._fi = _t(donor), donor >= 0
    acc = torch.zeros((S, 4), dtype=torch.uint8, device=DEV)
    acc[5, 1] = 1   # solution 5 accepted a change: kept
    acc[11, 0] = 1  # an unforced solution that improved
    X0, o0, c0, n0 = opt.X.clone(), opt.obj.clone(), opt.cache.clone(), opt.nis.clone()
    opt._after_forcing([(None, acc)])
    for s, d in ((0, 7), (9, 0), (5, 5), (3, 3)):
        assert torch.equal(opt.X[s], X0[d]) and torch.equal(opt.obj[s], o0[d]) and torch.equal(opt.cache[s], c0[d])
    assert opt.fi_replaced == 2
    nis = opt.nis.cpu().numpy()
    assert nis[0] == nis[5] == nis[9] == nis[11] == 0 and nis[3] == n0[3].item() + 1


def test_single_objective_acceptance():
    """A member of a single-objective cluster accepts a feasible change iff it
    lowers that objective; the others use the Pareto / archive rule."""
    w = W.batched()
    gp = dsm.Problem.from_workload(w)
    I = gp.topology()["identity"]
    S, T = 5, gp.T
    X = _t(np.repeat(np.stack([I, I])[None], S, axis=0))
    pts = _t(np.array([31], np.int32))
    cand = X[:, :, 31, :].reshape(S, 1, 2, 3).contiguous()
    old = torch.zeros((S, 1, 3), dtype=torch.float64, device=DEV)
    new = _t(np.array([[[-1, 1, 0]], [[-1, 1, 0]], [[1, -1, 0]], [[-1, -1, 0]], [[0, 0, -1]]], np.float64))
    flags = torch.zeros((S, 1), dtype=torch.uint32, device=DEV)
    flags[4, 0] = 1  # infeasible: never accepted
    so = _t(np.array([0, -1, 0, 1, 2], np.int32))
    cache = torch.zeros((S, T, 3), dtype=torch.float64, device=DEV)
    obj = torch.zeros((S, 3), dtype=torch.float64, device=DEV)
    acc = torch.empty((S, 1), dtype=torch.uint8, device=DEV)
    gp.accept(X, pts, cand, old, new, flags, torch.zeros_like(cache), cache, obj, accepted=acc, single_objective=so)
    assert acc.reshape(-1).cpu().tolist() == [1, 0, 0, 1, 0]
    gp.accept(X, pts, cand, old, new, flags, torch.zeros_like(cache), cache, obj, accepted=acc)
    assert acc.reshape(-1).cpu().tolist() == [0, 0, 0, 1, 0]
    # the multi-point entry point takes the same rule
    off = _t(np.array([0, 1], np.int32))
    gp.accept_elements(X, off, pts, cand, old, new, flags, torch.zeros_like(cache), cache, obj, accepted=acc,
                       single_objective=so)
    assert acc.reshape(-1).cpu().tolist() == [1, 0, 0, 1, 0]


@pytest.mark.parametrize("fos", ["point", "tetrahedron"])
def test_optimiser_with_single_objective_clusters(fos):
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4 if fos == "tetrahedron" else 1)
    _say(f"6 generations, {fos} FOS, 5 clusters, single-objective clusters")
    log, opt, _ = O.run(gp, _t(X), 6, seed=6, sampler="estimated", fos=fos, clusters=5,
                        single_objective_clusters=True)
    assert log.hypervolume[-1] > log.hypervolume[0]
    so = opt._so.cpu().numpy()
    assert so.shape == (opt.S,) and set(np.unique(so).tolist()) <= {-1, 0, 1, 2} and (so >= 0).any()
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    obj, flags = gp.eval_full(opt.X)
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    with pytest.raises(ValueError):
        O.Optimiser(gp, _t(X), sampler="estimated", single_objective_clusters=True)  # needs clusters


@pytest.mark.parametrize("npts", [1, 4])
def test_improvement_ratio_matches_reference(npts):
    """Standard-deviation ratio per (cluster, element) against
    oracle/gomea_ref.standard_deviation_ratio on random accepted sets."""
    rng = np.random.default_rng(20 + npts)
    S, F, C = 40, 7, 3
    nv = 6 if npts == 1 else 24
    off = np.arange(F + 1, dtype=np.int32) * npts
    cand = rng.normal(30, 3, (S, F * npts, 2, 3)).astype(np.float32)
    acc = (rng.uniform(0, 1, (S, F)) < 0.3).astype(np.uint8)
    acc[:, 2] = 0  # an element with no accepted candidate
    cl = rng.integers(0, C, S).astype(np.int32)
    mean = rng.normal(30, 1, (C, F, nv))
    Ls = np.zeros((C, F, nv, nv))
    for j in range(C):
        for f in range(F):
            A = rng.normal(0, 1, (nv, nv))
            Cv = A @ A.T + 0.5 * np.eye(nv)
            Cv[:, 3] = Cv[3, :] = 0  # a pinned variable
            Ls[j, f] = G.cholesky_semidefinite(Cv)
    packed = np.array([[G.packed_lower(Ls[j, f]) for f in range(F)] for j in range(C)])
    got = dsm.improvement_ratio(_t(off), _t(cand), _t(acc), _t(mean), _t(packed), cluster=_t(cl)).cpu().numpy()
    for j in range(C):
        for f in range(F):
            rows = [cand[s, off[f]:off[f + 1]].reshape(-1) for s in range(S) if cl[s] == j and acc[s, f]]
            want = G.standard_deviation_ratio(np.array(rows).reshape(-1, nv), mean[j, f], Ls[j, f] @ Ls[j, f].T)
            np.testing.assert_allclose(got[j, f], want, rtol=1e-9, atol=1e-12)
    assert np.all(got[:, 2] == -1.0)


@pytest.mark.parametrize("fos", ["point", "tetrahedron"])
def test_optimiser_with_sdr_schedule(fos):
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4 if fos == "tetrahedron" else 1)
    _say(f"6 generations, {fos} FOS, 3 clusters, standard-deviation-ratio multipliers")
    log, opt, _ = O.run(gp, _t(X), 6, seed=7, sampler="estimated", fos=fos, clusters=3, multiplier_schedule="sdr")
    assert log.hypervolume[-1] > log.hypervolume[0]
    m = torch.cat([x.reshape(-1) for x in opt.mult]) if fos == "point" else opt.mult_cube.reshape(-1)
    assert float(m.min()) >= 0.05 and float(m.max()) <= 10.0 and float(m.max()) > 1.0
    obj, flags = gp.eval_full(opt.X)
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    with pytest.raises(ValueError):
        O.Optimiser(gp, _t(X), sampler="estimated", multiplier_schedule="other")


def test_rv_gomea_preset_run():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    _say("5 generations with the full RV-GOMEA preset, tetrahedron FOS")
    log, opt, _ = O.run(gp, _t(X), 5, seed=8, fos="tetrahedron", **O.RV_GOMEA)
    assert log.hypervolume[-1] > log.hypervolume[0]
    obj, flags = gp.eval_full(opt.X)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
