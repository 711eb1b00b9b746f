"""GPU generation steps: counter-based candidate sampling, acceptance and
application of independent partial changes (Sec. 2.2), and short optimiser
runs (plain and screened)."""
import sys

import numpy as np
import pytest

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
    print(f"[gpu-optimiser] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_sampler_properties():
    _say("sampler")
    w = W.batched()
    gp = dsm.Problem.from_workload(w)
    I = gp.topology()["identity"]
    X = np.repeat(np.stack([I, I])[None], 8, axis=0)
    Xd = _t(X)
    pts = _t(np.arange(w.P, dtype=np.int32))
    a = gp.sample_candidates(Xd, pts, 4, 1.5, 42, 7).cpu().numpy()
    b = gp.sample_candidates(Xd, pts, 4, 1.5, 42, 7).cpu().numpy()
    c = gp.sample_candidates(Xd, pts, 4, 1.5, 42, 8).cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    free = W.free_mask(w.mesh)  # [P][3]
    cur = np.broadcast_to(X.transpose(0, 2, 1, 3)[:, :, None], a.shape)
    d = a - cur
    fr = np.broadcast_to(free[None, :, None, None, :], a.shape)
    assert np.all(d[~fr] == 0)
    assert np.all(np.rint((a + 0.5) * 128) == (a + 0.5) * 128)
    hi = np.array(w.dims) - 0.5
    assert np.all(a >= -0.5) and np.all(a <= hi)
    dd = d[fr]
    assert abs(dd.mean()) < 0.02 and abs(dd.std() - 1.5) < 0.03


def test_accept_applies_independent_changes():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S = X.shape[0]
    gp = dsm.Problem.from_workload(w)
    Xd = _t(X)
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=DEV)
    obj, _ = gp.eval_full(Xd, tet_terms=cache)
    obj0 = obj.clone()
    arch = _t(O.nondominated(obj.cpu().numpy()))
    cls = O.parity_classes(w.mesh)
    pts = _t(cls[0])
    F = len(cls[0])
    off = _t(np.arange(F + 1, dtype=np.int32))
    _say("accept one parity class")
    cand = gp.sample_candidates(Xd, pts, 1, 2.0, 3, 1)
    terms_cand = torch.zeros_like(cache)
    old, new, fl, _ = gp.eval_partial(Xd, off, pts, cand, tet_terms_in=cache, tet_terms_new=terms_cand)
    acc = torch.empty((S, F), dtype=torch.uint8, device=DEV)
    X1 = Xd.clone()
    gp.accept(X1, pts, cand, old, new, fl, terms_cand, cache, obj, archive=arch, accepted=acc)
    torch.cuda.synchronize()
    # the rule on the GPU's own deltas
    d = (new - old).cpu().numpy()
    o0 = obj0.cpu().numpy()
    A = arch.cpu().numpy()
    expect = np.zeros((S, F), dtype=bool)
    for s in range(S):
        for f in range(F):
            if fl[s, f].item() != 0:
                continue
            dd = d[s, f]
            if np.all(dd <= 0) and np.any(dd < 0):
                expect[s, f] = True
            elif np.any(dd < 0):
                nv = o0[s] + dd
                expect[s, f] = not np.any(np.all(A <= nv, axis=1) & np.any(A < nv, axis=1))
    got = acc.cpu().numpy().astype(bool)
    assert np.array_equal(got, expect)
    assert 0 < got.sum() < got.size
    # coordinates moved exactly where accepted
    Xn = X1.cpu().numpy()
    cn = cand.cpu().numpy()
    for s in range(S):
        for f, p in enumerate(cls[0]):
            want = cn[s, f] if got[s, f] else X[s, :, p]
            assert np.array_equal(Xn[s, :, p], want)
    # objectives and cache agree with a fresh full evaluation of the new solutions
    cache2 = torch.empty_like(cache)
    obj2, fl2 = gp.eval_full(X1, tet_terms=cache2)
    assert int((fl2 != 0).sum()) == 0
    np.testing.assert_allclose(obj.cpu().numpy(), obj2.cpu().numpy(), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(cache.cpu().numpy(), cache2.cpu().numpy(), rtol=1e-4, atol=1e-7)


def test_short_runs_plain_and_screened():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w)
    _say("plain run")
    log, opt, _ = O.run(gp, _t(X), generations=6, sigma=1.0, seed=5)
    hv = np.array(log.hypervolume)
    assert np.all(np.diff(hv) >= -1e-12 * hv[0]) and hv[-1] > hv[0]
    assert all(e == X.shape[0] * w.P for e in log.exact_evals)
    _say("screened run")
    log2, opt2, sur = O.run(gp, _t(X), generations=6, sigma=1.0, seed=5, train_generations=3, train_steps=300)
    assert sur is not None
    assert log2.hypervolume[-1] > log2.hypervolume[0]
    assert all(e <= X.shape[0] * w.P for e in log2.exact_evals[3:])
    # screened generations evaluate at most the picks flagged by the surrogate
    obj2, fl2 = gp.eval_full(opt2.X)
    assert int((fl2 != 0).sum()) == 0
    np.testing.assert_allclose(opt2.obj.cpu().numpy(), obj2.cpu().numpy(), rtol=1e-5, atol=1e-9)


def _state(opt):
    return (opt.X.cpu().numpy(), opt.obj.cpu().numpy(), opt.cache.cpu().numpy(), np.array(opt.archive), opt.counter)


def test_graph_generations_match_eager():
    """Generations replayed from a captured HIP graph equal eager ones bit for
    bit (plain and screened), with host work between the replays."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w)
    Xd = _t(X)
    _say("graph vs eager, plain")
    oe = O.Optimiser(gp, Xd, sigma=1.0, seed=9, graph=False)
    og = O.Optimiser(gp, Xd, sigma=1.0, seed=9, graph=True)
    for gen in range(3):
        re_ = oe.generation()
        rg = og.generation()
        torch.cuda.synchronize()
        assert re_ == rg, (gen, re_, rg)
        for a, b in zip(_state(oe), _state(og)):
            np.testing.assert_array_equal(a, b)
    assert og._graph is not None and oe.counter == 24
    _say("graph vs eager, screened")
    oc = O.Optimiser(gp, Xd, sigma=1.0, seed=3)
    oc.collect = []
    for _ in range(2):
        oc.generation()
    sur, _, _ = O.train_surrogate(oc.collect, steps=200, max_rows=1 << 16)
    oe = O.Optimiser(gp, Xd, sigma=1.0, seed=4, graph=False)
    og = O.Optimiser(gp, Xd, sigma=1.0, seed=4, graph=True)
    for gen in range(2):
        re_ = oe.generation(surrogate=sur)
        rg = og.generation(surrogate=sur)
        torch.cuda.synchronize()
        assert re_ == rg, (gen, re_, rg)
        for a, b in zip(_state(oe), _state(og)):
            np.testing.assert_array_equal(a, b)


def test_multiresolution_seeding():
    """Sec. 2.4: a coarse run keeps its approximation set's solutions; a random
    sample of them, refined on the GPU, starts a feasible finer run."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=32)
    gp = dsm.Problem.from_workload(w, max_solutions=64)
    _say("coarse run keeping archive solutions")
    oc = O.Optimiser(gp, _t(X), sigma=1.0, seed=2, keep_solutions=True)
    for _ in range(3):
        oc.generation()
    assert oc.archive_X.shape == (len(oc.archive), 2, w.P, 3)
    # every archived solution reproduces its archived objective vector
    obj, fl = gp.eval_full(_t(oc.archive_X))
    np.testing.assert_allclose(obj.cpu().numpy(), oc.archive, rtol=1e-6, atol=1e-12)
    nf = tuple(2 * n - 1 for n in w.mesh)
    wf = W.Workload(w.name + "-fine", w.moving, w.fixed, nf, w.spacing, w.tau, 64, w.sigma_pop, w.sigma_cand,
                    w.seed_pop, w.seed_cand, w.guid_moving, w.guid_fixed, w.corr_moving, w.corr_fixed)
    gpf = dsm.Problem.from_workload(wf, max_solutions=64)
    Xf, rejected = O.seed_finer(oc, gpf, 64, seed=5)
    assert Xf.shape == (64, 2, wf.P, 3)
    _say(f"fine run from the refined sample ({rejected} draws rejected)")
    of = O.Optimiser(gpf, Xf, sigma=0.5, seed=3)
    hv0 = of.hypervolume()
    for _ in range(2):
        of.generation()
    assert of.hypervolume() > hv0
    # no rounds of rejection draws: every place is drawn from the feasible refined archive members
    Xg, rej = O.seed_finer(oc, gpf, 64, seed=6, rounds=0)
    assert Xg.shape == (64, 2, wf.P, 3) and rej == 0
    assert int((gpf.fold_check(Xg) != 0).sum().item()) == 0
    refined = dsm.refine_population(w.mesh, _t(oc.archive_X)).cpu().numpy()
    got = Xg.cpu().numpy()
    assert all(np.any(np.all(refined == g, axis=(1, 2, 3))) for g in got)  # each a refined archive member


def test_device_archive_merge_equals_host():
    """The device archive (dsm_archive_merge) against the harness's host merge,
    with duplicates inside a batch and of archived points."""
    rng = np.random.default_rng(12)
    A = dsm.Archive(capacity=4096, m_max=300)
    host = np.zeros((0, 3))
    for step in range(6):
        new = rng.integers(0, 40, size=(300, 3)).astype(np.float64)  # many ties and duplicates
        new[:20] = new[20:40]  # exact duplicates within the batch
        if len(host):
            new[40:50] = host[rng.integers(0, len(host), 10)]  # duplicates of archived points
        host = O.merge_archive(host, new)
        A.merge(_t(new))
        n = A.n
        got = A.vec[:n].cpu().numpy()
        np.testing.assert_array_equal(got, host)
        assert torch.all(torch.isinf(A.vec[n:]))


def test_accept_tetrahedron_elements():
    """Elements of 4 points (one tetrahedron per cube of one class of cubes 3
    apart): accepted changes move all 4 points, the kept objectives and term
    cache equal a fresh full evaluation, and single-point elements through the
    CSR entry point give the same result as the single-point one."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S = X.shape[0]
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    Xd = _t(X)
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=DEV)
    obj, _ = gp.eval_full(Xd, tet_terms=cache)
    arch = _t(O.nondominated(obj.cpu().numpy()))
    cubes = O.cube_classes(w.mesh)[0]
    tets = gp.topology()["tets"]
    r = np.random.default_rng(9).integers(0, 6, size=len(cubes))
    pts_h = tets[6 * cubes + r].reshape(-1).astype(np.int32)
    off_h = (4 * np.arange(len(cubes) + 1)).astype(np.int32)
    pts, off = _t(pts_h), _t(off_h)
    _say(f"accept {len(cubes)} tetrahedron elements")
    cand = gp.sample_candidates(Xd, pts, 1, 1.5, 5, 1)
    terms_cand = torch.zeros_like(cache)
    old, new, fl, _ = gp.eval_partial(Xd, off, pts, cand, tet_terms_in=cache, tet_terms_new=terms_cand)
    acc = torch.empty((S, len(cubes)), dtype=torch.uint8, device=DEV)
    X1 = Xd.clone()
    gp.accept_elements(X1, off, pts, cand, old, new, fl, terms_cand, cache, obj, archive=arch, accepted=acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy().astype(bool)
    assert 0 < got.sum() < got.size
    Xn, cn = X1.cpu().numpy(), cand.cpu().numpy()
    for s in range(S):
        for f in range(len(cubes)):
            for j in range(off_h[f], off_h[f + 1]):
                p = pts_h[j]
                want = cn[s, j] if got[s, f] else X[s, :, p]
                assert np.array_equal(Xn[s, :, p], want)
    cache2 = torch.empty_like(cache)
    obj2, fl2 = gp.eval_full(X1, tet_terms=cache2)
    assert int((fl2 != 0).sum()) == 0
    np.testing.assert_allclose(obj.cpu().numpy(), obj2.cpu().numpy(), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(cache.cpu().numpy(), cache2.cpu().numpy(), rtol=1e-4, atol=1e-7)
    # single-point elements: the CSR entry point equals the single-point one
    cls = _t(O.parity_classes(w.mesh)[1])
    F = cls.shape[0]
    off1 = _t(np.arange(F + 1, dtype=np.int32))
    cache_a = torch.empty_like(cache)
    obj_a, _ = gp.eval_full(Xd, tet_terms=cache_a)
    cache_b, obj_b = cache_a.clone(), obj_a.clone()
    c1 = gp.sample_candidates(Xd, cls, 1, 2.0, 6, 2)
    tc = torch.zeros_like(cache)
    o1, n1, f1, _ = gp.eval_partial(Xd, off1, cls, c1, tet_terms_in=cache_a, tet_terms_new=tc)
    Xa, Xb = Xd.clone(), Xd.clone()
    aa = torch.empty((S, F), dtype=torch.uint8, device=DEV)
    ab = torch.empty_like(aa)
    gp.accept(Xa, cls, c1, o1, n1, f1, tc, cache_a, obj_a, archive=arch, accepted=aa)
    gp.accept_elements(Xb, off1, cls, c1, o1, n1, f1, tc, cache_b, obj_b, archive=arch, accepted=ab)
    for a, b in ((Xa, Xb), (cache_a, cache_b), (obj_a, obj_b), (aa, ab)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("sampler", ["isotropic", "estimated"])
def test_optimiser_tetrahedron_fos(sampler):
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    Xd = _t(X)
    _say(f"6 generations, tetrahedron FOS, {sampler} sampler")
    log, opt, _ = O.run(gp, Xd, 6, sigma=w.sigma_cand, seed=4, sampler=sampler, fos="tetrahedron")
    assert log.hypervolume[-1] > log.hypervolume[0] and sum(log.accepted) > 0
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    obj, flags = gp.eval_full(opt.X)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    with pytest.raises(ValueError):
        O.Optimiser(gp, Xd, fos="tetrahedron", graph=True)
