"""GPU distribution estimation and sampling for RV-GOMEA-style partial changes
of single-point elements, against the FP64 reference oracle/gomea_ref.py, and
a short optimiser run with the estimated sampler."""
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
    print(f"[gpu-gomea] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_estimate_matches_reference():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S = X.shape[0]
    gp = dsm.Problem.from_workload(w)
    pts = np.concatenate([np.arange(w.P), [-1, w.P]]).astype(np.int32)  # every point, plus two invalid ones
    sel = np.array(list(range(0, S, 3)) + [-5, S, S + 7], dtype=np.int32)  # out-of-range indices are skipped
    _say(f"estimate {len(pts)} elements over {len(sel)} indices")
    mean, chol = gp.estimate_distributions(_t(X), _t(sel), _t(pts))
    rmean, _, rchol = G.estimate(X, sel, pts, w.mesh)
    np.testing.assert_allclose(mean.cpu().numpy(), rmean, rtol=1e-12, atol=1e-12)
    rpacked = np.array([G.packed_lower(L) for L in rchol])
    np.testing.assert_allclose(chol.cpu().numpy(), rpacked, rtol=1e-9, atol=1e-12)
    assert np.all(mean.cpu().numpy()[-2:] == 0) and np.all(chol.cpu().numpy()[-2:] == 0)
    # no valid solution: zeros
    m0, c0 = gp.estimate_distributions(_t(X), _t(np.array([-1, S], dtype=np.int32)), _t(pts[:5]))
    assert torch.all(m0 == 0) and torch.all(c0 == 0)


def test_sampler_distribution():
    w = W.batched()
    gp = dsm.Problem.from_workload(w)
    I = gp.topology()["identity"]
    S, K = 16, 512
    X = np.repeat(np.stack([I, I])[None], S, axis=0)
    # an interior point, a face point (one pinned axis) and an edge point (two pinned axes)
    pts = np.array([1 + 5 * (2 + 5 * 2), 2 + 5 * (2 + 5 * 0), 0 + 5 * (2 + 5 * 0)], dtype=np.int32)
    rng = np.random.default_rng(4)
    F = len(pts)
    mean = np.zeros((F, 6))
    Ls = np.zeros((F, 6, 6))
    for f, p in enumerate(pts):
        fr = G.free_axes(p, w.mesh)
        mean[f] = np.concatenate([I[p], I[p]]) + rng.uniform(-2, 2, 6) * fr
        A = rng.normal(0, 1.0, (6, 6)) * fr[:, None] * fr[None, :]
        C = A @ A.T + np.diag(0.3 * fr)
        Ls[f] = G.cholesky_semidefinite(C)
    packed = np.array([G.packed_lower(L) for L in Ls])
    mult = np.array([1.0, 0.25, 2.0], dtype=np.float32)
    _say("sample 8192 candidates per element")
    cand = gp.sample_estimated(_t(X), _t(pts), K, _t(mean), _t(packed), _t(mult), 99, 3).cpu().numpy()
    again = gp.sample_estimated(_t(X), _t(pts), K, _t(mean), _t(packed), _t(mult), 99, 3).cpu().numpy()
    other = gp.sample_estimated(_t(X), _t(pts), K, _t(mean), _t(packed), _t(mult), 99, 4).cpu().numpy()
    assert np.array_equal(cand, again) and not np.array_equal(cand, other)
    assert np.all(np.rint((cand + 0.5) * 128) == (cand + 0.5) * 128)
    hi = np.array(w.dims) - 0.5
    assert np.all(cand >= -0.5) and np.all(cand <= np.concatenate([hi, hi]).reshape(2, 3))
    for f, p in enumerate(pts):
        fr = G.free_axes(p, w.mesh)
        x = cand[:, f].reshape(-1, 6).astype(np.float64)  # [S*K][6]
        cur = np.concatenate([I[p], I[p]])
        assert np.all(x[:, ~fr] == cur[~fr])
        C = mult[f] * Ls[f] @ Ls[f].T
        sd = np.sqrt(np.diag(C))
        n = len(x)
        free = np.nonzero(fr)[0]
        # the box clamp is far (the point is at least 2 cube widths from it at these scales)
        assert np.all(np.abs(x[:, free].mean(axis=0) - mean[f, free]) < 5 * sd[free] / np.sqrt(n) + 0.01)
        emp = np.cov(x[:, free].T, bias=True)
        assert np.allclose(emp, C[np.ix_(free, free)], atol=0.08 * sd[free].max() ** 2)


def test_optimiser_with_estimated_sampler():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    gp = dsm.Problem.from_workload(w)
    Xd = _t(X)
    _say("8 generations, estimated sampler")
    log, opt, _ = O.run(gp, Xd, 8, sigma=w.sigma_cand, seed=3, sampler="estimated")
    assert log.hypervolume[-1] > log.hypervolume[0]
    assert sum(log.accepted) > 0
    assert int((gp.fold_check(opt.X) != 0).sum().item()) == 0
    # objectives kept by the generation steps equal a fresh full evaluation
    obj, flags = gp.eval_full(opt.X)
    assert int((flags != 0).sum().item()) == 0
    np.testing.assert_allclose(opt.obj.cpu().numpy(), obj.cpu().numpy(), rtol=1e-5, atol=1e-9)
    # selection: tau of the population, distinct indices, none dominated by an unselected solution
    sel = opt.select().cpu().numpy()
    assert len(sel) == round(0.35 * opt.S) and len(set(sel.tolist())) == len(sel)
    o = opt.obj.cpu().numpy()
    rest = np.setdiff1d(np.arange(opt.S), sel)
    dom = lambda i: int(np.sum(np.all(o <= o[i], axis=1) & np.any(o < o[i], axis=1)))
    assert max(dom(i) for i in sel) <= min(dom(i) for i in rest)
    with pytest.raises(ValueError):
        O.Optimiser(gp, Xd, sampler="estimated", graph=True)


def test_estimate_elements_matches_reference():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S = X.shape[0]
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    tets = gp.topology()["tets"]
    cubes = O.cube_classes(w.mesh)[0]
    r = np.random.default_rng(2).integers(0, 6, size=len(cubes))
    pts = list(tets[6 * cubes + r].reshape(-1))
    off = list(4 * np.arange(len(cubes) + 1))
    # a one-point element, a 5-point one, one with an invalid point, an empty one
    for extra in ([37], [1, 2, 3, 4, 5], [6, -1], []):
        pts += extra
        off.append(off[-1] + len(extra))
    off, pts = np.array(off, dtype=np.int32), np.array(pts, dtype=np.int32)
    sel = np.array(list(range(0, S, 2)) + [-3, S], dtype=np.int32)
    _say(f"estimate {len(off) - 1} elements jointly")
    mean, chol = gp.estimate_elements(_t(X), _t(sel), _t(off), _t(pts))
    rmean, _, rchol = G.estimate_elements(X, sel, off, pts, w.mesh)
    np.testing.assert_allclose(mean.cpu().numpy(), rmean, rtol=1e-12, atol=1e-12)
    rpacked = np.array([G.packed_lower(L) for L in rchol])
    np.testing.assert_allclose(chol.cpu().numpy(), rpacked, rtol=1e-8, atol=1e-10)
    assert np.all(mean.cpu().numpy()[-3:] == 0) and np.all(chol.cpu().numpy()[-3:] == 0)


def test_sample_elements_joint_distribution():
    w = W.batched()
    gp = dsm.Problem.from_workload(w, max_fos_points=4)
    I = gp.topology()["identity"]
    S = 4096
    X = np.repeat(np.stack([I, I])[None], S, axis=0)
    # one interior tetrahedron-like element of 4 points, one of them on a face (z pinned)
    ps = np.array([1 + 5 * (2 + 5 * 2), 2 + 5 * (2 + 5 * 2), 2 + 5 * (3 + 5 * 2), 2 + 5 * (2 + 5 * 0)], dtype=np.int32)
    off = np.array([0, 4], dtype=np.int32)
    free = np.concatenate([G.free_axes(p, w.mesh) for p in ps])
    rng = np.random.default_rng(8)
    A = rng.normal(0, 0.6, (24, 24)) * free[:, None] * free[None, :]
    C = A @ A.T + np.diag(0.2 * free)
    L = G.cholesky_semidefinite(C)
    mean = np.concatenate([np.concatenate([I[p], I[p]]) for p in ps]) + rng.uniform(-1, 1, 24) * free
    mult = np.array([0.5], dtype=np.float32)
    _say(f"sample {S} joint candidates")
    cand = gp.sample_elements(_t(X), _t(off), _t(ps), _t(mean[None]), _t(G.packed_lower(L)[None]), _t(mult), 17, 2)
    x = cand.cpu().numpy().reshape(S, 24).astype(np.float64)
    cur = np.concatenate([np.concatenate([I[p], I[p]]) for p in ps])
    assert np.all(x[:, ~free] == cur[~free])
    assert np.all(np.rint((x + 0.5) * 128) == (x + 0.5) * 128)
    fr = np.nonzero(free)[0]
    Cm = mult[0] * C
    sd = np.sqrt(np.diag(Cm))
    assert np.all(np.abs(x[:, fr].mean(axis=0) - mean[fr]) < 5 * sd[fr] / np.sqrt(S) + 0.01)
    emp = np.cov(x[:, fr].T, bias=True)
    assert np.allclose(emp, Cm[np.ix_(fr, fr)], atol=0.1 * sd[fr].max() ** 2)
    # a rejected element (5 points) gets NaN candidates
    off5 = np.array([0, 5], dtype=np.int32)
    p5 = np.array([ps[0], ps[1], ps[2], ps[3], 7], dtype=np.int32)
    c5 = gp.sample_elements(_t(X[:2]), _t(off5), _t(p5), _t(np.zeros((1, 24))), _t(np.zeros((1, 300))),
                            _t(mult), 1, 1)
    assert torch.all(torch.isnan(c5))
