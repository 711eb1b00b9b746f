"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  Voxel sets and constraint flags bit-exact; every
objective within 1e-5 relative (absolute floor 1e-7); deltas of partial
changes within 1e-5 (|old| + |new|)."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W
from tests._common import (assert_delta_close, assert_objectives_close, feasible_population,
                           oracle_problem)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-parity] {msg}", file=sys.stderr, flush=True)


def _gpu_problem(w, S, F=None, max_fos_points=1):
    return dsm.Problem.from_workload(w, max_solutions=S, max_fos=w.P if F is None else F,
                                     max_fos_points=max_fos_points)


def _t(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _small_workload(dims=(20, 18, 14), mesh=(4, 3, 3), seed=0, spacing=(1.0, 1.2, 2.0), tau=0.15, S=6):
    rng = np.random.default_rng(seed)
    shp = dims[::-1]
    fixed = W._blur(rng.uniform(0, 1, shp) * (rng.uniform(0, 1, shp) > 0.3), 1.0).astype(np.float32)
    moving = W._blur(rng.uniform(0, 1, shp) * (rng.uniform(0, 1, shp) > 0.3), 1.0).astype(np.float32)
    hi = np.array(dims) - 1.0
    gm = W.snap(rng.uniform(0, 1, (5, 3)) * hi)
    gf = W.snap(rng.uniform(0, 1, (6, 3)) * hi)
    return W.Workload(f"random-{dims}", moving, fixed, mesh, spacing, tau, S, 1.2, 1.0, seed + 1, seed + 2,
                      gm, gf, np.array([0, 1, 2, 2, 3], np.int32), np.array([0, 1, 1, 2, 3, 3], np.int32))


# ---------------------------------------------------------------- rasterisation

@pytest.mark.parametrize("dims,mesh,sigma", [((33, 33, 33), (3, 3, 3), 0.0), ((33, 33, 33), (3, 3, 3), 3.0),
                                             ((37, 23, 19), (5, 4, 3), 1.5), ((2, 2, 2), (2, 2, 2), 0.0),
                                             ((64, 64, 64), (5, 5, 5), 1.0), ((17, 9, 25), (3, 2, 4), 0.0)])
def test_owner_map_bitexact(dims, mesh, sigma):
    _say(f"owner map dims={dims} mesh={mesh} sigma={sigma}")
    z = np.zeros(dims[::-1], np.float32)
    rp = ref.Problem(z, z, mesh)
    if sigma > 0:
        X = W.population(dims, mesh, 2, sigma, 5, reject=lambda X: rp.fold_check(X)[0] != 0)
    else:
        X = np.stack([rp.identity(), rp.identity()])[None]
    gp = dsm.Problem(z, z, mesh, max_solutions=1)
    for g in range(2):
        owner, overlap = gp.rasterize_owner(_t(X[0, g]))
        torch.cuda.synchronize()
        ro, rc = rp.owner_bruteforce(X[0, g])
        assert int(overlap.item()) == 0
        np.testing.assert_array_equal(owner.cpu().numpy(), ro)


# ---------------------------------------------------------------- fold check

def test_fold_flags_bitexact():
    w = _small_workload(dims=(24, 24, 24), mesh=(4, 4, 4))
    rp = oracle_problem(w)
    I = rp.identity()
    base = np.stack([I, I])
    cases = [base.copy()]
    v = 1 + 4 * (1 + 4 * 1)
    for (g, p, a, val) in [(0, v, 0, None), (1, v, 0, None), (0, 4 * (1 + 4 * 1), 0, 0.5),
                           (1, 3 + 4 * (2 + 4 * 1), 0, 22.0), (1, v, 2, -3.0), (1, v, 1, 1.0 / 256), (0, v, 1, np.nan),
                           (0, v, 1, np.inf)]:
        Y = base.copy()
        if val is None:
            Y[g, p, a] = Y[g, p + 1, a] + 1.0
        elif val == 1.0 / 256:
            Y[g, p, a] += val
        else:
            Y[g, p, a] = val
        cases.append(Y)
    rng = np.random.default_rng(3)
    for k in range(20):  # random large perturbations: many folds
        cases.append(W.population(w.dims, w.mesh, 1, 4.0, 100 + k)[0])
    X = np.stack(cases).astype(np.float32)
    _say(f"fold flags S={len(X)}")
    gp = _gpu_problem(w, len(X))
    flags, fb = gp.fold_check(_t(X), first_bad=True)
    torch.cuda.synchronize()
    rf, rfb = rp.fold_check(X)
    np.testing.assert_array_equal(flags.cpu().numpy().astype(np.uint32), rf)
    np.testing.assert_array_equal(fb.cpu().numpy(), rfb)
    assert (rf != 0).sum() > 10


# ---------------------------------------------------------------- full evaluation

@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("which", ["tiny", "random", "random_aniso"])
def test_full_eval(which, order):
    """Full evaluation against the oracle, with rows swept slice by slice and
    in slice pairs."""
    if which == "tiny":
        w = W.tiny()
    elif which == "random":
        w = _small_workload()
    else:
        w = _small_workload(dims=(37, 23, 19), mesh=(5, 4, 3), spacing=(0.7, 1.1, 2.5), seed=4)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    X[0] = np.stack([rp.identity(), rp.identity()])
    _say(f"full eval {w.name} S={len(X)} row order {order}")
    gp = _gpu_problem(w, len(X))
    gp.set_row_order(order)
    terms = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
    obj, flags = gp.eval_full(_t(X), tet_terms=terms)
    torch.cuda.synchronize()
    robj, rflags, rterms, _ = rp.eval_full(X, want_terms=True)
    np.testing.assert_array_equal(flags.cpu().numpy().astype(np.uint32), rflags)
    assert_objectives_close(obj.cpu().numpy(), robj, what="full objectives")
    # per-tetrahedron terms: absolute tolerance relative to the solution total
    tt = terms.cpu().numpy()
    tol = 1e-5 * np.abs(rterms).sum(axis=1, keepdims=True) / gp.T + 1e-9
    assert np.all(np.abs(tt - rterms) <= tol + 1e-5 * np.abs(rterms))


def test_identity_closed_forms_gpu():
    """Identity mesh and identical images: every objective 0 (GPU floor 1e-7)."""
    img = W._blur(np.random.default_rng(1).uniform(0, 1, (12, 14, 16)), 1.0).astype(np.float32)
    gp = dsm.Problem(img, img, (3, 4, 3), tau=0.2, max_solutions=1)
    I = gp.topology()["identity"]
    obj, flags = gp.eval_full(_t(np.stack([I, I])[None]))
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    assert np.all(np.abs(obj.cpu().numpy()) <= 1e-7)


# ---------------------------------------------------------------- partial evaluation

_SINGLE_POINT_CASES = ([(w, c, 0) for w in ("tiny", "random", "tall", "very_tall") for c in (True, False)] +
                       [(w, True, 1) for w in ("tiny", "random", "tall", "very_tall")])


@pytest.mark.parametrize("which,use_cache,order", _SINGLE_POINT_CASES)
def test_partial_single_point(which, use_cache, order):
    """Every (solution, single-point element) pair against the oracle.  The
    tall workloads have tetrahedra spanning up to about 60 slices (slice tables
    built in four rounds of 16 lanes, and with order 1 slice pairs within each
    round, the last pair of an odd count a single slice) and about 75 slices
    (more than the 64-slice table: rows enumerated over the bounding box)."""
    if which == "tiny":
        w = W.tiny()
    elif which == "random":
        w = _small_workload()
    elif which == "tall":
        w = _small_workload(dims=(22, 18, 118), mesh=(3, 3, 3), seed=6)
    else:
        w = _small_workload(dims=(18, 16, 150), mesh=(3, 3, 3), seed=7)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    _say(f"partial {w.name} S={len(X)} F={len(off) - 1} cache={use_cache} row order {order}")
    robj, rflags, rterms, _ = rp.eval_full(X, want_terms=True)
    rold, rnew, rfl, rnv = rp.eval_partial(X, off, pts, cand, tet_terms=rterms if use_cache else None)
    gp = _gpu_problem(w, len(X))
    gp.set_row_order(order)
    Xd = _t(X)
    cache = None
    if use_cache:
        cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
        gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    fl = fl.cpu().numpy().astype(np.uint32)
    np.testing.assert_array_equal(fl, rfl)
    np.testing.assert_array_equal(vc.cpu().numpy()[fl == 0], rnv[fl == 0])
    assert_objectives_close(new.cpu().numpy(), rnew, flags=fl, what="part_new")
    assert_objectives_close(old.cpu().numpy(), rold, what="part_old")
    assert_delta_close(old.cpu().numpy(), new.cpu().numpy(), rold, rnew, fl)


def test_partial_multi_point_fos_and_edge_cases():
    """FOS elements of several points (one tetrahedron per cube, Sec. 2.2),
    an empty element, a malformed element, and candidates that fold or leave
    the lattice."""
    w = _small_workload(dims=(26, 22, 18), mesh=(4, 4, 3), seed=7)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    tets = rp.tets()
    rng = np.random.default_rng(9)
    elems = [list(tets[6 * c + rng.integers(6)]) for c in range(0, (w.mesh[0] - 1) * (w.mesh[1] - 1) * (w.mesh[2] - 1), 2)]
    elems.append([])              # empty element
    elems.append([0, 1, 2, 3, 5, 6, 7])
    good = len(elems)
    off = np.zeros(good + 1, np.int32)
    for i, e in enumerate(elems):
        off[i + 1] = off[i] + len(e)
    pts = np.concatenate([np.asarray(e, np.int32) for e in elems]).astype(np.int32)
    cand = W.candidates(X, off, pts, w.mesh, w.dims, 2.5, 77)
    # plant infeasible candidates: a NaN, an off-lattice value, a far jump
    cand[0, 0, 0, 0] = np.nan
    cand[1, 1, 1, 2] += 1.0 / 1024
    cand[2, 2, 0, 1] = cand[2, 2, 0, 1] + 15.0
    _say(f"partial multi-point S={len(X)} F={good}")
    rterms = rp.eval_full(X, want_terms=True)[2]
    rold, rnew, rfl, rnv = rp.eval_partial(X, off, pts, cand, tet_terms=rterms)
    gp = _gpu_problem(w, len(X), F=good + 1, max_fos_points=7)
    Xd = _t(X)
    cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
    gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    fl = fl.cpu().numpy().astype(np.uint32)
    np.testing.assert_array_equal(fl, rfl)
    assert (fl != 0).sum() >= 3
    np.testing.assert_array_equal(vc.cpu().numpy()[fl == 0], rnv[fl == 0])
    assert_objectives_close(new.cpu().numpy(), rnew, flags=fl, what="part_new")
    assert_objectives_close(old.cpu().numpy(), rold, what="part_old")
    # malformed element: point index out of range, and one above max_fos_points
    off2 = np.array([0, 1, 9], np.int32)
    pts2 = np.array([rp.P + 3, 0, 1, 2, 3, 4, 5, 6, 7], np.int32)
    cand2 = np.repeat(X[:, :, :1].transpose(0, 2, 1, 3), 9, axis=1).copy()
    old2, new2, fl2, _ = gp.eval_partial(Xd, _t(off2), _t(pts2), _t(cand2), tet_terms_in=cache)
    torch.cuda.synchronize()
    assert np.all(fl2.cpu().numpy() == dsm.FLAG_BAD_FOS)


def test_partial_full_consistency_gpu():
    """full(new) = full(old) - part_old + part_new on the GPU, and the written
    candidate terms equal a full evaluation of the changed solution."""
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    gp = _gpu_problem(w, len(X))
    Xd = _t(X)
    cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
    obj, _ = gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, _ = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache)
    f = 13  # the centre point: its star is every tetrahedron
    Y = X.copy()
    Y[:, :, f] = cand[:, f]
    obj2, fl2 = gp.eval_full(_t(Y))
    torch.cuda.synchronize()
    ok = (fl.cpu().numpy()[:, f] == 0)
    lhs = obj2.cpu().numpy()[ok]
    rhs = (obj.cpu().numpy() - old.cpu().numpy()[:, f] + new.cpu().numpy()[:, f])[ok]
    assert ok.sum() > 5
    np.testing.assert_allclose(lhs, rhs, rtol=1e-5, atol=1e-7)


def test_determinism():
    w = _small_workload(seed=11)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    gp = _gpu_problem(w, len(X))
    Xd, od, pd, cd = _t(X), _t(off), _t(pts), _t(cand)
    r1 = [t.cpu().numpy() for t in gp.eval_partial(Xd, od, pd, cd)[:3]]
    r2 = [t.cpu().numpy() for t in gp.eval_partial(Xd, od, pd, cd)[:3]]
    for a, b in zip(r1, r2):
        np.testing.assert_array_equal(a, b)


def test_batched_all_pairs():
    """64^3 blurred-ellipsoid pair, 5^3 meshes, 96 solutions x 125 single-point
    elements in one launch; the oracle recomputes every full evaluation and
    every one of the 12,000 (solution, element) pairs, against which both
    row orders of the sweep are checked."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    _say(f"batched {w.name} S={len(X)} F={len(off) - 1}")
    gp = _gpu_problem(w, len(X))
    Xd = _t(X)
    cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    _say("batched: oracle on all pairs")
    robj, rflags, rterms, _ = rp.eval_full(X, want_terms=True)
    np.testing.assert_array_equal(flags.cpu().numpy().astype(np.uint32), rflags)
    assert_objectives_close(obj.cpu().numpy(), robj, what="full objectives")
    rold, rnew, rfl, rnv = rp.eval_partial(X, off, pts, cand, tet_terms=rterms)
    flg = fl.cpu().numpy().astype(np.uint32)
    np.testing.assert_array_equal(flg, rfl)
    assert (flg == 0).sum() > 0.5 * flg.size
    np.testing.assert_array_equal(vc.cpu().numpy()[flg == 0], rnv[flg == 0])
    assert_objectives_close(new.cpu().numpy(), rnew, flags=flg, what="part_new")
    assert_objectives_close(old.cpu().numpy(), rold, what="part_old")
    assert_delta_close(old.cpu().numpy(), new.cpu().numpy(), rold, rnew, flg)
    # exactly-once coverage: every single-point element's samples add up to 8 V per solution
    vcs = vc.cpu().numpy().astype(np.int64)
    allok = (flg == 0).all(axis=1)
    assert np.all(vcs[allok].sum(axis=1) == 8 * gp.V)
    _say("batched: rows in slice pairs")
    gp.set_row_order(1)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(flags.cpu().numpy().astype(np.uint32), rflags)
    assert_objectives_close(obj.cpu().numpy(), robj, what="full objectives, slice pairs")
    np.testing.assert_array_equal(fl.cpu().numpy().astype(np.uint32), rfl)
    np.testing.assert_array_equal(vc.cpu().numpy()[flg == 0], rnv[flg == 0])
    assert_objectives_close(new.cpu().numpy(), rnew, flags=flg, what="part_new, slice pairs")
    assert_objectives_close(old.cpu().numpy(), rold, what="part_old, slice pairs")


def test_clinical_full_size_all_elements():
    """512x512x100 clinical-shaped workload in the benchmark's launch
    configuration (512 solutions x 600 single-point elements in one launch,
    cached old terms); the oracle recomputes the full evaluation and all 600
    elements (every star size, 2 to 48 tetrahedra) of 4 solutions.  Checked
    with the defaults (8 tetrahedra per workgroup, rows by slice) and with the
    setting the benchmark's autotuners keep on this workload (4, slice
    pairs)."""
    w = W.clinical()
    _say(f"clinical full size {w.name}")
    gp = _gpu_problem(w, w.S)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    Xd = _t(X)
    cache = torch.empty((w.S, gp.T, 3), dtype=torch.float64, device=DEV)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    assert int((flags != 0).sum()) == 0
    vcs = vc.cpu().numpy().astype(np.int64)
    fln = fl.cpu().numpy().astype(np.uint32)
    allok = (fln == 0).all(axis=1)
    assert np.all(vcs[allok].sum(axis=1) == 8 * gp.V)  # exactly-once coverage, both grids, every star
    star_off, _ = rp.star()
    assert sorted(set(np.diff(star_off).tolist())) == [2, 4, 6, 8, 12, 16, 24, 48]
    rng = np.random.default_rng(0)
    sols = np.sort(rng.choice(w.S, 4, replace=False))
    _say(f"clinical: oracle on all {w.P} elements of solutions {sols.tolist()}")
    robj, rflags, rterms, _ = rp.eval_full(X[sols], want_terms=True)
    assert_objectives_close(obj.cpu().numpy()[sols], robj, what="full objectives")
    rold, rnew, rfl, rnv = rp.eval_partial(X[sols], off, pts, cand[sols], tet_terms=rterms)
    g_fl = fln[sols]
    np.testing.assert_array_equal(g_fl, rfl)
    assert (g_fl == 0).sum() > 0.5 * g_fl.size
    np.testing.assert_array_equal(vcs[sols][g_fl == 0], rnv[g_fl == 0])
    assert_objectives_close(new.cpu().numpy()[sols], rnew, flags=g_fl, what="part_new")
    assert_objectives_close(old.cpu().numpy()[sols], rold, what="part_old")
    assert_delta_close(old.cpu().numpy()[sols], new.cpu().numpy()[sols], rold, rnew, g_fl)
    _say("clinical: chunk 4, rows in slice pairs")
    gp.set_part_chunk(4)
    gp.set_row_order(1)
    obj, flags = gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    assert_objectives_close(obj.cpu().numpy()[sols], robj, what="full objectives, slice pairs")
    np.testing.assert_array_equal(fl.cpu().numpy().astype(np.uint32), fln)
    np.testing.assert_array_equal(vc.cpu().numpy().astype(np.int64), vcs)
    assert_objectives_close(new.cpu().numpy()[sols], rnew, flags=g_fl, what="part_new, chunk 4, slice pairs")
    assert_objectives_close(old.cpu().numpy()[sols], rold, what="part_old, chunk 4, slice pairs")
    assert_delta_close(old.cpu().numpy()[sols], new.cpu().numpy()[sols], rold, rnew, g_fl)


def test_clinical_tetrahedron_voxel_sets_bitexact():
    """512x512x100, deformed feasible grids of two solutions: the GPU's
    rasterised owner map covers every voxel exactly once, and the voxel set
    of each of 150 tetrahedra per grid (border, corner and interior cubes)
    equals the oracle's scan of its bounding box, voxel for voxel."""
    w = W.clinical()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=2)
    gp = _gpu_problem(w, 2)
    rng = np.random.default_rng(5)
    T = rp.T
    corner = [0, 1, 2, 3, 4, 5, T - 6, T - 5, T - 4, T - 3, T - 2, T - 1]
    for s in range(2):
        for g in range(2):
            owner, overlap = gp.rasterize_owner(_t(X[s, g]))
            torch.cuda.synchronize()
            assert int(overlap.item()) == 0
            own = owner.cpu().numpy().ravel()
            assert own.min() >= 0
            order = np.argsort(own, kind="stable")
            bounds = np.searchsorted(own[order], np.arange(T + 1))
            tets = np.unique(np.concatenate([corner, rng.choice(T, 138, replace=False)]))
            _say(f"tetrahedron voxel sets: solution {s} grid {g}, {len(tets)} tetrahedra")
            for t in tets:
                mine = np.sort(order[bounds[t]:bounds[t + 1]])
                theirs = np.sort(rp.tet_voxels(X[s, g], int(t)))
                assert len(mine) == len(theirs) and np.array_equal(mine, theirs), (s, g, int(t))


@pytest.mark.parametrize("level", [0, 1])
def test_uneven_batch_one_launch(level):
    """Problems of uneven volume and mesh size evaluated in one fused launch:
    results identical to one launch per problem; a sample checked against the
    oracle.  Level 0 is the 2x box-averaged pyramid level; level 1 starts from
    its population handed off to full resolution."""
    idx = [0, 3, 6, 9] if level == 1 else [0, 3, 6, 9, 10]
    ws = W.uneven(idx, level=level)
    jobs, single, probs = [], [], []
    batch = dsm.Batch(max_jobs=len(ws))
    for i, w in zip(idx, ws):
        rp = oracle_problem(w)
        if level == 0:
            X = feasible_population(w, rp)
        else:
            # hand-off: a feasible half-resolution population mapped to full resolution stays feasible
            wh = W.uneven([i], level=0)[0]
            X = W.upsample_population(feasible_population(wh, oracle_problem(wh)))
            assert np.all(rp.fold_check(X)[0] == 0)
        off, pts = w.fos()
        cand = w.candidates(X, off, pts)
        gp = _gpu_problem(w, len(X))
        gp.set_part_chunk(4 + len(probs) % 5)  # every problem its own work split
        gp.set_row_order(len(probs) % 2)        # and rows by slice or by slice pair
        probs.append((w, rp, X, off, pts, cand, gp))
        Xd = _t(X)
        cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
        gp.eval_full(Xd, tet_terms=cache)
        jobs.append(dict(problem=gp, X=Xd, fos_off=_t(off), fos_pts=_t(pts), cand=_t(cand), tet_terms_in=cache))
        single.append(gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True))
    _say(f"uneven batch level {level}: {[w.name for w in ws]}")
    outs = batch.eval_partial(jobs)
    torch.cuda.synchronize()
    for o, sgl in zip(outs, single):
        for a, b in zip(o, sgl):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    rng = np.random.default_rng(level)
    for (w, rp, X, off, pts, cand, gp), o in zip(probs, outs):
        s = int(rng.integers(len(X)))
        elems = np.sort(rng.choice(w.P, 5, replace=False)).astype(np.int32)
        rold, rnew, rfl, rnv = rp.eval_partial(X[s:s + 1], np.arange(6, dtype=np.int32), elems, cand[s:s + 1, elems])
        g_fl = o[2].cpu().numpy()[s, elems][None].astype(np.uint32)
        np.testing.assert_array_equal(g_fl, rfl)
        assert_objectives_close(o[1].cpu().numpy()[s, elems][None], rnew, flags=g_fl, what=f"{w.name} part_new")
        assert_objectives_close(o[0].cpu().numpy()[s, elems][None], rold, what=f"{w.name} part_old")


def test_layout_pitch_changes_nothing():
    """The row pitch of the device image layout changes no result bit, and
    the autotuner keeps one of its candidates."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    gp = _gpu_problem(w, len(X))
    Xd, offd, ptsd, cd = _t(X), _t(off), _t(pts), _t(cand)
    Dx = w.dims[0]

    def run():
        obj, fl = gp.eval_full(Xd)
        res = gp.eval_partial(Xd, offd, ptsd, cd, voxel_count=True)
        torch.cuda.synchronize()
        return [obj.cpu().numpy(), fl.cpu().numpy()] + [r.cpu().numpy() for r in res]

    _say(f"pitch default {gp.pitch}")
    ref_out = run()
    for pitch in (Dx + 2, Dx + 13, Dx + 2 + 64, 0):
        gp.set_pitch(pitch)
        assert gp.pitch == (pitch if pitch else ref_pitch_default(Dx))
        for a, b in zip(run(), ref_out):
            np.testing.assert_array_equal(a, b)
    cands = [Dx + 2, Dx + 6, Dx + 10]
    best, table = gp.autotune_pitch(Xd, offd, ptsd, cd, pitches=cands)
    assert best in cands and gp.pitch == best and len(table) == 3 and all(t > 0 for t in table.values())
    for a, b in zip(run(), ref_out):
        np.testing.assert_array_equal(a, b)
    with pytest.raises(dsm.DsmError):
        gp.set_pitch(Dx + 1)


# Two work splits or row orders sum the same FP32 contributions in different
# orders.  Each per-lane compensated FP32 sum is within 2u|S| of the exact sum
# of its (positive) contributions, u = 2^-24, and the lanes' sums are combined
# in FP64, so each result is within 2u relative of the exact sum of the same
# contributions and two splits differ by at most 4u = 2.4e-7 relative (plus
# the second-order terms of compensated summation and the FP64 combination:
# the 25 % margin).
_SPLIT_RTOL = 4 * 2.0 ** -24 * 1.25


def test_part_chunk_changes_no_voxel_set():
    """The affected tetrahedra per workgroup (4..8) change no flag and no voxel
    count, and the terms only by rounding: the voxels a wave sums in its
    per-lane compensated FP32 sums follow the work split (measured differences
    below 4e-9 relative for the element sums, 1e-7 for single tetrahedra;
    bound _SPLIT_RTOL); the chunk autotuner keeps one of its candidates; the
    allocation-free entry point follows the problem's chunk bit for bit."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)[:48]
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    gp = _gpu_problem(w, len(X))
    assert gp.part_chunk == 8
    Xd, offd, ptsd, cd = _t(X), _t(off), _t(pts), _t(cand)
    cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
    gp.eval_full(Xd, tet_terms=cache)

    def run(noalloc=False):
        f = gp.eval_partial_noalloc if noalloc else gp.eval_partial
        res = f(Xd, offd, ptsd, cd, tet_terms_in=cache, voxel_count=True)
        torch.cuda.synchronize()
        return [r.cpu().numpy() for r in res]

    ref8 = run()
    assert gp.max_star > 8  # several chunks per element at every chunk size tried
    for chunk in (4, 5, 6, 7, 8):
        gp.set_part_chunk(chunk)
        assert gp.part_chunk == chunk
        got = run()
        _say(f"part chunk {chunk}")
        np.testing.assert_array_equal(got[2], ref8[2])
        np.testing.assert_array_equal(got[3], ref8[3])
        for a, b in zip(got[:2], ref8[:2]):
            np.testing.assert_allclose(a, b, rtol=_SPLIT_RTOL, atol=1e-12)
        for a, b in zip(run(noalloc=True), got):
            np.testing.assert_array_equal(a, b)
    for bad in (3, 9):
        with pytest.raises(dsm.DsmError):
            gp.set_part_chunk(bad)
    assert gp.part_chunk == 8
    best, table = gp.autotune_chunk(Xd, offd, ptsd, cd, tet_terms_in=cache, chunks=[5, 8])
    assert best in (5, 8) and gp.part_chunk == best and sorted(table) == [5, 8] and all(t > 0 for t in table.values())


def test_row_order_changes_no_voxel_set():
    """Sweeping rows in slice pairs instead of slice by slice changes no flag
    and no voxel count, full or partial, and the terms only by rounding (the
    per-lane FP32 sums follow the order); the allocation-free entry point
    follows the problem's order bit for bit; the autotuner keeps one order."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)[:48]
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    gp = _gpu_problem(w, len(X))
    assert gp.row_order == 0
    Xd, offd, ptsd, cd = _t(X), _t(off), _t(pts), _t(cand)
    cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)

    def run(noalloc=False):
        obj, fl = gp.eval_full(Xd, tet_terms=cache)
        f = gp.eval_partial_noalloc if noalloc else gp.eval_partial
        res = f(Xd, offd, ptsd, cd, tet_terms_in=cache, voxel_count=True)
        torch.cuda.synchronize()
        return [obj.cpu().numpy(), fl.cpu().numpy(), cache.cpu().numpy()] + [r.cpu().numpy() for r in res]

    ref = run()
    for order in (1, 0, 1):
        gp.set_row_order(order)
        assert gp.row_order == order
        _say(f"row order {order}")
        got = run()
        for i in (1, 5, 6):  # full flags, partial flags, voxel counts
            np.testing.assert_array_equal(got[i], ref[i])
        for i in (0, 2, 3, 4):  # full objectives, terms, part_old, part_new
            np.testing.assert_allclose(got[i], ref[i], rtol=_SPLIT_RTOL, atol=1e-12)
        for a, b in zip(run(noalloc=True), got):
            np.testing.assert_array_equal(a, b)
    for bad in (-1, 2):
        with pytest.raises(dsm.DsmError):
            gp.set_row_order(bad)
    assert gp.row_order == 1
    best, table = gp.autotune_row_order(Xd, offd, ptsd, cd, tet_terms_in=cache)
    assert best in (0, 1) and gp.row_order == best and sorted(table) == [0, 1] and all(t > 0 for t in table.values())


def ref_pitch_default(Dx):
    """Smallest pitch >= Dx + 2 that is 8 mod 16."""
    p = Dx + 2
    while p % 16 != 8:
        p += 1
    return p


def test_tetrahedron_fos_clinical_sampled():
    """The paper's FOS (per cube one tetrahedron, its 4 points move together)
    at 512x512x100 in one launch of all elements and solutions; a sample of
    (solution, element) pairs is recomputed by the oracle."""
    w = W.clinical()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    n_cubes = rp.T // 6
    off, pts = W.tetrahedron_fos(rp.tets(), n_cubes, seed=41)
    cand = w.candidates(X, off, pts)
    _say(f"tetrahedron FOS at {w.name}: {n_cubes} elements x {w.S} solutions")
    gp = _gpu_problem(w, w.S, F=n_cubes, max_fos_points=4)
    Xd = _t(X)
    cache = torch.empty((w.S, gp.T, 3), dtype=torch.float64, device=DEV)
    gp.eval_full(Xd, tet_terms=cache)
    old, new, fl, vc = gp.eval_partial(Xd, _t(off), _t(pts), _t(cand), tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for s in rng.choice(w.S, 2, replace=False):
        elems = np.sort(rng.choice(n_cubes, 3, replace=False))
        off_s = (4 * np.arange(len(elems) + 1)).astype(np.int32)
        pts_s = np.concatenate([pts[off[e]:off[e + 1]] for e in elems]).astype(np.int32)
        cand_s = np.concatenate([cand[s, off[e]:off[e + 1]] for e in elems])[None]
        rold, rnew, rfl, rnv = rp.eval_partial(X[s:s + 1], off_s, pts_s, cand_s)
        g_fl = fl.cpu().numpy()[s, elems][None].astype(np.uint32)
        np.testing.assert_array_equal(g_fl, rfl)
        np.testing.assert_array_equal(vc.cpu().numpy()[s, elems][None][g_fl == 0], rnv[g_fl == 0])
        assert_objectives_close(new.cpu().numpy()[s, elems][None], rnew, flags=g_fl, what="part_new")
        assert_objectives_close(old.cpu().numpy()[s, elems][None], rold, what="part_old")


def test_empty_calls_are_no_ops():
    """S = 0, F = 0 and empty batches enqueue nothing and report success."""
    w = W.tiny()
    gp = _gpu_problem(w, w.S)
    X0 = torch.zeros((0, 2, w.P, 3), dtype=torch.float32, device=DEV)
    obj, fl = gp.eval_full(X0)
    assert obj.shape == (0, 3) and fl.shape == (0,)
    assert gp.fold_check(X0).shape == (0,)
    off0 = torch.zeros(1, dtype=torch.int32, device=DEV)
    pts0 = torch.zeros(0, dtype=torch.int32, device=DEV)
    X = _t(w.population())
    cand0 = torch.zeros((w.S, 0, 2, 3), dtype=torch.float32, device=DEV)
    old, new, flg, _ = gp.eval_partial(X, off0, pts0, cand0)
    assert old.shape == (w.S, 0, 3)
    assert dsm.refine_population(w.mesh, X0).shape[0] == 0
    assert dsm.Batch(max_jobs=2).eval_partial([]) == []
    torch.cuda.synchronize()


def test_maximum_image_size():
    """512^3 images (the largest the exact lattice predicates support): two
    full evaluations and every single-point element of one solution against
    the oracle."""
    shape = (512, 512, 512)
    rng = np.random.default_rng(8)
    coarse = rng.uniform(0, 1, (17, 17, 17)).astype(np.float32)
    from scipy import ndimage
    fixed = ndimage.zoom(coarse, 512 / 17, order=1)[:512, :512, :512].astype(np.float32)
    moving = np.roll(fixed, 3, axis=2)
    w = W.Workload("max-512^3", moving, fixed, (4, 4, 4), (1.0, 1.0, 1.0), 0.2, 4, 6.0, 4.0, 51, 52)
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    _say(f"{w.name}: {w.S} solutions, {w.P} points")
    gp = _gpu_problem(w, w.S)
    obj, fl = gp.eval_full(_t(X))
    old, new, flg, vc = gp.eval_partial(_t(X), _t(off), _t(pts), _t(cand), voxel_count=True)
    torch.cuda.synchronize()
    _say(f"{w.name}: oracle on every element of solution 1")
    robj, rfl, rterms, _ = rp.eval_full(X[:2], want_terms=True)
    np.testing.assert_array_equal(fl.cpu().numpy()[:2], rfl)
    assert_objectives_close(obj.cpu().numpy()[:2], robj, what="full objectives at 512^3")
    rold, rnew, rfl2, rnv = rp.eval_partial(X[1:2], off, pts, cand[1:2], tet_terms=rterms[1:2])
    g_fl = flg.cpu().numpy()[1:2].astype(np.uint32)
    np.testing.assert_array_equal(g_fl, rfl2)
    assert (g_fl == 0).sum() > w.P // 2
    np.testing.assert_array_equal(vc.cpu().numpy()[1:2][g_fl == 0], rnv[g_fl == 0])
    assert_objectives_close(new.cpu().numpy()[1:2], rnew, flags=g_fl, what="part_new at 512^3")
    assert_objectives_close(old.cpu().numpy()[1:2], rold, what="part_old at 512^3")


def _uneven_level(level, idx):
    """Oracle and GPU problems, feasible populations, candidates and cached
    current terms of the uneven problems idx at one pyramid level (level 1
    starts from a level-0 population handed off to full resolution)."""
    out = []
    for i, w in zip(idx, W.uneven(idx, level=level)):
        rp = oracle_problem(w)
        if level == 0:
            X = feasible_population(w, rp)
        else:
            wh = W.uneven([i], level=0)[0]
            X = W.upsample_population(feasible_population(wh, oracle_problem(wh)))
        off, pts = w.fos()
        cand = w.candidates(X, off, pts)
        gp = _gpu_problem(w, len(X))
        Xd = _t(X)
        cache = torch.empty((len(X), gp.T, 3), dtype=torch.float64, device=DEV)
        gp.eval_full(Xd, tet_terms=cache)
        job = dict(problem=gp, X=Xd, fos_off=_t(off), fos_pts=_t(pts), cand=_t(cand), tet_terms_in=cache)
        out.append((w, rp, X, off, pts, cand, job))
    return out


def test_uneven_batch_graph_both_levels():
    """All 12 uneven problems at both pyramid levels as two stored batch
    configurations, enqueued by dsm_batch_run and captured together in one HIP
    graph: every replay (with eager work in between) equals the eager run bit
    for bit, the eager run equals one launch per problem, and every problem is
    checked against the oracle on sampled pairs.  Rows by slice at level 0 and
    by slice pair at level 1, the orders the benchmark keeps."""
    idx = list(range(12))
    levels = []
    for level in (0, 1):
        probs = _uneven_level(level, idx)
        for p in probs:
            p[-1]["problem"].set_row_order(level)
        batch = dsm.Batch(max_jobs=len(probs))
        outs = batch.set_jobs([p[-1] for p in probs])
        levels.append((probs, batch, outs))
        _say(f"uneven level {level}: {[p[0].name for p in probs]}")
    single = [[p[-1]["problem"].eval_partial(p[-1]["X"], p[-1]["fos_off"], p[-1]["fos_pts"], p[-1]["cand"],
                                             tet_terms_in=p[-1]["tet_terms_in"], voxel_count=True) for p in probs]
              for probs, _, _ in levels]
    for _, batch, _ in levels:
        batch.run()
    torch.cuda.synchronize()
    eager = [[[t.cpu().numpy().copy() for t in o] for o in outs] for _, _, outs in levels]
    for lv in range(2):
        for e, sg in zip(eager[lv], single[lv]):
            for a, b in zip(e, sg):
                np.testing.assert_array_equal(a, b.cpu().numpy())
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    _say("capturing both levels")
    with torch.cuda.graph(graph, stream=stream):
        for _, batch, _ in levels:
            batch.run()
    torch.cuda.synchronize()
    w0, _, X0, off0, pts0, cand0, job0 = levels[1][0][0]
    for rep in range(3):
        for _, _, outs in levels:
            for o in outs:
                o[0].fill_(float("nan"))
                o[1].fill_(float("nan"))
                o[2].fill_(-1)
                o[3].fill_(-1)
        graph.replay()
        # eager work of the program between replays
        job0["problem"].eval_partial(job0["X"], job0["fos_off"], job0["fos_pts"], job0["cand"],
                                     tet_terms_in=job0["tet_terms_in"])
        torch.cuda.synchronize()
        for lv, (_, _, outs) in enumerate(levels):
            for e, o in zip(eager[lv], outs):
                for a, b in zip(e, o):
                    np.testing.assert_array_equal(a, b.cpu().numpy(), err_msg=f"replay {rep} level {lv}")
        _say(f"replay {rep} equal to eager")
    rng = np.random.default_rng(17)
    for lv, (probs, _, _) in enumerate(levels):
        for k, (w, rp, X, off, pts, cand, _) in enumerate(probs):
            s = int(rng.integers(len(X)))
            elems = np.sort(rng.choice(w.P, 4, replace=False)).astype(np.int32)
            rold, rnew, rfl, rnv = rp.eval_partial(X[s:s + 1], np.arange(5, dtype=np.int32), elems,
                                                    cand[s:s + 1, elems])
            o = eager[lv][k]
            g_fl = o[2][s, elems][None].astype(np.uint32)
            np.testing.assert_array_equal(g_fl, rfl)
            np.testing.assert_array_equal(o[3][s, elems][None][g_fl == 0], rnv[g_fl == 0])
            assert_objectives_close(o[1][s, elems][None], rnew, flags=g_fl, what=f"level {lv} {w.name} part_new")
            assert_objectives_close(o[0][s, elems][None], rold, what=f"level {lv} {w.name} part_old")


def test_stored_batch_keeps_its_chunk():
    """A stored multi-problem configuration keeps the work split and row order
    it was stored with: changing a problem's chunk and row order afterwards
    changes neither what dsm_batch_run computes nor its bits, while a new
    dsm_eval_partial follows the new settings."""
    probs = _uneven_level(0, [0, 4])
    for *_, job in probs:
        job["problem"].set_part_chunk(5)
        job["problem"].set_row_order(1)
    batch = dsm.Batch(max_jobs=2)
    outs = batch.set_jobs([p[-1] for p in probs])
    batch.run()
    torch.cuda.synchronize()
    stored5 = [[t.cpu().numpy().copy() for t in o] for o in outs]
    single5 = [p[-1]["problem"].eval_partial(p[-1]["X"], p[-1]["fos_off"], p[-1]["fos_pts"], p[-1]["cand"],
                                             tet_terms_in=p[-1]["tet_terms_in"], voxel_count=True) for p in probs]
    for *_, job in probs:
        job["problem"].set_part_chunk(8)
        job["problem"].set_row_order(0)
    batch.run()
    single8 = [p[-1]["problem"].eval_partial(p[-1]["X"], p[-1]["fos_off"], p[-1]["fos_pts"], p[-1]["cand"],
                                             tet_terms_in=p[-1]["tet_terms_in"], voxel_count=True) for p in probs]
    torch.cuda.synchronize()
    for o, s5, s8, st5 in zip(outs, single5, single8, stored5):
        for a, b, c, d in zip(o, s5, s8, st5):
            a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
            np.testing.assert_array_equal(a, d)      # the stored run repeats itself bit for bit
            np.testing.assert_array_equal(a, b)      # and equals a launch at the stored chunk
            if a.dtype.kind == "f":
                np.testing.assert_allclose(c, a, rtol=_SPLIT_RTOL, atol=1e-12)
            else:
                np.testing.assert_array_equal(c, a)  # flags and counts do not depend on the chunk
