"""Pins of the oracle's objectives (Sec. 2.3.1-2.3.3), partial evaluation
(Sec. 2.2-2.3) and constraint flags (Sec. 2.3.4) against closed forms,
symmetries and an independent numpy/scipy evaluation."""
import itertools

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

from oracle import ref
from paper_2202_11001_amd import workloads as W

PERMS = list(itertools.permutations(range(3)))


def _contrib(a, b, eb, tau):
    ea = (a <= tau).astype(np.float64)
    m = np.abs(ea - eb)
    return (1 - m) * (a - b) ** 2 + m


def _small_problem(seed=0, dims=(20, 18, 14), mesh=(4, 3, 3), spacing=(1.0, 1.2, 2.0), tau=0.15, guid=True):
    rng = np.random.default_rng(seed)
    shp = dims[::-1]
    fixed = W._blur(rng.uniform(0, 1, shp) * (rng.uniform(0, 1, shp) > 0.3), 1.0).astype(np.float32)
    moving = W._blur(rng.uniform(0, 1, shp) * (rng.uniform(0, 1, shp) > 0.3), 1.0).astype(np.float32)
    kw = {}
    if guid:
        hi = np.array(dims) - 1.0
        kw = dict(guid_moving=W.snap(rng.uniform(0, 1, (5, 3)) * hi), corr_moving=np.array([0, 1, 2, 2, 3]),
                  guid_fixed=W.snap(rng.uniform(0, 1, (6, 3)) * hi), corr_fixed=np.array([0, 1, 1, 2, 3, 3]))
    p = ref.Problem(moving, fixed, mesh, spacing, tau, **kw)
    return p, moving, fixed, kw


def _feasible(p, S, sigma, seed):
    dims = tuple(int(d) for d in p.dims)
    return W.population(dims, tuple(p.mesh), S, sigma, seed, reject=lambda X: p.fold_check(X)[0] != 0)


def test_identity_identical_images_zero():
    img = W._blur(np.random.default_rng(1).uniform(0, 1, (12, 14, 16)), 1.0).astype(np.float32)
    p = ref.Problem(img, img, (3, 4, 3), (1, 1, 1), 0.2)
    X = np.stack([p.identity(), p.identity()])[None]
    obj, flags = p.eval_full(X)
    assert flags[0] == 0
    assert obj[0, 0] == pytest.approx(0.0, abs=1e-20)
    assert obj[0, 1] == 0.0 and obj[0, 2] == 0.0


@pytest.mark.parametrize("hard", [False, True])
def test_same_mesh_both_grids_closed_form(hard):
    """When both grids hold the same mesh the map is the identity on every
    tetrahedron: each voxel is compared with the same voxel of the other image,
    forward and backward, whatever the mesh (exactly-once coverage)."""
    p0, moving, fixed, _ = _small_problem(2, guid=False)
    p = ref.Problem(moving, fixed, p0.mesh, p0.spacing, 0.15, hard_threshold=hard)
    X = _feasible(p, 3, 1.2, 4)
    X[:, 1] = X[:, 0]
    X[0] = np.stack([p.identity(), p.identity()])
    obj, flags = p.eval_full(X)
    assert np.all(flags == 0)
    a = fixed.astype(np.float64)
    b = moving.astype(np.float64)
    tau = 0.15
    if hard:
        m = ((a <= tau) != (b <= tau)).astype(np.float64)
        fw = np.where(m > 0, 1.0, (a - b) ** 2)
        bw = fw
    else:
        fw = _contrib(a, b, (b <= tau).astype(np.float64), tau)
        bw = _contrib(b, a, (a <= tau).astype(np.float64), tau)
    expect = (fw.sum() + bw.sum()) / (2 * a.size)
    np.testing.assert_allclose(obj[:, 0], expect, rtol=1e-11)
    assert np.all(obj[:, 1] == 0)


def _independent_sim(p, moving, fixed, X, tau):
    """Dissimilarity computed without the oracle's arithmetic: owner tetrahedron
    per voxel from the brute-force owner map, barycentric coordinates by
    np.linalg.solve, trilinear sampling with clamp-to-edge by scipy."""
    tets = p.tets()
    imgs = [moving.astype(np.float64), fixed.astype(np.float64)]
    total = 0.0
    for own in (1, 0):
        other = 1 - own
        owner, count = p.owner_bruteforce(X[own])
        assert np.all(count == 1)
        Dz, Dy, Dx = imgs[own].shape
        k, j, i = np.meshgrid(np.arange(Dz), np.arange(Dy), np.arange(Dx), indexing="ij")
        pts = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.float64)
        own_v = X[own].astype(np.float64)[tets[owner.ravel()]]  # [V][4][3]
        oth_v = X[other].astype(np.float64)[tets[owner.ravel()]]
        A = np.concatenate([own_v.transpose(0, 2, 1), np.ones((len(pts), 1, 4))], axis=1)  # [V][4][4]
        rhs = np.concatenate([pts, np.ones((len(pts), 1))], axis=1)
        lam = np.linalg.solve(A, rhs[..., None])[..., 0]  # [V][4]
        q = np.einsum("vi,via->va", lam, oth_v)
        coords = [q[:, 2], q[:, 1], q[:, 0]]
        b = map_coordinates(imgs[other], coords, order=1, mode="nearest")
        eb = map_coordinates((imgs[other] <= tau).astype(np.float64), coords, order=1, mode="nearest")
        total += _contrib(imgs[own].ravel(), b, eb, tau).sum()
    return total / (2 * imgs[0].size)


@pytest.mark.parametrize("seed", [0, 1])
def test_dissimilarity_vs_scipy(seed):
    p, moving, fixed, _ = _small_problem(seed, guid=False)
    X = _feasible(p, 2, 1.5, 10 + seed)
    obj, flags = p.eval_full(X)
    assert np.all(flags == 0)
    for s in range(2):
        np.testing.assert_allclose(obj[s, 0], _independent_sim(p, moving, fixed, X[s], 0.15), rtol=1e-9)


def test_ramp_images_samples_exactly():
    """Trilinear interpolation reproduces a linear ramp exactly, so on ramp
    images the dissimilarity of any feasible mesh matches the scipy path
    without interpolation error (clamping aside: the ramp is sampled inside)."""
    dims, mesh = (18, 16, 12), (3, 3, 3)
    mov = W.ramp(dims[::-1], (0.02, 0.01, 0.03), 0.2)
    fix = W.ramp(dims[::-1], (0.015, 0.02, 0.01), 0.1)
    p = ref.Problem(mov, fix, mesh, (1, 1, 1), 0.05)
    X = _feasible(p, 1, 1.0, 3)
    obj, _ = p.eval_full(X)
    np.testing.assert_allclose(obj[0, 0], _independent_sim(p, mov, fix, X[0], 0.05), rtol=1e-10)


def test_deformation_uniform_scaling_closed_form():
    """Sec. 2.3.2: if the target grid is the source grid scaled by 1/2, every
    edge and spoke changes by half its length, so the energy is
    (1/4) * (sum of squared edge lengths + squared spoke lengths) / (E + 4T)."""
    dims, mesh, sp = (32, 32, 32), (3, 3, 3), (1.0, 0.8, 2.5)
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh, sp, 0.1)
    X0 = p.identity()
    U = np.rint((X0.astype(np.float64) + 0.5) * 128)
    X1 = (U / 2 / 128 - 0.5).astype(np.float32)
    obj, _ = p.eval_full(np.stack([X0, X1])[None])
    h = np.array([16.0, 16.0, 16.0]) * sp  # cube extent in mm
    nx, ny, nz = mesh
    C = (nx - 1) * (ny - 1) * (nz - 1)
    hx2, hy2, hz2 = h ** 2
    edges = ((nx - 1) * ny * nz * hx2 + nx * (ny - 1) * nz * hy2 + nx * ny * (nz - 1) * hz2
             + (nx - 1) * (ny - 1) * nz * (hx2 + hy2) + (nx - 1) * ny * (nz - 1) * (hx2 + hz2)
             + nx * (ny - 1) * (nz - 1) * (hy2 + hz2) + C * (hx2 + hy2 + hz2))
    spokes = 0.0
    for perm in PERMS:  # Kuhn path of each tetrahedron; mirroring does not change lengths
        v = [np.zeros(3)]
        for a in perm:
            w = v[-1].copy()
            w[a] = 1
            v.append(w)
        v = [x * h for x in v]
        for i in range(4):
            c = sum(v[j] for j in range(4) if j != i) / 3
            spokes += np.sum((v[i] - c) ** 2)
    spokes *= C
    E, T = p.E, p.T
    assert obj[0, 1] == pytest.approx(0.25 * (edges + spokes) / (E + 4 * T), rel=1e-12)


def test_guidance_identity_closed_form():
    """Sec. 2.3.3 on the undeformed mesh: each point is compared with the
    nearest point of its correspondence in the other image, both ways."""
    p, moving, fixed, kw = _small_problem(3)
    X = np.stack([p.identity(), p.identity()])[None]
    obj, _ = p.eval_full(X)
    gm, gf = kw["guid_moving"].astype(np.float64), kw["guid_fixed"].astype(np.float64)
    cm, cf = kw["corr_moving"], kw["corr_fixed"]
    sp = p.spacing
    tot = 0.0
    for A, ca, B, cb in ((gm, cm, gf, cf), (gf, cf, gm, cm)):
        for q, c in zip(A, ca):
            d = [np.sum(((q - r) * sp) ** 2) for r, cr in zip(B, cb) if cr == c]
            tot += min(d)
    assert obj[0, 2] == pytest.approx(tot / (len(gm) + len(gf)), rel=1e-12)


def test_swap_symmetry():
    """Exchanging source and target (images, grids, guidance) leaves all
    three objectives unchanged (forward and backward are both summed)."""
    p, moving, fixed, kw = _small_problem(4)
    X = _feasible(p, 2, 1.2, 6)
    q = ref.Problem(fixed, moving, p.mesh, p.spacing, 0.15, guid_moving=kw["guid_fixed"], corr_moving=kw["corr_fixed"],
                    guid_fixed=kw["guid_moving"], corr_fixed=kw["corr_moving"])
    a, _ = p.eval_full(X)
    b, _ = q.eval_full(X[:, ::-1].copy())
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_partial_consistency():
    """Sec. 2.3: objectives decompose into per-cell values.  One FOS element
    holding every point equals full evaluation; for single points,
    full(new) = full(old) - part_old + part_new; cached terms reproduce part_old."""
    p, moving, fixed, kw = _small_problem(5)
    dims = tuple(int(d) for d in p.dims)
    X = _feasible(p, 2, 1.0, 8)
    obj, flags, terms, nvox = p.eval_full(X, want_terms=True)
    assert np.all(nvox == 2 * p.V)
    # everything in one element, candidate = current
    off = np.array([0, p.P], np.int32)
    pts = np.arange(p.P, dtype=np.int32)
    cand = X.transpose(0, 2, 1, 3).copy()
    old, new, fl, nv = p.eval_partial(X, off, pts, cand)
    np.testing.assert_allclose(new[:, 0], obj, rtol=1e-12)
    np.testing.assert_allclose(old[:, 0], obj, rtol=1e-12)
    # single points
    off, pts = W.single_point_fos(p.P)
    cand = W.candidates(X, off, pts, p.mesh, dims, 1.0, 12)
    old, new, fl, nv = p.eval_partial(X, off, pts, cand)
    old2, new2, _, _ = p.eval_partial(X, off, pts, cand, tet_terms=terms)
    np.testing.assert_allclose(old2, old, rtol=1e-12, atol=1e-300)
    np.testing.assert_array_equal(new2, new)
    star_off, star = p.star()
    checked = 0
    for s in range(2):
        for f in range(p.P):
            if fl[s, f]:
                continue
            Y = X[s:s + 1].copy()
            Y[0, :, f] = cand[s, f]
            o2, fl2 = p.eval_full(Y)
            assert fl2[0] == 0
            np.testing.assert_allclose(o2[0], obj[s] - old[s, f] + new[s, f], rtol=1e-11, atol=1e-14)
            # voxels sampled = voxels of the star region in both grids (invariant region)
            nstar = sum(len(p.tet_voxels(X[s, g], t)) for g in range(2) for t in star[star_off[f]:star_off[f + 1]])
            assert nv[s, f] == nstar
            checked += 1
    assert checked > 30


def test_flags():
    """Sec. 2.3.4: folds and border constraints are reported per solution."""
    p, moving, fixed, _ = _small_problem(6, dims=(24, 24, 24), mesh=(4, 4, 4), guid=False)
    I = p.identity()
    base = np.stack([I, I])
    cases = []
    Y = base.copy(); cases.append((Y, 0))
    # interior point (1,1,1) pushed past its +x neighbour in the source grid only -> inverted source tetrahedra
    v = 1 + 4 * (1 + 4 * 1)
    Y = base.copy(); Y[0, v, 0] = Y[0, v + 1, 0] + 1.0; cases.append((Y, ref.FLAG_INV_MOVING))
    Y = base.copy(); Y[1, v, 0] = Y[1, v + 1, 0] + 1.0; cases.append((Y, ref.FLAG_INV_FIXED))
    # border point leaves its border plane (x index 0 must stay at -0.5)
    b = 0 + 4 * (1 + 4 * 1)
    Y = base.copy(); Y[0, b, 0] = 0.5; cases.append((Y, ref.FLAG_BORDER))
    # upper border (x index 3 must stay at D - 0.5)
    bu = 3 + 4 * (2 + 4 * 1)
    Y = base.copy(); Y[1, bu, 0] -= 1.0; cases.append((Y, ref.FLAG_BORDER))
    # border point sliding within its border plane is fine
    Y = base.copy(); Y[0, b, 1] += 1.0; cases.append((Y, 0))
    # outside the box
    Y = base.copy(); Y[1, v, 2] = -3.0; cases.append((Y, ref.FLAG_DOMAIN))
    # off the 1/128 lattice
    Y = base.copy(); Y[1, v, 1] += 1.0 / 256; cases.append((Y, ref.FLAG_LATTICE))
    Y = base.copy(); Y[0, v, 1] = np.nan; cases.append((Y, ref.FLAG_NONFINITE))
    X = np.stack([c[0] for c in cases])
    flags, first_bad = p.fold_check(X)
    for (Y, want), got in zip(cases, flags):
        assert got == want
    assert first_bad[0] == -1 and first_bad[1] >= 0
    tets = p.tets()
    assert v in tets[first_bad[1]]


def test_degenerate_zero_volume_is_a_fold():
    """A tetrahedron flattened to zero volume is infeasible (its grid point lies
    on a face of the surrounding polyhedron)."""
    z = np.zeros((16, 16, 16), np.float32)
    p = ref.Problem(z, z, (3, 3, 3))
    I = p.identity()
    X = np.stack([I, I])[None].copy()
    c = 1 + 3 * (1 + 3 * 1)  # centre point
    X[0, 0, c] = X[0, 0, c - 1]
    X[0, 0, c, 0] = X[0, 0, c - 1, 0]  # move onto the -x border point's position
    flags, _ = p.fold_check(X)
    assert flags[0] & ref.FLAG_INV_MOVING
