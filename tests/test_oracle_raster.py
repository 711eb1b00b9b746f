"""Pins of the oracle's exact predicates and rasterisation (Sec. 2.3.1: slices
rasterised with the top-left rule, extended to 3-D by a symbolic perturbation
of the voxel centre by (+e, +e^2, +e^3))."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W

PERMS = list(itertools.permutations(range(3)))  # lexicographic: xyz xzy yxz yzx zxy zyx


def _exact_orient(a, b, c, d):
    a, b, c, d = ([int(v) for v in x] for x in (a, b, c, d))
    m = [[b[i] - a[i] for i in range(3)], [c[i] - a[i] for i in range(3)], [d[i] - a[i] for i in range(3)]]
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def test_orient3d_fp64_exact_on_lattice():
    """FP64 orientation of lattice points (|u| <= 2^16) equals big-integer arithmetic,
    including exactly coplanar and nearly coplanar configurations."""
    rng = np.random.default_rng(0)
    for trial in range(4000):
        pts = rng.integers(0, 2 ** 16 + 1, size=(4, 3))
        if trial % 3 == 1:  # coplanar: d = a + i (b - a) + j (c - a) with small integers
            i, j = rng.integers(-2, 3, size=2)
            pts[3] = pts[0] + i * (pts[1] - pts[0]) + j * (pts[2] - pts[0])
            if np.any(pts[3] < 0) or np.any(pts[3] > 2 ** 16):
                continue
        if trial % 3 == 2:  # nearly coplanar
            pts[3] = np.clip((pts[0] + pts[1] + pts[2]) // 3 + rng.integers(-1, 2, size=3), 0, 2 ** 16)
        got = ref.orient3d(*pts.astype(np.float64))
        assert got == _exact_orient(*pts)


def _expected_owner(dims, mesh, vox):
    """Closed-form owner of a voxel centre in the undeformed mesh, without any
    orientation test: its cube by comparing with the grid planes, its Kuhn
    tetrahedron by sorting the (mirrored) local coordinates; exact ties are
    broken by the perturbation (+e, +e^2, +e^3) of the centre."""
    nx, ny, nz = mesh
    cube, tloc, sgn = [], [], []
    for a in range(3):
        D, n = dims[a], mesh[a]
        u = [(2 * i * 128 * D + (n - 1)) // (2 * (n - 1)) for i in range(n)]
        x = 128 * vox[a] + 64
        c = max(i for i in range(n - 1) if u[i] <= x)  # x == u[i] -> perturbed into cube i
        t = Fraction(x - u[c], u[c + 1] - u[c])
        mirrored = c & 1
        cube.append(c)
        tloc.append(1 - t if mirrored else t)
        sgn.append(-1 if mirrored else 1)
    # order of perturbed local coordinates: t_a + sgn_a * e^(a+1)
    def key(a):
        return tloc[a]

    def greater(a, b):  # is perturbed local coord a > b ?
        if tloc[a] != tloc[b]:
            return tloc[a] > tloc[b]
        first = min(a, b)
        return (sgn[first] > 0) == (first == a)

    order = [0, 1, 2]
    for i in range(3):
        for j in range(2 - i):
            if greater(order[j + 1], order[j]):
                order[j], order[j + 1] = order[j + 1], order[j]
    sigma = PERMS.index(tuple(order))
    cid = cube[0] + (nx - 1) * (cube[1] + (ny - 1) * cube[2])
    return 6 * cid + sigma


@pytest.mark.parametrize("dims,mesh", [((33, 33, 33), (3, 3, 3)), ((17, 9, 25), (3, 2, 4)), ((32, 32, 32), (3, 3, 3)),
                                       ((25, 13, 9), (4, 4, 3))])
def test_owner_closed_form_identity(dims, mesh):
    """Undeformed mesh: every voxel centre is owned exactly once, by the
    tetrahedron the closed form predicts.  Odd dims put grid planes, face
    diagonals and vertices on voxel centres, so most tie-break cases occur."""
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh)
    owner, count = p.owner_bruteforce(p.identity())
    assert np.all(count == 1)
    rng = np.random.default_rng(1)
    Dx, Dy, Dz = dims
    sample = [(i, j, k) for k in range(Dz) for j in range(Dy) for i in range(Dx)]
    if len(sample) > 6000:
        idx = rng.choice(len(sample), 6000, replace=False)
        sample = [sample[i] for i in idx]
    for (i, j, k) in sample:
        assert owner[k, j, i] == _expected_owner(dims, mesh, (i, j, k)), (i, j, k)


def _feasible_population(p, dims, mesh, S, sigma, seed):
    def reject(X):
        return p.fold_check(X)[0] != 0
    return W.population(dims, mesh, S, sigma, seed, reject=reject)


@pytest.mark.parametrize("dims,mesh,sigma", [((33, 33, 33), (3, 3, 3), 3.0), ((20, 17, 12), (5, 4, 3), 1.5),
                                             ((16, 16, 16), (5, 5, 5), 0.8)])
def test_exactly_once_coverage_random_meshes(dims, mesh, sigma):
    """Every voxel centre lies in exactly one tetrahedron of a feasible mesh
    (both grids, random perturbations on the lattice)."""
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh)
    X = _feasible_population(p, dims, mesh, 3, sigma, seed=7)
    assert np.all(p.fold_check(X)[0] == 0)
    for s in range(3):
        for g in range(2):
            _, count = p.owner_bruteforce(X[s, g])
            assert np.all(count == 1)


def test_bbox_scan_equals_bruteforce():
    """The per-tetrahedron voxel lists equal the brute-force owner map."""
    dims, mesh = (21, 19, 17), (4, 3, 3)
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh)
    X = _feasible_population(p, dims, mesh, 2, 1.5, seed=3)
    for s in range(2):
        owner, count = p.owner_bruteforce(X[s, 0])
        flat = owner.ravel()
        total = 0
        for t in range(p.T):
            vox = p.tet_voxels(X[s, 0], t)
            total += len(vox)
            np.testing.assert_array_equal(np.sort(vox), np.nonzero(flat == t)[0])
        assert total == p.V


def test_star_region_invariance():
    """Moving one point feasibly does not change the voxel set of its star
    (the union of its tetrahedra's voxels) -- partial evaluations only touch it."""
    dims, mesh = (24, 20, 16), (4, 4, 3)
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh)
    off, st = p.star()
    rng = np.random.default_rng(5)
    X = _feasible_population(p, dims, mesh, 1, 1.0, seed=9)[0]
    free = W.free_mask(mesh)
    moved = 0
    for trial in range(60):
        v = int(rng.integers(p.P))
        Y = X.copy()
        Y[0, v] = W.snap(Y[0, v] + free[v] * rng.normal(0, 2.0, 3))
        if p.fold_check(Y[None])[0][0] != 0:
            continue
        moved += 1
        star = st[off[v]:off[v + 1]]
        before = np.sort(np.concatenate([p.tet_voxels(X[0], t) for t in star]))
        after = np.sort(np.concatenate([p.tet_voxels(Y[0], t) for t in star]))
        np.testing.assert_array_equal(before, after)
    assert moved > 20


def test_top_left_rule_in_a_slice():
    """Footnote of Sec. 2.3.1 in one axial slice: a voxel centre on an edge
    shared by two triangles goes to the triangle on its +x side (left edge);
    on a horizontal edge to the one on its +y side (rows grow downward)."""
    dims, mesh = (33, 33, 33), (3, 3, 3)
    z = np.zeros(dims[::-1], np.float32)
    p = ref.Problem(z, z, mesh)
    owner, _ = p.owner_bruteforce(p.identity())
    tets = p.tets()
    L = np.rint((p.identity().astype(np.float64) + 0.5) * 128)
    # voxel on the grid plane x = 16 (interior of a cube face): owner lies at x >= 16
    t = owner[5, 5, 16]
    assert L[tets[t], 0].max() > 128 * 16 + 64 - 1 and L[tets[t], 0].min() >= 128 * 16 + 64 - 1
    # voxel on the plane y = 16 away from x/z planes: owner lies at y >= 16
    t = owner[5, 16, 5]
    assert L[tets[t], 1].min() >= 128 * 16 + 64 - 1
