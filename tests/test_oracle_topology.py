"""Pins of the oracle's mesh topology (Sec. 2.1, Fig. 1 A/B; Sec. 2.2 stars;
Sec. 2.3.2 edges) against closed-form counts and symmetries."""
import itertools
import os
from collections import Counter

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W

MESHES = [(2, 2, 2), (3, 3, 3), (5, 5, 5), (4, 3, 5), (10, 10, 6), (6, 6, 6)]


def _problem(mesh, dims=(16, 16, 16)):
    z = np.zeros(dims[::-1], np.float32)
    return ref.Problem(z, z, mesh)


def _lattice(X):
    return np.rint((X.astype(np.float64) + 0.5) * 128.0)


@pytest.mark.parametrize("mesh", MESHES)
def test_counts_closed_form(mesh):
    nx, ny, nz = mesh
    p = _problem(mesh, dims=(40, 40, 40))
    C = (nx - 1) * (ny - 1) * (nz - 1)
    assert p.P == nx * ny * nz
    assert p.T == 6 * C  # 6 tetrahedra per cube (Sec. 2.1)
    axis = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    face_diag = (nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1)
    # a conforming split has exactly one diagonal per square face and one body diagonal per cube
    assert p.E == axis + face_diag + C
    e, k = p.edges()
    assert k.sum() == 6 * p.T


@pytest.mark.parametrize("mesh", MESHES)
def test_faces_conform_and_euler(mesh):
    p = _problem(mesh, dims=(40, 40, 40))
    tets = p.tets()
    faces = Counter()
    for t in tets:
        for f in itertools.combinations(sorted(t), 3):
            faces[f] += 1
    assert max(faces.values()) <= 2
    nx, ny, nz = mesh
    boundary_squares = 2 * ((nx - 1) * (ny - 1) + (nx - 1) * (nz - 1) + (ny - 1) * (nz - 1))
    assert sum(1 for c in faces.values() if c == 1) == 2 * boundary_squares
    # Euler characteristic of a triangulated ball
    assert p.P - p.E + len(faces) - p.T == 1


@pytest.mark.parametrize("mesh,dims", [((3, 3, 3), (32, 32, 32)), ((5, 4, 3), (33, 17, 9)), ((10, 10, 6), (512, 512, 100))])
def test_positive_and_volume_fills_box(mesh, dims):
    p = _problem(mesh, dims)
    L = _lattice(p.identity())
    tets = p.tets()
    vol = 0
    for t in tets:
        o = ref.orient3d(*L[t])
        assert o > 0
        vol += int(o)
    # the tetrahedra tile the image box exactly: sum of 6*volume = 6 * prod(128 D)
    assert vol == 6 * np.prod([128 * d for d in dims], dtype=object)


def test_identity_matches_input_generator():
    for mesh, dims in [((3, 3, 3), (32, 32, 32)), ((10, 10, 6), (512, 512, 100)), ((4, 5, 6), (33, 17, 9))]:
        p = _problem(mesh, dims)
        np.testing.assert_array_equal(p.identity(), W.regular_grid(dims, mesh))


def test_mirror_and_axis_symmetry():
    """Sec. 2.1: groups of 2x2x2 cubes are mirrored, which makes the split
    symmetric: the tetrahedron set of an even cube count is invariant under
    reflection of any axis and, for a cubic mesh, under axis permutations."""
    n = 5
    p = _problem((n, n, n))
    tets = {frozenset(t) for t in p.tets().tolist()}

    def pid(i, j, k):
        return i + n * (j + n * k)

    coords = [(v % n, (v // n) % n, v // (n * n)) for v in range(n ** 3)]
    maps = []
    for a in range(3):
        maps.append(lambda c, a=a: tuple((n - 1 - c[b]) if b == a else c[b] for b in range(3)))
    for perm in itertools.permutations(range(3)):
        maps.append(lambda c, perm=perm: tuple(c[perm[b]] for b in range(3)))
    for m in maps:
        image = {frozenset(pid(*m(coords[v])) for v in t) for t in tets}
        assert image == tets


def test_star_histogram_clinical_mesh():
    """Stars (tetrahedra re-evaluated when a point moves, Sec. 2.2) of a
    10x10x6 mesh: sizes 2..48 with this histogram under the mirrored split."""
    p = _problem((10, 10, 6), (512, 512, 100))
    off, _ = p.star()
    hist = Counter(np.diff(off).tolist())
    assert hist == {2: 6, 4: 60, 6: 2, 8: 192, 12: 20, 16: 192, 24: 64, 48: 64}
    assert p.max_star == 48


def test_parameter_counts_golden():
    """Sec. 2.5: 6^3 and 11^3 grids give 1296 and 7986 parameters."""
    path = os.path.join(os.path.dirname(__file__), "golden", "param_counts.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows
    for nx, ny, nz, params in rows:
        p = _problem((int(nx), int(ny), int(nz)), (64, 64, 64))
        X = p.identity()
        assert 2 * X.size == int(params)  # 3 coordinates per point, 2 grids
