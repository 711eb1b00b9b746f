"""Oracle pins for the grid refinement of Sec. 2.4 (multi-resolution): every
cube becomes 8 cubes with points at edge middles, face middles and the cube
centre; fine meshes have 2n-1 points per axis."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ref
from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

LAT = 128.0


def _lattice(X):
    return (X.astype(np.float64) + 0.5) * LAT


def _zoom_means(Xc, mesh):
    """Independent construction: linear interpolation (scipy) of each coordinate
    field at the half-integer grid positions = the mean of the corners."""
    nx, ny, nz = mesh
    S = Xc.shape[0]
    U = _lattice(Xc).reshape(S, 2, nz, ny, nx, 3)
    out = np.zeros((S, 2, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1, 3))
    for s in range(S):
        for g in range(2):
            for c in range(3):
                out[s, g, ..., c] = ndimage.zoom(U[s, g, ..., c], ((2 * nz - 1) / nz, (2 * ny - 1) / ny,
                                                                     (2 * nx - 1) / nx), order=1)
    return out.reshape(S, 2, -1, 3)


@pytest.mark.parametrize("mesh,dims", [((3, 3, 3), (32, 32, 32)), ((4, 3, 5), (37, 23, 41)), ((2, 2, 2), (9, 9, 9))])
def test_refine_is_the_rounded_corner_mean(mesh, dims):
    rng = np.random.default_rng(1)
    Xc = W.population(dims, mesh, 4, 2.0, 7)
    Xf = ref.refine(mesh, Xc)
    nf = tuple(2 * n - 1 for n in mesh)
    assert Xf.shape == (4, 2, int(np.prod(nf)), 3)
    means = _zoom_means(Xc, mesh)
    np.testing.assert_array_equal(_lattice(Xf), np.rint(means))  # numpy rint: half to even
    # fine points with all indices even are the coarse points, unchanged
    I = np.arange(int(np.prod(nf)))
    i, j, k = I % nf[0], (I // nf[0]) % nf[1], I // (nf[0] * nf[1])
    even = (i % 2 == 0) & (j % 2 == 0) & (k % 2 == 0)
    ci = (i // 2) + mesh[0] * ((j // 2) + mesh[1] * (k // 2))
    np.testing.assert_array_equal(Xf[:, :, even], Xc[:, :, ci[even]])
    assert rng is not None


def test_refined_identity_is_the_finer_identity_within_one_lattice_step():
    for mesh, dims in [((3, 3, 3), (32, 32, 32)), ((6, 6, 6), (64, 64, 64)), ((10, 10, 6), (512, 512, 100)),
                       ((4, 5, 3), (37, 23, 19))]:
        z = np.zeros(dims[::-1], np.float32)
        rc = ref.Problem(z, z, mesh)
        nf = tuple(2 * n - 1 for n in mesh)
        rf = ref.Problem(z, z, nf)
        Ic, If = rc.identity(), rf.identity()
        Xf = ref.refine(mesh, np.stack([Ic, Ic])[None])
        d = np.abs(_lattice(Xf[0, 0]) - _lattice(If))
        assert d.max() <= 1.0
        assert rf.fold_check(Xf)[0][0] == 0


def test_translation_by_even_lattice_steps_commutes():
    mesh, dims = (4, 3, 3), (40, 30, 30)
    Xc = W.population(dims, mesh, 3, 1.5, 11)
    t = np.array([6.0, -4.0, 2.0]) / LAT  # even numbers of lattice steps keep the rounding ties' parity
    a = ref.refine(mesh, Xc)
    b = ref.refine(mesh, (Xc.astype(np.float64) + t).astype(np.float32))
    np.testing.assert_array_equal(_lattice(b) - _lattice(a), np.broadcast_to(t * LAT, a.shape))


def test_refinement_keeps_border_pins_and_feasibility():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    nf = tuple(2 * n - 1 for n in w.mesh)
    Xf = ref.refine(w.mesh, X)
    rf = ref.Problem(w.moving, w.fixed, nf, w.spacing, w.tau)
    flags, _ = rf.fold_check(Xf)
    assert np.all((flags & 4) == 0)  # border pins
    # Sec. 2.4: refinement preserves feasibility (mild deformations)
    assert int((flags != 0).sum()) == 0
