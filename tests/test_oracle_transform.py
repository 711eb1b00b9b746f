"""Pins of the oracle's piecewise-affine transformation (ref_transform: the DVF
and the transformed image of Sec. 2.1 / Fig. 2) against closed forms, a
symmetry and an independent barycentric solve."""
import numpy as np

from oracle import ref
from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

SHAPE = (32, 32, 32)
MESH = (3, 3, 3)


def _problem(moving=None, fixed=None):
    w = W.tiny()
    return ref.Problem(w.moving if moving is None else moving, w.fixed if fixed is None else fixed, MESH, tau=0.1)


def _plane_moved(rp, delta):
    """identity grid with the interior x-plane (i = 1) moved by delta voxels"""
    I = rp.identity()
    J = I.copy()
    i = np.arange(rp.P) % MESH[0]
    J[i == 1, 0] += delta
    return I, J


def test_identity_maps_every_voxel_to_itself():
    rp = _problem()
    I = rp.identity()
    for own in (0, 1):
        dvf, warped = rp.transform(own, np.stack([I, I]))
        assert np.all(np.isfinite(dvf)) and np.abs(dvf).max() < 1e-12
        other = W.tiny().moving if own == 1 else W.tiny().fixed
        np.testing.assert_allclose(warped, other, rtol=0, atol=1e-12)


def test_moved_plane_closed_form_both_directions():
    ramp = W.ramp(SHAPE)
    rp = _problem(moving=ramp, fixed=ramp)
    I, J = _plane_moved(rp, 4.0)
    xs = I[np.arange(rp.P) % 3 == 1, 0][0]
    assert xs == 15.5
    x = np.arange(32, dtype=np.float64)
    # own = 1: target voxels (identity grid) into the source grid (plane at 19.5)
    want_t = np.where(x < 15.5, -0.5 + (x + 0.5) * 20.0 / 16.0, 19.5 + (x - 15.5) * 12.0 / 16.0)
    # own = 0: source voxels (moved grid) back into the target grid
    want_s = np.where(x < 19.5, -0.5 + (x + 0.5) * 16.0 / 20.0, 15.5 + (x - 19.5) * 16.0 / 12.0)
    for own, want in ((1, want_t), (0, want_s)):
        dvf, warped = rp.transform(own, np.stack([J, I]))
        np.testing.assert_allclose(dvf[..., 0], np.broadcast_to(want - x, SHAPE), rtol=0, atol=1e-10)
        assert np.abs(dvf[..., 1:]).max() < 1e-10
        # the ramp is linear, so trilinear sampling at the mapped point is exact (clamped at the box)
        z, y = np.meshgrid(np.arange(32.0), np.arange(32.0), indexing="ij")
        xc = np.clip(want, 0, 31)
        exp = 0.1 + 0.01 * xc[None, None, :] + 0.02 * y[..., None] + 0.03 * z[..., None]
        np.testing.assert_allclose(warped, exp, rtol=0, atol=1e-6)


def test_swapping_grids_swaps_direction():
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=2)
    d1, _ = rp.transform(1, X[0])
    d0, _ = rp.transform(0, X[0][::-1])
    assert np.array_equal(d1, d0)
    d1, _ = rp.transform(0, X[1])
    d0, _ = rp.transform(1, X[1][::-1])
    assert np.array_equal(d1, d0)


def test_barycentric_coordinates_carry_over():
    """For a deformed feasible pair every voxel is covered, and the mapped point
    has, in the other grid's tetrahedron, the barycentric coordinates the voxel
    has in its own (checked by linear solves on sampled voxels)."""
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=1)[0]
    tets = rp.tets()
    rng = np.random.default_rng(5)
    for own in (0, 1):
        dvf, warped = rp.transform(own, X)
        assert np.all(np.isfinite(dvf)) and np.all(np.isfinite(warped))
        owner, count = rp.owner_bruteforce(X[own])
        assert np.all(count >= 1)
        for _ in range(200):
            k, j, i = (int(a) for a in rng.integers(0, 32, 3))
            t = owner[k, j, i]
            Vo = X[own][tets[t]].astype(np.float64)   # [4][3]
            Vt = X[1 - own][tets[t]].astype(np.float64)
            A = np.vstack([Vo.T, np.ones(4)])
            lam = np.linalg.solve(A, np.array([i, j, k, 1.0]))
            assert lam.min() > -1e-9
            x = np.array([i, j, k]) + dvf[k, j, i]
            mu = np.linalg.solve(np.vstack([Vt.T, np.ones(4)]), np.append(x, 1.0))
            np.testing.assert_allclose(mu, lam, rtol=0, atol=1e-9)
