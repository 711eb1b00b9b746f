"""Pins of the oracle's guidance term (Sec. 2.3.3) under deformation.

A guidance point of one image is located in that image's own grid, carried by
the piecewise-affine map of the dual meshes onto the other grid, and scored by
its squared mm distance to the nearest point of the same correspondence in the
other image, in both directions; the sum is divided by the number of points.

Two pins that do not use the oracle's arithmetic:
* a closed form under a known piecewise-affine map: the target grid is the
  undeformed grid with one interior x-plane of points shifted along x, so the
  map is a 1-D piecewise-linear function of x alone;
* an independent numpy evaluation on random feasible meshes in both grids:
  the owning tetrahedron from non-negative barycentric coordinates solved by
  np.linalg.solve (the map is continuous, so any tetrahedron containing the
  point gives the same image), the map by those coordinates, the nearest
  same-correspondence point by brute force.
"""
import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W


def _guidance_points(rng, dims, n_mov, n_fix, n_corr):
    hi = np.array(dims, np.float64) - 1.0
    gm = W.snap(rng.uniform(0, 1, (n_mov, 3)) * hi)
    gf = W.snap(rng.uniform(0, 1, (n_fix, 3)) * hi)
    # every correspondence gets at least one point on each image, some get several
    cm = np.concatenate([np.arange(n_corr), rng.integers(0, n_corr, n_mov - n_corr)]).astype(np.int32)
    cf = np.concatenate([np.arange(n_corr), rng.integers(0, n_corr, n_fix - n_corr)]).astype(np.int32)
    return gm, cm, gf, cf


def _nearest_sq(pt, others, corr_others, c, sp):
    d = [np.sum(((pt - q) * sp) ** 2) for q, cq in zip(others, corr_others) if cq == c]
    return min(d)


def _problem(dims, mesh, sp, guid):
    z = np.zeros(dims[::-1], np.float32)
    gm, cm, gf, cf = guid
    return ref.Problem(z, z, mesh, sp, 0.1, guid_moving=gm, corr_moving=cm, guid_fixed=gf, corr_fixed=cf)


@pytest.mark.parametrize("delta", [2.0, -3.5])
def test_guidance_plane_shift_closed_form(delta):
    """Source grid undeformed; target grid with the x-plane of index 1 moved by
    delta voxels.  Every tetrahedron lies between two adjacent x-planes and its
    vertices keep y and z, so the map source -> target is
    (x, y, z) -> (phi(x), y, z) with phi piecewise linear through the plane
    positions; target points map back by the inverse of phi."""
    dims, mesh, sp = (24, 20, 16), (4, 3, 3), np.array([1.0, 1.5, 2.0])
    rng = np.random.default_rng(7)
    guid = _guidance_points(rng, dims, 9, 8, 4)
    p = _problem(dims, mesh, sp, guid)
    I = p.identity()
    Xt = I.copy()
    nx = mesh[0]
    plane1 = np.arange(p.P) % nx == 1
    Xt[plane1, 0] = I[plane1, 0] + np.float32(delta)
    X = np.stack([I, Xt])[None]
    flags, _ = p.fold_check(X)
    assert flags[0] == 0
    obj, _ = p.eval_full(X)

    a = np.array(sorted(set(I[:, 0].astype(np.float64))))   # source plane positions
    b = a.copy()
    b[1] += delta                                             # target plane positions
    phi = lambda x: np.interp(x, a, b)
    phi_inv = lambda x: np.interp(x, b, a)
    gm, cm, gf, cf = (np.asarray(v, np.float64) if v.dtype.kind == "f" else v for v in guid)
    tot = 0.0
    for q, c in zip(gm, cm):
        tot += _nearest_sq(np.array([phi(q[0]), q[1], q[2]]), gf, cf, c, sp)
    for q, c in zip(gf, cf):
        tot += _nearest_sq(np.array([phi_inv(q[0]), q[1], q[2]]), gm, cm, c, sp)
    expect = tot / (len(gm) + len(gf))
    assert obj[0, 2] == pytest.approx(expect, rel=1e-12)
    # the undeformed pair differs: the map is not the identity on these points
    obj0, _ = p.eval_full(np.stack([I, I])[None])
    assert abs(obj0[0, 2] - expect) > 1e-3 * expect


def _independent_guidance(tets, X2, gm, cm, gf, cf, sp):
    """Guidance objective of one solution X2 [2][P][3] by numpy."""
    pts = (np.asarray(gm, np.float64), np.asarray(gf, np.float64))
    corr = (cm, cf)
    tot = 0.0
    for g in (0, 1):
        own = X2[g].astype(np.float64)[tets]        # [T][4][3]
        oth = X2[1 - g].astype(np.float64)[tets]
        A = np.concatenate([own.transpose(0, 2, 1), np.ones((len(tets), 1, 4))], axis=1)  # [T][4][4]
        for q, c in zip(pts[g], corr[g]):
            lam = np.linalg.solve(A, np.broadcast_to(np.append(q, 1.0), (len(tets), 4))[..., None])[..., 0]
            hit = np.nonzero(np.all(lam >= -1e-9, axis=1))[0]
            assert len(hit) >= 1
            mapped = lam[hit[0]] @ oth[hit[0]]
            tot += _nearest_sq(mapped, pts[1 - g], corr[1 - g], c, sp)
    return tot / (len(pts[0]) + len(pts[1]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_guidance_vs_numpy_on_deformed_meshes(seed):
    dims, mesh, sp = (22, 18, 14), (4, 4, 3), np.array([1.0, 1.2, 2.0])
    rng = np.random.default_rng(100 + seed)
    guid = _guidance_points(rng, dims, 7, 6, 3)
    p = _problem(dims, mesh, sp, guid)
    X = W.population(dims, mesh, 3, 1.6, 200 + seed, reject=lambda X: p.fold_check(X)[0] != 0)
    obj, flags = p.eval_full(X)
    assert np.all(flags == 0)
    tets = p.tets()
    for s in range(len(X)):
        expect = _independent_guidance(tets, X[s], *guid, sp)
        assert obj[s, 2] == pytest.approx(expect, rel=1e-9)
    # the solutions are deformed enough for the map to matter
    ident = _independent_guidance(tets, np.stack([p.identity(), p.identity()]), *guid, sp)
    assert np.all(np.abs(obj[:, 2] - ident) > 1e-3 * ident)
