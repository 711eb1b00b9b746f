"""GPU parity of dsm_transform (the registration's DVF and transformed image,
Sec. 2.1 / Fig. 2) against the FP64 oracle: every voxel on small and ragged
workloads, sampled voxels at 512x512x100 and at 512^3, the largest size."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"
DVF_ATOL = 1e-5    # FP64 map rounded to FP32 (positions below 512 voxels: ulp <= 3e-5 relative to 512)
IMG_ATOL = 1e-6


def _say(msg):
    print(f"[gpu-transform] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _ragged():
    rng = np.random.default_rng(3)
    dims = (37, 23, 19)
    shp = dims[::-1]
    fixed = W._blur(rng.uniform(0, 1, shp), 1.0).astype(np.float32)
    moving = W._blur(rng.uniform(0, 1, shp), 1.0).astype(np.float32)
    return W.Workload("ragged-37x23x19", moving, fixed, (5, 4, 3), (1.0, 1.0, 1.0), 0.2, 3, 1.5, 1.0, 7, 8)


WORKLOADS = {"tiny": W.tiny, "ragged": _ragged, "batched": W.batched}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_transform_matches_oracle(name):
    w = WORKLOADS[name]()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=2)
    gp = dsm.Problem.from_workload(w)
    for s in range(2):
        for own in (0, 1):
            _say(f"{w.name} solution {s} own {own}")
            d, m = gp.transform(_t(X[s]), own=own)
            rd, rm = rp.transform(own, X[s])
            d, m = d.cpu().numpy(), m.cpu().numpy()
            assert np.all(np.isfinite(rd)) and np.all(np.isfinite(d)) and np.all(np.isfinite(m))
            np.testing.assert_allclose(d, rd, rtol=0, atol=DVF_ATOL)
            np.testing.assert_allclose(m, rm, rtol=0, atol=IMG_ATOL)
    # outputs are optional
    d, m = gp.transform(_t(X[0]), own=1, dvf=False)
    assert d is None and np.allclose(m.cpu().numpy(), rp.transform(1, X[0])[1], atol=IMG_ATOL)
    d, m = gp.transform(_t(X[0]), own=1, dvf=False, warped=False)
    assert d is None and m is None
    with pytest.raises(dsm.DsmError):
        gp.transform(_t(X[0]), own=2)


def test_transform_identity_closed_form():
    w = W.tiny()
    gp = dsm.Problem.from_workload(w)
    I = gp.topology()["identity"]
    X2 = _t(np.stack([I, I]))
    for own, other in ((1, w.moving), (0, w.fixed)):
        d, m = gp.transform(X2, own=own)
        assert float(d.abs().max()) < 1e-6
        np.testing.assert_allclose(m.cpu().numpy(), other, rtol=0, atol=1e-7)


def test_transform_clinical_sampled():
    """512x512x100 with the clinical mesh: every voxel covered; on sampled
    voxels the oracle locates the voxel by testing every tetrahedron, maps it
    with barycentric coordinates from a linear solve and samples the other image
    there."""
    w = W.clinical()
    _say(f"{w.name}")
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=1)[0]
    gp = dsm.Problem.from_workload(w, max_solutions=1, max_fos=1)
    tets = rp.tets()
    rng = np.random.default_rng(11)
    Dz, Dy, Dx = w.fixed.shape
    for own in (1, 0):
        d, m = gp.transform(_t(X), own=own)
        d, m = d.cpu().numpy(), m.cpu().numpy()
        assert np.all(np.isfinite(d)) and np.all(np.isfinite(m))
        L = np.rint((X[own].astype(np.float64) + 0.5) * 128)   # lattice coordinates
        for _ in range(60):
            v = np.array([rng.integers(0, Dx), rng.integers(0, Dy), rng.integers(0, Dz)])
            U = 128.0 * v + 64.0
            owners = [t for t in range(rp.T) if ref.lib().ref_inside(ref._p(np.ascontiguousarray(L[tets[t]])),
                                                                      ref._p(np.ascontiguousarray(U)))]
            assert len(owners) == 1
            t = owners[0]
            lam = np.linalg.solve(np.vstack([X[own][tets[t]].astype(np.float64).T, np.ones(4)]), np.append(v, 1.0))
            x = lam @ X[1 - own][tets[t]].astype(np.float64)
            np.testing.assert_allclose(v + d[v[2], v[1], v[0]], x, rtol=0, atol=1e-4)
            np.testing.assert_allclose(m[v[2], v[1], v[0]], rp.trilinear(1 - own, x), rtol=0, atol=1e-5)


def test_transform_maximum_size_sampled():
    """512^3 images (the largest the exact lattice predicates support), 4^3
    meshes: every voxel covered, and sampled voxels against the oracle's exact
    location, a linear solve and its trilinear sample."""
    shape = (512, 512, 512)
    rng = np.random.default_rng(8)
    coarse = rng.uniform(0, 1, (17, 17, 17)).astype(np.float32)
    from scipy import ndimage
    fixed = ndimage.zoom(coarse, 512 / 17, order=1)[:512, :512, :512].astype(np.float32)
    moving = np.roll(fixed, 3, axis=2)
    w = W.Workload("max-512^3", moving, fixed, (4, 4, 4), (1.0, 1.0, 1.0), 0.2, 1, 6.0, 4.0, 51, 52)
    _say(w.name)
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=1)[0]
    gp = dsm.Problem.from_workload(w, max_solutions=1, max_fos=1)
    tets = rp.tets()
    vox = rng.integers(0, 512, (40, 3))
    for own in (1, 0):
        d, m = gp.transform(_t(X), own=own)
        assert not bool(torch.isnan(d).any()) and not bool(torch.isnan(m).any())
        iz, iy, ix = (torch.from_numpy(vox[:, a]).to(DEV) for a in (2, 1, 0))
        ds, ms = d[iz, iy, ix].cpu().numpy(), m[iz, iy, ix].cpu().numpy()
        del d, m
        L = np.rint((X[own].astype(np.float64) + 0.5) * 128)
        for n, v in enumerate(vox):
            U = 128.0 * v + 64.0
            owners = [t for t in range(rp.T) if ref.lib().ref_inside(ref._p(np.ascontiguousarray(L[tets[t]])),
                                                                      ref._p(np.ascontiguousarray(U)))]
            assert len(owners) == 1
            t = owners[0]
            lam = np.linalg.solve(np.vstack([X[own][tets[t]].astype(np.float64).T, np.ones(4)]), np.append(v, 1.0))
            x = lam @ X[1 - own][tets[t]].astype(np.float64)
            np.testing.assert_allclose(v + ds[n], x, rtol=0, atol=2e-4)
            np.testing.assert_allclose(ms[n], rp.trilinear(1 - own, x), rtol=0, atol=1e-5)
