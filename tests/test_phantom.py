"""The synthetic phantom (Sec. 3): the cube's faces are pushed in by 3-D
parabolas, the central sphere shrinks, and the guidance pairs lie on the two
spheres along shared directions."""
import numpy as np

from paper_2202_11001_amd import workloads as W


def test_phantom_geometry():
    w = W.phantom()
    c = np.full(3, 24.5)
    src, tgt = w.moving, w.fixed
    assert src.shape == tgt.shape == (50, 50, 50) and w.mesh == (6, 6, 6)
    # face centres: the source cube reaches half = 15 from the centre, the target only half - depth = 9
    ci = 24  # a voxel row next to the centre axis
    row_s = src[ci, ci, :] > 0.25
    row_t = tgt[ci, ci, :] > 0.25
    assert row_s.sum() in (30, 31) and row_t.sum() in (18, 19)
    # face corners keep their position (the parabola vanishes at the face edges)
    assert src[11, 11, 11] > 0.25 and tgt[11, 11, 11] > 0.25
    # the sphere shrinks from radius 9 to 5
    assert (src > 0.75).sum() > 4 * (tgt > 0.75).sum()
    # the phantom is symmetric under swapping axes
    assert np.allclose(tgt, tgt.transpose(2, 1, 0), atol=1e-6) and np.allclose(src, src.transpose(1, 0, 2), atol=1e-6)
    rs = np.linalg.norm(w.guid_moving - c, axis=1)
    rt = np.linalg.norm(w.guid_fixed - c, axis=1)
    assert np.allclose(rs, 9.0, atol=0.01) and np.allclose(rt, 5.0, atol=0.01)
    ds = (w.guid_moving - c) / rs[:, None]
    dt = (w.guid_fixed - c) / rt[:, None]
    assert np.all(np.sum(ds * dt, axis=1) > 0.999)
    assert np.array_equal(w.corr_moving, w.corr_fixed)
