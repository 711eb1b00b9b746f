"""Seeded synthetic inputs for dual simplex-mesh registration.

This module only draws inputs: images, mesh-point populations, FOS candidates
and guidance point pairs.  It contains none of the method's arithmetic (no
rasterisation, sampling, objectives or constraint tests), so both the GPU
library's tests and the CPU oracle can be fed from it.  A fold test, where a
draw must be feasible, is passed in by the caller (``reject``).

Conventions shared by every consumer: images are float32 ``[Dz][Dy][Dx]``
(x fastest); grid point (i, j, k) of an ``(nx, ny, nz)`` mesh has index
``i + nx * (j + ny * k)``; coordinates are float32 voxel units whose value
``(x + 0.5) * 128`` is an integer (the 1/128-voxel lattice); populations are
``[S][2][P][3]`` with grid 0 on the source ("moving") image and grid 1 on the
target ("fixed") image.

The paper's inputs (a clinical CT pair and a synthetic cube phantom whose
parameters are not printed) are not available; the generators below stand in
for them with the shapes, intensity ranges and deformation magnitudes stated
for each configuration.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LAT = 128.0


# --------------------------------------------------------------------- lattice

def snap(x):
    """Round voxel-unit coordinates to the 1/128-voxel lattice (half to even)."""
    x = np.asarray(x, dtype=np.float64)
    return (np.rint((x + 0.5) * LAT) / LAT - 0.5).astype(np.float32)


def regular_grid(dims, mesh):
    """Undeformed mesh points [P][3] spanning the image box [-0.5, D-0.5]:
    point i of n on an axis of D voxels at lattice round-half-up(i*128*D/(n-1))."""
    dims = [int(d) for d in dims]
    mesh = [int(n) for n in mesh]
    axes = []
    for D, n in zip(dims, mesh):
        i = np.arange(n, dtype=np.int64)
        u = (2 * i * 128 * D + (n - 1)) // (2 * (n - 1))
        axes.append(u.astype(np.float64) / LAT - 0.5)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float32)


def free_mask(mesh):
    """[P][3] bool: coordinate a of point p may move (border points stay on their border)."""
    nx, ny, nz = (int(n) for n in mesh)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = [i.ravel(), j.ravel(), k.ravel()]
    return np.stack([(idx[a] > 0) & (idx[a] < (nx, ny, nz)[a] - 1) for a in range(3)], axis=1)


def _clip_box(x, dims):
    hi = np.asarray(dims, dtype=np.float64) - 0.5
    return np.clip(x, -0.5, hi)


def population(dims, mesh, S, sigma, seed, reject=None, max_redraw=50):
    """S solutions [S][2][P][3]: the undeformed grid in both grids plus
    N(0, sigma) voxels on free coordinates, snapped.  ``reject(X) -> bool[S]``
    marks draws to redraw (e.g. folded ones)."""
    rng = np.random.default_rng(seed)
    base = regular_grid(dims, mesh).astype(np.float64)
    free = free_mask(mesh)
    P = base.shape[0]

    def draw(n):
        d = rng.normal(0.0, sigma, size=(n, 2, P, 3)) * free[None, None]
        return snap(_clip_box(base[None, None] + d, dims))

    X = draw(S)
    if reject is not None:
        for _ in range(max_redraw):
            bad = np.nonzero(np.asarray(reject(X)))[0]
            if len(bad) == 0:
                break
            X[bad] = draw(len(bad))
    return X


def single_point_fos(P):
    """FOS of single grid points as CSR (offsets [F+1], points)."""
    return np.arange(P + 1, dtype=np.int32), np.arange(P, dtype=np.int32)


def candidates(X, fos_off, fos_pts, mesh, dims, sigma, seed, K=1):
    """Candidate coordinates [S][fos_off[F]][2][3] (K=1) or [S][F*..][K]...:
    current position + N(0, sigma) on free coordinates, both grids, snapped.
    With K > 1 the layout is [S][F][K][|f|][2][3] flattened per element."""
    rng = np.random.default_rng(seed)
    S = X.shape[0]
    free = free_mask(mesh)[fos_pts]  # [n][3]
    cur = X[:, :, fos_pts, :].transpose(0, 2, 1, 3).astype(np.float64)  # [S][n][2][3]
    if K == 1:
        d = rng.normal(0.0, sigma, size=cur.shape) * free[None, :, None, :]
        return snap(_clip_box(cur + d, dims))
    d = rng.normal(0.0, sigma, size=(S, K) + cur.shape[1:]) * free[None, None, :, None, :]
    return snap(_clip_box(cur[:, None] + d, dims))  # [S][K][n][2][3]


# --------------------------------------------------------------------- images

def _grid(shape):
    Dz, Dy, Dx = shape
    z, y, x = np.meshgrid(np.arange(Dz, dtype=np.float64), np.arange(Dy, dtype=np.float64),
                          np.arange(Dx, dtype=np.float64), indexing="ij")
    return x, y, z


def ellipsoid(shape, centre, semi, coords=None):
    x, y, z = coords if coords is not None else _grid(shape)
    r = ((x - centre[0]) / semi[0]) ** 2 + ((y - centre[1]) / semi[1]) ** 2 + ((z - centre[2]) / semi[2]) ** 2
    return r <= 1.0


@dataclass
class Workload:
    name: str
    moving: np.ndarray          # source image [Dz][Dy][Dx] float32
    fixed: np.ndarray           # target image
    mesh: tuple
    spacing: tuple
    tau: float
    S: int
    sigma_pop: float
    sigma_cand: float
    seed_pop: int
    seed_cand: int
    guid_moving: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.float32))
    guid_fixed: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.float32))
    corr_moving: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    corr_fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def dims(self):
        Dz, Dy, Dx = self.fixed.shape
        return (Dx, Dy, Dz)

    @property
    def P(self):
        return int(np.prod(self.mesh))

    def population(self, reject=None, S=None):
        return population(self.dims, self.mesh, S or self.S, self.sigma_pop, self.seed_pop, reject)

    def fos(self):
        return single_point_fos(self.P)

    def candidates(self, X, fos_off=None, fos_pts=None, K=1, seed=None):
        if fos_off is None:
            fos_off, fos_pts = self.fos()
        return candidates(X, fos_off, fos_pts, self.mesh, self.dims, self.sigma_cand,
                          self.seed_cand if seed is None else seed, K)


def tiny(seed_shift=0):
    """32^3 ellipsoid pair (intensity 1 on 0, noise sigma 0.02; source ellipsoid
    1.3x longer in z), 3x3x3 meshes, 16 solutions, 4 guidance pairs."""
    shape = (32, 32, 32)
    c = (15.5, 15.5, 15.5)
    fixed = ellipsoid(shape, c, (10, 8, 6)).astype(np.float64)
    moving = ellipsoid(shape, c, (10, 8, 7.8)).astype(np.float64)
    fixed += np.random.default_rng(11 + seed_shift).normal(0, 0.02, shape)
    moving += np.random.default_rng(12 + seed_shift).normal(0, 0.02, shape)
    gm = snap([[25.5, 15.5, 15.5], [5.5, 15.5, 15.5], [15.5, 15.5, 23.3], [15.5, 15.5, 7.7]])
    gf = snap([[25.5, 15.5, 15.5], [5.5, 15.5, 15.5], [15.5, 15.5, 21.5], [15.5, 15.5, 9.5]])
    return Workload("tiny-32^3", moving.astype(np.float32), fixed.astype(np.float32), (3, 3, 3),
                    (1.0, 1.0, 1.0), 0.1, 16, 1.0, 1.0, 13 + seed_shift, 14 + seed_shift,
                    gm, gf, np.arange(4, dtype=np.int32), np.arange(4, dtype=np.int32))


def _blur(vol, sigma):
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(vol, sigma=sigma, mode="nearest")


def _two_ellipsoids(shape, coords, scale=1.0):
    s = scale
    e1 = ellipsoid(shape, (26 * s, 32 * s, 32 * s), (14 * s, 10 * s, 9 * s), coords) * 0.8
    e2 = ellipsoid(shape, (38 * s, 30 * s, 34 * s), (9 * s, 13 * s, 8 * s), coords) * 0.6
    return np.minimum(e1 + e2, 1.0)


def batched(shape=(64, 64, 64), mesh=(5, 5, 5), S=96, seed=21):
    """Two overlapping blurred ellipsoids; the source is the target content under
    a 10% shear in x along y and a translation of 6 voxels in x (scaled with the
    volume), 8 guidance pairs on the ellipsoid surfaces."""
    Dz, Dy, Dx = shape
    sc = Dx / 64.0
    x, y, z = _grid(shape)
    fixed = _blur(_two_ellipsoids(shape, (x, y, z), sc), 1.5)
    cy = Dy / 2.0
    # source point q shows target content at A^-1 (q - t): x_t = q_x - 6 s - 0.1 (q_y - cy)
    xs = x - 6 * sc - 0.1 * (y - cy)
    moving = _blur(_two_ellipsoids(shape, (xs, y, z), sc), 1.5)
    rng = np.random.default_rng(seed + 3)
    pts = []
    for centre, semi in (((26, 32, 32), (14, 10, 9)), ((38, 30, 34), (9, 13, 8))):
        for _ in range(4):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            pts.append(np.array(centre) * sc + np.array(semi) * sc * d)
    gf = np.array(pts)
    gm = gf.copy()
    gm[:, 0] = gf[:, 0] + 6 * sc + 0.1 * (gf[:, 1] - cy)
    hi = np.array([Dx - 1, Dy - 1, Dz - 1], dtype=np.float64)
    gf = snap(np.clip(gf, 0, hi))
    gm = snap(np.clip(gm, 0, hi))
    n = len(gf)
    return Workload(f"batched-{Dx}x{Dy}x{Dz}", moving.astype(np.float32), fixed.astype(np.float32), tuple(mesh),
                    (1.0, 1.0, 1.0), 0.01, S, 1.0, 1.0, seed + 1, seed + 2, gm, gf,
                    np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32))


def _bspline_basis(n_out, spacing, n_ctrl):
    """[n_out][n_ctrl] uniform cubic B-spline basis, control point c at (c-1)*spacing."""
    t = np.arange(n_out, dtype=np.float64) / spacing + 1.0
    c = np.arange(n_ctrl, dtype=np.float64)
    u = np.abs(t[:, None] - c[None, :])
    B = np.where(u < 1, 2.0 / 3.0 - u ** 2 + 0.5 * u ** 3, np.where(u < 2, (2 - u) ** 3 / 6.0, 0.0))
    return B


def clinical(shape=(100, 512, 512), mesh=(10, 10, 6), S=512, seed=31, n_guid=20):
    """CT-shaped pair: int16 HU (air -1000, soft tissue N(40,20), bone N(700,150),
    smoothed ellipsoidal blobs) mapped to [0,1]; the source is the target under a
    smooth cubic B-spline displacement of up to 25 mm plus a content-mismatch
    region covering ~20% of the body.  Voxel spacing 0.977 x 0.977 x 3 mm."""
    Dz, Dy, Dx = shape
    spacing = (0.9765625, 0.9765625, 3.0)
    rng = np.random.default_rng(seed)
    x, y, z = _grid(shape)
    cx, cy = (Dx - 1) / 2.0, (Dy - 1) / 2.0
    ax, ay = 230.0 * Dx / 512, 170.0 * Dy / 512
    body = ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 <= 1.0
    hu = np.full(shape, -1000.0)
    hu[body] = rng.normal(40, 20, size=int(body.sum()))
    for b in range(24):
        c = np.array([cx + rng.uniform(-0.7, 0.7) * ax, cy + rng.uniform(-0.7, 0.7) * ay,
                      rng.uniform(0.15, 0.85) * (Dz - 1)])
        r = np.array([rng.uniform(10, 60) * Dx / 512, rng.uniform(10, 60) * Dy / 512, rng.uniform(3, 15) * Dz / 100])
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, [Dx, Dy, Dz])
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        m = ellipsoid(None, c, r, (x[sl], y[sl], z[sl])) & body[sl]
        if b % 2 == 0:
            hu[sl][m] = rng.normal(700, 150, size=int(m.sum()))
        else:
            hu[sl][m] = rng.normal(40 + rng.uniform(-40, 40), 20, size=int(m.sum()))
    for _ in range(4):
        c = np.array([cx + rng.uniform(-0.5, 0.5) * ax, cy + rng.uniform(-0.5, 0.5) * ay,
                      rng.uniform(0.2, 0.8) * (Dz - 1)])
        r = np.array([rng.uniform(8, 25) * Dx / 512, rng.uniform(8, 25) * Dy / 512, rng.uniform(2, 6) * Dz / 100])
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int) + 1, [Dx, Dy, Dz])
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        m = ellipsoid(None, c, r, (x[sl], y[sl], z[sl]))
        hu[sl][m] = -1000.0
    del x, y, z
    hu = _blur(hu, (0.7, 1.5, 1.5))
    fixed_hu = np.clip(np.rint(hu), -32768, 32767).astype(np.int16)
    del hu
    # smooth displacement u (voxel units), control spacing 64 x 64 x 20 voxels
    sp_ctrl = (64.0, 64.0, 20.0)
    nctrl = [int(np.ceil(D / s)) + 3 for D, s in zip((Dx, Dy, Dz), sp_ctrl)]
    coef = np.random.default_rng(seed + 1).normal(size=(3, nctrl[2], nctrl[1], nctrl[0]))
    Bx = _bspline_basis(Dx, sp_ctrl[0], nctrl[0])
    By = _bspline_basis(Dy, sp_ctrl[1], nctrl[1])
    Bz = _bspline_basis(Dz, sp_ctrl[2], nctrl[2])
    u = np.einsum("ckji,xi->ckjx", coef, Bx)
    u = np.einsum("ckjx,yj->ckyx", u, By)
    u = np.einsum("ckyx,zk->czyx", u, Bz)  # [3][Dz][Dy][Dx] arbitrary units
    mm = np.sqrt(sum((u[a] * spacing[a]) ** 2 for a in range(3)))
    u *= 25.0 / mm.max()
    del mm
    from scipy.ndimage import map_coordinates
    zz, yy, xx = np.meshgrid(np.arange(Dz, dtype=np.float32), np.arange(Dy, dtype=np.float32),
                             np.arange(Dx, dtype=np.float32), indexing="ij")
    coords = np.stack([zz + u[2] / spacing[2], yy + u[1] / spacing[1], xx + u[0] / spacing[0]])
    del zz, yy, xx
    mov = map_coordinates(fixed_hu.astype(np.float32), coords, order=1, mode="nearest")
    del coords
    # content mismatch: an ellipsoid of ~20% of the body volume refilled with N(10, 15) HU
    rng3 = np.random.default_rng(seed + 2)
    frac = 0.2 ** (1.0 / 3.0)
    c = np.array([cx + rng3.uniform(-0.2, 0.2) * ax, cy + rng3.uniform(-0.2, 0.2) * ay, (Dz - 1) / 2.0])
    r = np.array([ax * frac, ay * frac, (Dz / 2.0) * frac * 1.2])
    x, y, z = _grid(shape)
    m = ellipsoid(None, c, r, (x, y, z)) & body
    del x, y, z
    mov[m] = rng3.normal(10, 15, size=int(m.sum()))
    moving_hu = np.clip(np.rint(mov), -32768, 32767).astype(np.int16)
    del mov, m

    def norm(h):
        return np.clip((h.astype(np.float32) + 1000.0) / 2000.0, 0.0, 1.0).astype(np.float32)

    # guidance: source points inside the body, target point = p + u(p)
    rg = np.random.default_rng(seed + 5)
    gm, gf = [], []
    while len(gm) < n_guid:
        p = np.array([cx + rg.uniform(-0.6, 0.6) * ax, cy + rg.uniform(-0.6, 0.6) * ay, rg.uniform(0.1, 0.9) * (Dz - 1)])
        if ((p[0] - cx) / ax) ** 2 + ((p[1] - cy) / ay) ** 2 > 0.8:
            continue
        i, j, k = (int(round(p[0])), int(round(p[1])), int(round(p[2])))
        q = p + np.array([u[0][k, j, i], u[1][k, j, i], u[2][k, j, i]]) / np.array(spacing)
        q = np.clip(q, 0, [Dx - 1, Dy - 1, Dz - 1])
        gm.append(p)
        gf.append(q)
    del u
    n = len(gm)
    return Workload(f"clinical-{Dx}x{Dy}x{Dz}", norm(moving_hu), norm(fixed_hu), tuple(mesh), spacing, 0.02, S,
                    2.0, 1.0, seed + 3, seed + 4, snap(gm), snap(gf),
                    np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32))


def phantom(shape=(50, 50, 50), mesh=(6, 6, 6), S=250, seed=41, half=15.0, depth=6.0, r_source=9.0,
            r_target=5.0, n_guid=16):
    """Replica of the synthetic problem of Sec. 3: a cube deformed in a
    non-affine way, with a shrinking sphere at its centre.  The paper prints no
    parameters; here the source holds an axis-aligned cube of half-width `half`
    voxels (intensity 0.5) around a sphere of radius `r_source` (intensity 1);
    in the target every face of the cube is pushed towards the centre by a 3-D
    parabola, depth(u, v) = depth * max(0, 1 - (u^2 + v^2) / half^2) over face
    coordinates (u, v) from the face centre, and the sphere has shrunk to
    `r_target`.  Both images are blurred (sigma 1 voxel); background 0, empty
    threshold 0.05; spacing 1 mm.  Guidance: `n_guid` points spread evenly over
    the source sphere (a Fibonacci lattice) and the same directions on the
    target sphere, one correspondence each."""
    Dz, Dy, Dx = shape
    x, y, z = _grid(shape)
    c = np.array([(Dx - 1) / 2.0, (Dy - 1) / 2.0, (Dz - 1) / 2.0])
    d = [x - c[0], y - c[1], z - c[2]]
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    src = np.where(np.maximum.reduce([np.abs(a) for a in d]) <= half, 0.5, 0.0)
    src[r <= r_source] = 1.0
    inside = np.ones(shape, dtype=bool)
    for a in range(3):
        u, v = d[(a + 1) % 3], d[(a + 2) % 3]
        inset = depth * np.maximum(0.0, 1.0 - (u ** 2 + v ** 2) / half ** 2)
        inside &= np.abs(d[a]) <= half - inset
    tgt = np.where(inside, 0.5, 0.0)
    tgt[r <= r_target] = 1.0
    k = np.arange(n_guid) + 0.5
    polar = np.arccos(1.0 - 2.0 * k / n_guid)
    azim = np.pi * (1.0 + 5.0 ** 0.5) * k
    dirs = np.stack([np.cos(azim) * np.sin(polar), np.sin(azim) * np.sin(polar), np.cos(polar)], axis=1)
    gm = snap(c + r_source * dirs)
    gf = snap(c + r_target * dirs)
    ids = np.arange(n_guid, dtype=np.int32)
    return Workload(f"phantom-{Dx}x{Dy}x{Dz}", _blur(src, 1.0).astype(np.float32), _blur(tgt, 1.0).astype(np.float32),
                    tuple(mesh), (1.0, 1.0, 1.0), 0.05, S, 1.0, 1.0, seed + 1, seed + 2, gm, gf, ids, ids.copy())


def ramp(shape, coef=(0.01, 0.02, 0.03), offset=0.1):
    """Linear ramp image I(x, y, z) = offset + coef . (x, y, z) (float32)."""
    x, y, z = _grid(shape)
    return (offset + coef[0] * x + coef[1] * y + coef[2] * z).astype(np.float32)


UNEVEN_PROBLEMS = [  # (shape (Dz, Dy, Dx), mesh (nx, ny, nz), population)
    ((96, 96, 96), (4, 4, 4), 64), ((128, 128, 128), (5, 5, 5), 96), ((80, 192, 192), (6, 6, 4), 128),
    ((64, 256, 256), (8, 8, 6), 256), ((96, 96, 96), (5, 5, 5), 128), ((128, 128, 128), (6, 6, 6), 64),
    ((80, 192, 192), (8, 8, 6), 192), ((64, 256, 256), (7, 7, 5), 160), ((96, 96, 96), (8, 8, 6), 96),
    ((128, 128, 128), (4, 4, 4), 256), ((80, 192, 192), (5, 5, 4), 64), ((64, 256, 256), (6, 6, 5), 192),
]


def downsample2(img):
    """2x2x2 box average (all dims even)."""
    Dz, Dy, Dx = img.shape
    return img.reshape(Dz // 2, 2, Dy // 2, 2, Dx // 2, 2).mean(axis=(1, 3, 5)).astype(np.float32)


def uneven(indices=None, level=1):
    """Several registration problems of uneven volume and mesh size: the
    two-ellipsoid pair scaled to each shape (seed 100 + i); level 0 is the
    2x2x2 box-averaged pyramid level (populations drawn there, sigma halved),
    level 1 the full resolution."""
    out = []
    for i in (indices if indices is not None else range(len(UNEVEN_PROBLEMS))):
        shape, mesh, S = UNEVEN_PROBLEMS[i]
        w = batched(shape=shape, mesh=mesh, S=S, seed=100 + 4 * i)
        w.name = f"uneven-{i}-{shape[2]}x{shape[1]}x{shape[0]}"
        if level == 0:
            w.moving, w.fixed = downsample2(w.moving), downsample2(w.fixed)
            hi = np.array([shape[2] // 2 - 1, shape[1] // 2 - 1, shape[0] // 2 - 1], dtype=np.float64)
            w.guid_moving = snap(np.clip((w.guid_moving.astype(np.float64) - 0.5) / 2, 0, hi))
            w.guid_fixed = snap(np.clip((w.guid_fixed.astype(np.float64) - 0.5) / 2, 0, hi))
            w.sigma_pop, w.sigma_cand = w.sigma_pop / 2, w.sigma_cand / 2
            w.name += "-half"
        out.append(w)
    return out


def upsample_population(X_half):
    """Hand-off from the half-resolution level: voxel coordinate x at half
    resolution is 2 x + 0.5 at full resolution (lattice u -> 2 u, exact)."""
    return (2.0 * np.asarray(X_half, dtype=np.float64) + 0.5).astype(np.float32)


def tetrahedron_fos(tets, n_cubes, seed):
    """The paper's FOS for partial changes: per cube, one of its 6 tetrahedra
    (tetrahedron 6 c + r of cube c, r drawn uniformly), whose 4 points change
    together.  tets [T][4] is the mesh topology (tetrahedra numbered cube by
    cube).  Returns CSR (offsets [F+1], points)."""
    rng = np.random.default_rng(seed)
    r = rng.integers(0, 6, size=n_cubes)
    pts = np.asarray(tets, dtype=np.int32)[6 * np.arange(n_cubes) + r].reshape(-1)
    return (4 * np.arange(n_cubes + 1)).astype(np.int32), pts.astype(np.int32)
