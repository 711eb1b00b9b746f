"""Pins of the surrogate reference (oracle/surrogate_ref.py): backward pass
against finite differences, bfloat16 rounding, Adam's first step, and feature
invariants."""
import numpy as np
import pytest

from oracle import ref
from oracle import surrogate_ref as R
from paper_2202_11001_amd import workloads as W


def _params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, R.NPARAMS)
    p[R.W3 + R.OUT * R.HID:R.B3] = 0.0
    p[R.B3 + R.OUT:] = 0.0
    return p


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = _params(1)
    x = rng.normal(size=(7, R.IN))
    t = rng.normal(size=(7, R.OUT))
    loss, g = R.loss_and_grad(p, x, t, bf16_round=False)
    idx = np.concatenate([rng.choice(np.arange(R.W1, R.B1), 20), rng.choice(np.arange(R.B1, R.W2), 5),
                          rng.choice(np.arange(R.W2, R.B2), 20), rng.choice(np.arange(R.B2, R.W3), 5),
                          rng.choice(np.arange(R.W3, R.W3 + R.OUT * R.HID), 10), np.arange(R.B3, R.B3 + R.OUT)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_and_grad(pp, x, t, False)[0] - R.loss_and_grad(pm, x, t, False)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-3, 65504.0, 0.0])
    got = R.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                 # tie -> even
    assert got[2] == 1.0 + 2 ** -7       # above the tie -> up
    assert got[3] == -2.5
    assert abs(got[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert got[6] == 0.0
    assert np.all(R.bf16(got) == got)    # idempotent


def test_adam_first_step():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = R.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 1e-3, 0.9, 0.999, 1e-8)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    np.testing.assert_allclose(p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_feature_invariants():
    """On the undeformed mesh with candidate = current position, the geometry
    features vanish; with identical images, so do the intensity features."""
    img = W._blur(np.random.default_rng(2).uniform(0, 1, (12, 14, 16)), 1.0).astype(np.float32)
    rp = ref.Problem(img, img, (3, 4, 3))
    I = rp.identity()
    X = np.stack([I, I])[None].astype(np.float32)
    pts = np.arange(rp.P, dtype=np.int32)
    cand = np.stack([X[0, 0, pts], X[0, 1, pts]], axis=1)[None, :, None]  # [1][P][1][2][3]
    f = R.features(rp, X, pts, cand)
    assert np.all(f == 0.0)
    # moving the candidate by d shifts the first 6 features by d and every
    # existing neighbour feature by -d
    d = np.array([0.25, -0.5, 0.125])
    cand2 = cand.copy()
    cand2[0, :, 0, 0] += d
    f2 = R.features(rp, X, pts, cand2)
    np.testing.assert_allclose(f2[:, 0:3], np.broadcast_to(d, (rp.P, 3)))
    offs = R.neighbour_offsets()
    n = rp.mesh
    for p_ in (0, 5, rp.P - 1):
        pi, pj, pk = p_ % n[0], (p_ // n[0]) % n[1], p_ // (n[0] * n[1])
        for j, (dx, dy, dz) in enumerate(offs):
            inside = 0 <= pi + dx < n[0] and 0 <= pj + dy < n[1] and 0 <= pk + dz < n[2]
            np.testing.assert_allclose(f2[p_, 6 + 6 * j:6 + 6 * j + 3], -d if inside else 0.0)


def test_intensity_features_on_ramp_images_closed_form():
    """Features [162, 188): for each of the 26 offsets o (dz, dy, dx order,
    dx fastest) the source image sampled at the source candidate + h o minus
    the target image sampled at the target candidate + h o, with h half the
    undeformed cube extent per axis and positions clamped to [0, D - 1].  On
    linear ramp images trilinear sampling is exact, so each feature is
    g_src . clamp(c_src + h o) + k_src - g_tgt . clamp(c_tgt + h o) - k_tgt."""
    dims, mesh = (20, 16, 12), (4, 3, 3)
    g_src, k_src = np.array([0.02, -0.01, 0.03]), 0.2
    g_tgt, k_tgt = np.array([-0.015, 0.025, 0.01]), 0.6
    src = W.ramp(dims[::-1], tuple(g_src), k_src)
    tgt = W.ramp(dims[::-1], tuple(g_tgt), k_tgt)
    rp = ref.Problem(src, tgt, mesh)
    I = rp.identity()
    X = np.stack([I, I])[None].astype(np.float32)
    rng = np.random.default_rng(5)
    pts = np.arange(rp.P, dtype=np.int32)
    cand = np.stack([X[0, 0, pts], X[0, 1, pts]], axis=1)[None, :, None].astype(np.float64)
    cand = cand + rng.normal(0, 1.0, cand.shape)
    cand = np.asarray(W.snap(np.clip(cand, -0.5, np.array(dims) - 0.5)), np.float64)
    f = R.features(rp, X, pts, cand)
    h = np.array([dims[a] / (2.0 * (mesh[a] - 1)) for a in range(3)])
    hi = np.array(dims, np.float64) - 1.0
    ramp_s = lambda x: g_src @ np.clip(x, 0.0, hi) + k_src
    ramp_t = lambda x: g_tgt @ np.clip(x, 0.0, hi) + k_tgt
    # the offsets spelled out in their slot order
    slots = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]
    assert len(slots) == 26
    clamped = 0
    for q in range(rp.P):
        cs, ct = cand[0, q, 0, 0], cand[0, q, 0, 1]
        for j, o in enumerate(slots):
            ps, pt = cs + h * np.array(o), ct + h * np.array(o)
            clamped += np.any((ps < 0) | (ps > hi))
            want = ramp_s(ps) - ramp_t(pt)
            # the ramp images are float32: allow their rounding only
            assert abs(f[q, 162 + j] - want) <= 2e-6, (q, j, f[q, 162 + j], want)
    assert clamped > 0          # the border points exercise the clamp
    # sign and offset pinned: swapping the images or the direction of o changes values
    swapped = [ramp_t(ct + h * np.array(o)) - ramp_s(cs + h * np.array(o)) for o in slots]
    assert np.max(np.abs(np.array(swapped) - f[rp.P - 1, 162:188])) > 1e-2
