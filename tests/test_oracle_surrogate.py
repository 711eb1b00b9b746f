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
