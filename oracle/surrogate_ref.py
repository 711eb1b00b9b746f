"""FP64 reference of the candidate-screening MLP and its input features.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).  Shares no
code with the GPU library.

The network is 192 -> 128 -> 128 -> 3 with ReLU; the parameter vector has the
layout W1[128][192] b1[128] W2[128][128] b2[128] W3[16][128] b3[16] (rows 3..15
of W3 and b3 unused).  With ``bf16=True`` every operand of a matrix product is
rounded to bfloat16 (round to nearest even) at the same points as the GPU
kernels: inputs, weights, hidden activations after ReLU, and the back-propagated
output / hidden-layer gradients.  With ``bf16=False`` the arithmetic is plain
FP64 (used to pin the backward pass against finite differences).
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT, OUTPAD = 192, 128, 3, 16
W1, B1 = 0, HID * IN
W2 = B1 + HID
B2 = W2 + HID * HID
W3 = B2 + HID
B3 = W3 + OUTPAD * HID
NPARAMS = B3 + OUTPAD


def bf16(x):
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[W1:B1].reshape(HID, IN), p[B1:W2], p[W2:B2].reshape(HID, HID), p[B2:W3],
            p[W3:B3].reshape(OUTPAD, HID)[:OUT], p[B3:B3 + OUT])


def forward(p, x, bf16_round=True):
    """Outputs [N][3] and the cached activations."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(x)
    w1, w2, w3 = r(w1), r(w2), r(w3)
    h1 = r(np.maximum(x @ w1.T + b1, 0.0))
    h2 = r(np.maximum(h1 @ w2.T + b2, 0.0))
    y = h2 @ w3.T + b3
    return y, (x, h1, h2, w1, w2, w3)


def loss_and_grad(p, x, t, bf16_round=True):
    """Loss (1/N) sum_rows mean_outputs (y - t)^2 and its gradient [NPARAMS]."""
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    y, (xr, h1, h2, w1, w2, w3) = forward(p, x, bf16_round)
    n = len(xr)
    d = y - t
    loss = float((d ** 2).sum() / (3 * n))
    dy = r(2.0 * d / (3 * n))
    g = np.zeros(NPARAMS)
    g[W3:W3 + OUT * HID] = (dy.T @ h2).ravel()
    g[B3:B3 + OUT] = dy.sum(axis=0)
    dz2 = r((dy @ w3) * (h2 > 0))
    g[W2:B2] = (dz2.T @ h1).ravel()
    g[B2:W3] = dz2.sum(axis=0)
    dz1 = r((dz2 @ w2) * (h1 > 0))
    g[W1:B1] = (dz1.T @ xr).ravel()
    g[B1:W2] = dz1.sum(axis=0)
    return loss, g


def adam_step(p, g, m, v, t, lr, b1, b2, eps):
    """One Adam update (t = step number starting at 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def neighbour_offsets():
    """The 26 offsets (dx, dy, dz), dz then dy then dx, dx fastest, centre skipped."""
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx, dy, dz) != (0, 0, 0):
                    out.append((dx, dy, dz))
    return out


def features(rp, X, pts, cand):
    """Feature rows [S*F*K][192] (FP64) for candidates cand [S][F][K][2][3] of
    single-point elements pts [F]; rp is an oracle.ref.Problem (it supplies the
    undeformed grid and FP64 clamped trilinear sampling)."""
    X = np.asarray(X, dtype=np.float64)
    cand = np.asarray(cand, dtype=np.float64)
    S, F, K = cand.shape[:3]
    ident = rp.identity().astype(np.float64)
    n = [int(v) for v in rp.mesh]
    dims = [int(v) for v in rp.dims]
    h = np.array([dims[a] / (2.0 * (n[a] - 1)) for a in range(3)])
    offs = neighbour_offsets()
    out = np.zeros((S, F, K, IN))
    for f, p in enumerate(pts):
        pi, pj, pk = p % n[0], (p // n[0]) % n[1], p // (n[0] * n[1])
        for s in range(S):
            for k in range(K):
                c = cand[s, f, k]  # [2][3]
                row = out[s, f, k]
                row[0:3] = c[0] - X[s, 0, p]
                row[3:6] = c[1] - X[s, 1, p]
                for j, (dx, dy, dz) in enumerate(offs):
                    qi, qj, qk = pi + dx, pj + dy, pk + dz
                    if 0 <= qi < n[0] and 0 <= qj < n[1] and 0 <= qk < n[2]:
                        q = qi + n[0] * (qj + n[1] * qk)
                        for g in range(2):
                            row[6 + 6 * j + 3 * g:6 + 6 * j + 3 * g + 3] = (X[s, g, q] - c[g]) - (ident[q] - ident[p])
                    o = h * np.array([dx, dy, dz], dtype=np.float64)
                    row[162 + j] = rp.trilinear(0, c[0] + o) - rp.trilinear(1, c[1] + o)
    return out.reshape(S * F * K, IN)
