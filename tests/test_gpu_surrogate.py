"""GPU parity of the candidate-screening MLP (BF16 matrix cores, FP32
accumulation) against the FP64 reference on the same BF16-rounded operands,
features against the reference features, a full Adam step, the screening
rule, and an ablation showing what the trained network gains."""
import sys

import numpy as np
import pytest

from oracle import ref
from oracle import surrogate_ref as R
from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-surrogate] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _bf16_bits(x):
    """bfloat16 bit patterns (int16) of float values (nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)).view(np.int16)


def _rand_params(seed, scale=0.15):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, R.NPARAMS).astype(np.float32)
    p[R.W3 + R.OUT * R.HID:R.B3] = 0.0
    p[R.B3 + R.OUT:] = 0.0
    return p


@pytest.mark.parametrize("N", [1, 16, 37, 300])
def test_forward_matches_reference(N):
    _say(f"forward N={N}")
    rng = np.random.default_rng(N)
    p = _rand_params(3)
    x = rng.normal(size=(N, R.IN)).astype(np.float32)
    sur = dsm.Surrogate(seed=1, max_rows=1024, max_batch=512)
    sur.params(p)
    y = sur.forward(_t(_bf16_bits(x))).cpu().numpy()
    yr, _ = R.forward(p.astype(np.float64), x, bf16_round=True)
    scale = np.abs(yr).max() + 1e-6
    assert np.abs(y - yr).max() <= 2e-3 * scale


@pytest.mark.parametrize("N", [32, 70, 512])
def test_gradient_matches_reference(N):
    _say(f"gradient N={N}")
    rng = np.random.default_rng(10 + N)
    p = _rand_params(4)
    x = rng.normal(size=(N, R.IN)).astype(np.float32)
    t = rng.normal(size=(N, R.OUT)).astype(np.float32)
    sur = dsm.Surrogate(seed=1, max_rows=1024, max_batch=512)
    sur.params(p)
    g, loss = sur.gradient(_t(_bf16_bits(x)), _t(t))
    g = g.cpu().numpy().astype(np.float64)
    lr_, gr = R.loss_and_grad(p.astype(np.float64), R.bf16(x), t.astype(np.float64), bf16_round=True)
    assert float(loss.item()) == pytest.approx(lr_, rel=1e-3)
    for a, b in ((R.W1, R.B1), (R.B1, R.W2), (R.W2, R.B2), (R.B2, R.W3), (R.W3, R.B3), (R.B3, R.NPARAMS)):
        blk, ref_blk = g[a:b], gr[a:b]
        assert np.linalg.norm(blk - ref_blk) <= 1e-3 * np.linalg.norm(ref_blk) + 1e-9, (a, b)


def _splitmix_indices(seed, step, N, B):
    """The counter-based minibatch indices (splitmix64 finaliser of
    seed + golden * (step * 2^32 + step + slot + 1))."""
    out = []
    M = (1 << 64) - 1
    for b in range(B):
        z = (seed + 0x9E3779B97F4A7C15 * ((step * 0x100000001 + b + 1) & M)) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z ^= z >> 31
        out.append(z % N)
    return np.array(out)


def test_adam_step_matches_reference():
    _say("adam step")
    rng = np.random.default_rng(5)
    N, B = 200, 64
    p = _rand_params(6)
    x = rng.normal(size=(N, R.IN)).astype(np.float32)
    t = rng.normal(size=(N, R.OUT)).astype(np.float32)
    sur = dsm.Surrogate(seed=12345, lr=1e-3, max_rows=1024, max_batch=512)
    sur.params(p)
    loss = sur.train(_t(_bf16_bits(x)), _t(t), steps=1, batch=B)
    p_new = sur.params()
    idx = _splitmix_indices(12345, 0, N, B)
    lr_, g = R.loss_and_grad(p.astype(np.float64), R.bf16(x[idx]), t[idx].astype(np.float64), True)
    pr, _, _ = R.adam_step(p.astype(np.float64), g, np.zeros(R.NPARAMS), np.zeros(R.NPARAMS), 1, 1e-3, 0.9, 0.999, 1e-8)
    assert float(loss[0].item()) == pytest.approx(lr_, rel=1e-3)
    # the first Adam step moves each parameter by ~lr * sign(g): compare where |g| is not tiny
    big = np.abs(g) > 1e-4 * np.abs(g).max()
    np.testing.assert_allclose(p_new[big], pr[big], atol=2e-5)


def test_features_match_reference():
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=3)
    pts = np.arange(w.P, dtype=np.int32)
    K = 2
    cand = W.candidates(X, np.arange(w.P + 1, dtype=np.int32), pts, w.mesh, w.dims, 1.0, 99, K=K)  # [S][K][P][2][3]
    cand = np.ascontiguousarray(cand.transpose(0, 2, 1, 3, 4))  # [S][P][K][2][3]
    _say("features tiny")
    gp = dsm.Problem.from_workload(w, max_solutions=3)
    f = dsm.Surrogate.features(gp, _t(X), _t(pts), _t(cand)).cpu().numpy()
    fr = R.features(rp, X, pts, cand)
    assert f.shape == fr.shape
    np.testing.assert_allclose(f[:, :162], fr[:, :162], atol=1e-4)
    np.testing.assert_allclose(f[:, 162:188], fr[:, 162:188], atol=1e-4)
    assert np.all(f[:, 188:] == 0)


@pytest.mark.parametrize("K", [1, 3])
def test_fused_features_equal_pack_of_features(K):
    """The screening path's one-kernel features + standardisation + BF16
    rounding equals the two-step path bit for bit, and both equal numpy's
    rounding of the standardised FP32 rows; an out-of-range point (-1) gives
    the standardised zero row."""
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=3)
    pts = np.concatenate([[-1], np.arange(w.P)]).astype(np.int32)  # 28 elements: rows not a multiple of 8
    cand = W.candidates(X, np.arange(w.P + 1, dtype=np.int32), np.arange(w.P, dtype=np.int32), w.mesh, w.dims, 1.0,
                        17, K=K)  # [S][K][P][2][3], or [S][P][2][3] for K = 1
    cand = cand[:, :, None] if K == 1 else cand.transpose(0, 2, 1, 3, 4)  # [S][P][K][2][3]
    cand = np.concatenate([cand[:, :1], cand], axis=1)
    _say(f"fused features tiny K={K}")
    gp = dsm.Problem.from_workload(w, max_solutions=3)
    rng = np.random.default_rng(K)
    sur = dsm.Surrogate(seed=1, max_rows=3 * len(pts) * K)
    mean = rng.normal(0, 0.3, 192).astype(np.float32)
    rstd = rng.uniform(0.5, 4.0, 192).astype(np.float32)
    sur.set_scaling(mean, rstd, np.zeros(3, np.float32), np.ones(3, np.float32))
    Xd, ptsd, cd = _t(X), _t(pts), _t(cand)
    f = dsm.Surrogate.features(gp, Xd, ptsd, cd)
    two = sur.pack(f)[0].cpu().numpy()
    one = sur.features_packed(gp, Xd, ptsd, cd).cpu().numpy()
    assert one.shape == (3 * len(pts) * K, 192)
    np.testing.assert_array_equal(one, two)
    fn = f.cpu().numpy()
    np.testing.assert_array_equal(one, _bf16_bits((fn - mean) * rstd))
    zero_rows = fn.reshape(3, len(pts), K, 192)[:, 0]
    assert np.all(zero_rows == 0)


def _numpy_select(ps, K):
    """The screening rule on the GPU's own standardised predictions [M][K][3] (float32)."""
    picks = []
    for row in ps:
        best, best_rank, best_sum = 0, 1 << 30, np.float32(np.inf)
        for k in range(K):
            rank = sum(1 for j in range(K) if j != k and np.all(row[j] <= row[k]) and np.any(row[j] < row[k]))
            s = np.float32(np.float32(row[k, 0] + row[k, 1]) + row[k, 2])
            if rank < best_rank or (rank == best_rank and s < best_sum):
                best, best_rank, best_sum = k, rank, s
        picks.append(best)
    return np.array(picks)


def _collect(gp, w, X, Xd, cache, rounds, seed0):
    """(raw features, part_old, part_new) of `rounds` random single-point candidates per (s, f)."""
    off, pts = w.fos()
    offd, ptsd = _t(off), _t(pts)
    feats, olds, news = [], [], []
    for r in range(rounds):
        cand = w.candidates(X, off, pts, seed=seed0 + r)  # [S][P][2][3]
        cd = _t(cand)
        old, new, fl, _ = gp.eval_partial(Xd, offd, ptsd, cd, tet_terms_in=cache)
        f = dsm.Surrogate.features(gp, Xd, ptsd, cd.reshape(X.shape[0], len(pts), 1, 2, 3).contiguous())
        ok = (fl == 0).reshape(-1)
        feats.append(f[ok])
        olds.append(old.reshape(-1, 3)[ok])
        news.append(new.reshape(-1, 3)[ok])
    return torch.cat(feats), torch.cat(olds).contiguous(), torch.cat(news).contiguous()


def test_training_and_screening_gain():
    """Trained on exact deltas of random single-point moves (64^3 workload),
    the network's pick among 4 fresh candidates has a better exact outcome
    than a random pick or an untrained network's pick."""
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    S, P = X.shape[0], w.P
    gp = dsm.Problem.from_workload(w)
    Xd = _t(X)
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=DEV)
    gp.eval_full(Xd, tet_terms=cache)
    _say("collect training deltas")
    feats, old, new = _collect(gp, w, X, Xd, cache, rounds=8, seed0=1000)
    raw = (new - old).to(torch.float32).contiguous()
    K = 4
    sur = dsm.Surrogate(seed=7, lr=1e-3, max_rows=S * P * K, max_batch=1024)
    sur.fit_scaling(feats, raw)
    fb, tg, _ = sur.pack(feats, old, new)
    _say(f"train on {feats.shape[0]} rows")
    losses = sur.train(fb, tg, steps=600, batch=1024).cpu().numpy()
    assert losses[-50:].mean() < 0.5 * losses[:10].mean()
    # held-out: K candidates per (s, f), every one evaluated exactly
    off, pts = w.fos()
    candK = W.candidates(X, off, pts, w.mesh, w.dims, 1.0, 5000, K=K)  # [S][K][P][2][3]
    candK = np.ascontiguousarray(candK.transpose(0, 2, 1, 3, 4))      # [S][P][K][2][3]
    true = np.zeros((S, P, K, 3))
    ok = np.ones((S, P), dtype=bool)
    for k in range(K):
        o, n, fl, _ = gp.eval_partial(Xd, _t(off), _t(pts), _t(candK[:, :, k].copy()), tet_terms_in=cache)
        true[:, :, k] = (n - o).cpu().numpy()
        ok &= fl.cpu().numpy() == 0
    _, _, om, orr = sur.scaling()
    score = ((true - om) * orr).sum(axis=-1)  # standardised sum of exact deltas, lower is better
    ptsd = _t(pts)
    pick, run, pred, cpick = sur.screen(gp, Xd, ptsd, _t(candK))
    pick = pick.cpu().numpy()
    fresh = dsm.Surrogate(seed=8, max_rows=S * P * K, max_batch=1024)
    fresh.fit_scaling(feats, raw)
    pick0 = fresh.screen(gp, Xd, ptsd, _t(candK))[0].cpu().numpy()
    sel = lambda pk: np.take_along_axis(score, pk[..., None], axis=2)[..., 0][ok].mean()
    trained, untrained, rand = sel(pick), sel(pick0), score[..., 0][ok].mean()
    best_rate = (pick == score.argmin(axis=2))[ok].mean()
    _say(f"mean standardised exact delta of the pick: trained {trained:.3f} untrained {untrained:.3f} "
         f"random {rand:.3f}; trained pick is the exact best in {best_rate:.2%}")
    assert trained < rand - 0.2 and trained < untrained - 0.2
    assert best_rate > 0.4
    # the screening rule reproduced on the network's own standardised outputs
    fK = dsm.Surrogate.features(gp, Xd, ptsd, _t(candK))
    pstd = sur.forward(sur.pack(fK)[0]).cpu().numpy()
    assert np.array_equal(pick.reshape(-1), _numpy_select(pstd.reshape(-1, K, 3), K))
    # picked candidates are gathered correctly
    cp = cpick.cpu().numpy()
    assert np.array_equal(cp, np.take_along_axis(candK, pick[:, :, None, None, None], axis=2)[:, :, 0])


def test_set_scaling_roundtrip():
    rng = np.random.default_rng(3)
    sc = [rng.normal(size=192).astype(np.float32), rng.uniform(0.5, 2, 192).astype(np.float32),
          rng.normal(size=3).astype(np.float32), rng.uniform(0.5, 2, 3).astype(np.float32)]
    sur = dsm.Surrogate(seed=1)
    sur.set_scaling(*sc)
    for a, b in zip(sur.scaling(), sc):
        np.testing.assert_array_equal(a, b)
