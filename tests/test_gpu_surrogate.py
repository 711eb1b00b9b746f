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


def _assert_elementwise(got, want, what, rel=1e-3, floor=5e-4):
    """|got - want| <= rel |want| + floor * max|want| for every element.  The
    floor covers FP32-vs-FP64 accumulation of the same BF16 operands, where a
    rounding-order difference can move an intermediate BF16 rounding by one
    unit; FP32 accumulation emulated on the host needs at most 1.4e-4."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    tol = rel * np.abs(want) + floor * np.abs(want).max()
    bad = np.abs(got - want) > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} of {bad.size} elements off, worst at " \
        f"{np.unravel_index(np.argmax(np.abs(got - want) - tol), want.shape)}"


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
    # element-wise: FP32 accumulation differs from FP64 by rounding order only (same BF16 operands)
    _assert_elementwise(y, yr, "forward")


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
    for name, (a, b) in (("W1", (R.W1, R.B1)), ("b1", (R.B1, R.W2)), ("W2", (R.W2, R.B2)), ("b2", (R.B2, R.W3)),
                         ("W3", (R.W3, R.B3)), ("b3", (R.B3, R.NPARAMS))):
        _assert_elementwise(g[a:b], gr[a:b], f"gradient {name}")


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


def _o12(d, obj_s, arch):
    """Acceptance of a predicted delta d [3] (FP64) of a solution with
    objectives obj_s: it improves one objective and worsens none; or, when an
    archive is given, it improves one objective and obj_s + d is dominated by
    no archive row (rows up to the first +inf padding row)."""
    if np.all(d <= 0) and np.any(d < 0):
        return 1, "pareto"
    if arch is None or obj_s is None:
        return 0, "none"
    if not np.any(d < 0):
        return 0, "worse"
    nv = obj_s + d
    for a in arch:
        if a[0] == np.inf:
            break
        if np.all(a <= nv) and np.any(a < nv):
            return 0, "dominated"
    return 1, "archive"


def test_screen_run_exact_rule():
    """run_exact of every (solution, element) against the acceptance rule
    evaluated in FP64 on the returned raw predictions of the pick: without an
    archive, with an archive that dominates some picks and not others, and with
    an archive of padding rows only; the pick against the FP64 network on the
    same BF16 rows."""
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=6)
    S, P, K = X.shape[0], w.P, 4
    off, pts = w.fos()
    candK = W.candidates(X, off, pts, w.mesh, w.dims, 1.0, 77, K=K)
    candK = np.ascontiguousarray(candK.transpose(0, 2, 1, 3, 4))  # [S][P][K][2][3]
    gp = dsm.Problem.from_workload(w, max_solutions=S)
    sur = dsm.Surrogate(seed=3, max_rows=S * P * K)
    p = _rand_params(11, scale=0.12)
    sur.params(p)
    rng = np.random.default_rng(4)
    out_mean = np.array([0.01, -0.02, 0.0], np.float32)
    out_rstd = np.array([20.0, 10.0, 40.0], np.float32)
    sur.set_scaling(rng.normal(0, 0.1, 192).astype(np.float32), rng.uniform(0.5, 2.0, 192).astype(np.float32),
                    out_mean, out_rstd)
    Xd, ptsd, cd = _t(X), _t(pts), _t(candK)
    _say("screen without archive")
    pick, run, pred, _ = sur.screen(gp, Xd, ptsd, cd)
    pick, run, pred = pick.cpu().numpy(), run.cpu().numpy(), pred.cpu().numpy().astype(np.float64)
    dpick = np.take_along_axis(pred, pick[:, :, None, None], axis=2)[:, :, 0]  # [S][P][3]
    kinds = {}
    for s in range(S):
        for f in range(P):
            want, kind = _o12(dpick[s, f], None, None)
            assert run[s, f] == want, (s, f, dpick[s, f])
            kinds[kind] = kinds.get(kind, 0) + 1
    assert kinds.get("pareto", 0) > 0 and kinds.get("none", 0) > 0
    # the pick against the FP64 network on the same BF16 rows (rows whose
    # choice is not decided by a near-tie)
    rows_d = sur.features_packed(gp, Xd, ptsd, cd)
    rows = rows_d.cpu().numpy().view(np.uint16)
    xr = (rows.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    yref, _ = R.forward(p.astype(np.float64), xr, bf16_round=True)
    yref = yref.reshape(S * P, K, 3)
    ref_pick = _numpy_select(yref, K)
    # a row's pick is decided by the FP64 outputs when every comparison the
    # rule makes (per objective and of the sums) differs by more than twice the
    # row's GPU-vs-FP64 output error
    ygpu = sur.forward(rows_d).cpu().numpy().astype(np.float64).reshape(S * P, K, 3)
    err = np.abs(ygpu - yref).max(axis=(1, 2)) * 3
    gap = np.full(S * P, np.inf)
    for i in range(S * P):
        for j in range(K):
            for k in range(K):
                if j != k:
                    gap[i] = min(gap[i], np.abs(yref[i, j] - yref[i, k]).min(), abs(yref[i, j].sum() - yref[i, k].sum()))
    clear = gap > 2 * err
    assert clear.mean() > 0.5
    assert np.array_equal(pick.reshape(-1)[clear], ref_pick[clear])
    # the raw predictions are the de-standardised network outputs
    np.testing.assert_allclose(pred.reshape(S * P, K, 3), yref / out_rstd + out_mean,
                               rtol=1e-3, atol=5e-4 * np.abs(yref / out_rstd).max())
    # with objectives and an archive: half of the picks that improve some
    # objective but not all get an archive row that dominates their new vector
    obj = rng.uniform(0.5, 1.5, (S, 3))
    mixed = [(s, f) for s in range(S) for f in range(P)
             if np.any(dpick[s, f] < 0) and not np.all(dpick[s, f] <= 0)]
    assert len(mixed) >= 8
    rows_a = [obj[s] + dpick[s, f] - 1e-3 for (s, f) in mixed[::2]]
    rows_a += list(rng.uniform(3.0, 4.0, (5, 3)))  # far away: dominate nothing
    arch = np.concatenate([np.array(rows_a), np.full((4, 3), np.inf)])  # +inf rows end the archive
    for name, A in (("archive", arch), ("padding only", np.full((3, 3), np.inf))):
        _say(f"screen with {name}")
        pick2, run2, pred2, _ = sur.screen(gp, Xd, ptsd, cd, obj=_t(obj), archive=_t(A))
        assert np.array_equal(pick2.cpu().numpy(), pick)
        run2 = run2.cpu().numpy()
        kinds = {}
        for s in range(S):
            for f in range(P):
                want, kind = _o12(dpick[s, f], obj[s], A)
                assert run2[s, f] == want, (name, s, f, kind)
                kinds[kind] = kinds.get(kind, 0) + 1
        assert kinds.get("pareto", 0) > 0 and kinds.get("archive", 0) > 0
        if name == "archive":
            assert kinds.get("dominated", 0) > 0
