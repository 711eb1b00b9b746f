"""The allocation-free partial evaluation (dsm_eval_partial_noalloc) against
dsm_eval_partial on the same inputs: identical results, bit for bit, on two
calls in a row (the second smaller, so the fixed workspace holds the first
call's contents), with and without cached current terms; a problem created
without partial-evaluation capacity; and the capacity error."""
import sys

import numpy as np
import pytest

from paper_2202_11001_amd import workloads as W
from tests._common import feasible_population, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-noalloc] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _same(a, b, what):
    for x, y, name in zip(a, b, ("part_old", "part_new", "flags", "voxel_count")):
        if x is None and y is None:
            continue
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy(), err_msg=f"{what}: {name}")


def test_noalloc_equals_partial_two_calls():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    S, F = X.shape[0], len(off) - 1
    gp = dsm.Problem.from_workload(w, max_solutions=S)
    Xd, offd, ptsd, cd = _t(X), _t(off), _t(pts), _t(cand)
    cache = torch.empty((S, gp.T, 3), dtype=torch.float64, device=DEV)
    gp.eval_full(Xd, tet_terms=cache)
    # first call: the whole 64^3 batch with cached current terms
    _say(f"first call S={S} F={F}")
    want = gp.eval_partial(Xd, offd, ptsd, cd, tet_terms_in=cache, voxel_count=True)
    got = gp.eval_partial_noalloc(Xd, offd, ptsd, cd, tet_terms_in=cache, voxel_count=True)
    torch.cuda.synchronize()
    _same(got, want, "first call")
    assert (got[2] == 0).sum().item() > 0.5 * S * F
    # second call, smaller: 37 solutions x the first 61 elements, current terms recomputed
    S2, F2 = 37, 61
    off2 = off[:F2 + 1].copy()
    pts2 = pts[:off2[-1]].copy()
    X2 = X[5:5 + S2].copy()
    cand2 = cand[5:5 + S2, :off2[-1]].copy()
    X2d, off2d, pts2d, c2d = _t(X2), _t(off2), _t(pts2), _t(cand2)
    _say(f"second call S={S2} F={F2}")
    want2 = gp.eval_partial(X2d, off2d, pts2d, c2d, voxel_count=True)
    got2 = gp.eval_partial_noalloc(X2d, off2d, pts2d, c2d, voxel_count=True)
    torch.cuda.synchronize()
    _same(got2, want2, "second call")
    # the second call's results match the same pairs of the first call's: flags
    # exactly; sums to FP32 rounding (recomputing the current terms changes how a
    # workgroup's waves split the sweep, hence each wave's compensated FP32 sums)
    np.testing.assert_array_equal(got2[2].cpu().numpy(), got[2].cpu().numpy()[5:5 + S2, :F2])
    ok = got2[2].cpu().numpy() == 0
    np.testing.assert_allclose(got2[1].cpu().numpy()[ok], got[1].cpu().numpy()[5:5 + S2, :F2][ok], rtol=1e-6, atol=0)


def test_noalloc_without_partial_capacity_and_capacity_error():
    """A problem created for one solution and no FOS elements evaluates a
    population through the fixed workspace; a call whose workspace would exceed
    it fails on the host with DSM_ERR_CAPACITY."""
    w = W.tiny()
    rp = oracle_problem(w)
    X = feasible_population(w, rp)
    off, pts = w.fos()
    cand = w.candidates(X, off, pts)
    S = X.shape[0]
    big = dsm.Problem.from_workload(w, max_solutions=S)
    small = dsm.Problem.from_workload(w, max_solutions=1, max_fos=0, max_fos_points=1)
    Xd, offd, ptsd, cd = _t(X), _t(off), _t(pts), _t(cand)
    _say(f"tiny S={S} through a problem without partial capacity")
    want = big.eval_partial(Xd, offd, ptsd, cd, voxel_count=True)
    got = small.eval_partial_noalloc(Xd, offd, ptsd, cd, voxel_count=True)
    torch.cuda.synchronize()
    _same(got, want, "no-capacity problem")
    # workspace of 20,000 solutions x 27 elements without a cache: well above 64 MiB
    n = 20000
    Xb = torch.zeros((n, 2, w.P, 3), dtype=torch.float32, device=DEV)
    cb = torch.zeros((n, len(pts), 2, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(dsm.DsmError) as ei:
        small.eval_partial_noalloc(Xb, offd, ptsd, cb)
    assert ei.value.status == dsm.ERR_CAPACITY
    torch.cuda.synchronize()
