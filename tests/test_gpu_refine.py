"""GPU grid refinement (Sec. 2.4) against the oracle: bit-exact coordinates,
equal fold flags and objectives on the finer problem."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import workloads as W
from tests._common import assert_objectives_close, feasible_population, oracle_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_11001_amd import dsm  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(f"[gpu-refine] {msg}", file=sys.stderr, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("mesh,dims,sigma", [((3, 3, 3), (32, 32, 32), 1.0), ((4, 3, 5), (37, 23, 41), 2.5),
                                             ((2, 2, 2), (9, 9, 9), 0.7), ((10, 10, 6), (512, 512, 100), 2.0)])
def test_refine_bitexact(mesh, dims, sigma):
    _say(f"refine mesh {mesh}")
    Xc = W.population(dims, mesh, 5, sigma, 3)
    got = dsm.refine_population(mesh, _t(Xc)).cpu().numpy()
    np.testing.assert_array_equal(got, ref.refine(mesh, Xc))


def test_refined_population_on_the_finer_problem():
    w = W.batched()
    rp = oracle_problem(w)
    X = feasible_population(w, rp, S=12)
    nf = tuple(2 * n - 1 for n in w.mesh)
    _say(f"refine {w.mesh} -> {nf} and evaluate")
    Xf = dsm.refine_population(w.mesh, _t(X))
    wf = W.Workload(w.name + "-fine", w.moving, w.fixed, nf, w.spacing, w.tau, 12, w.sigma_pop, w.sigma_cand,
                    w.seed_pop, w.seed_cand, w.guid_moving, w.guid_fixed, w.corr_moving, w.corr_fixed)
    gpf = dsm.Problem.from_workload(wf, max_solutions=12)
    rpf = oracle_problem(wf)
    obj, fl = gpf.eval_full(Xf)
    Xfn = Xf.cpu().numpy()
    robj, rfl = rpf.eval_full(Xfn)
    np.testing.assert_array_equal(fl.cpu().numpy(), rfl)
    assert int((rfl != 0).sum()) == 0
    assert_objectives_close(obj.cpu().numpy(), robj, what="refined objectives")


def test_refine_rejects_bad_meshes():
    X = torch.zeros((1, 2, 8, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(dsm.DsmError):
        dsm.refine_population((1, 2, 2), X)
