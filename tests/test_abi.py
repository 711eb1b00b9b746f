"""C-ABI contract on the CPU: the library loads, exports every declared
symbol, validates host arguments before touching a device, and its host-side
topology equals the oracle's (Sec. 2.1 split, Sec. 2.2 stars)."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import ref
from paper_2202_11001_amd import dsm
from paper_2202_11001_amd import workloads as W


def test_exports_every_declared_symbol():
    L = dsm.lib()
    names = dsm.header_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_last_error():
    L = dsm.lib()
    for st in range(7):
        assert L.dsm_status_string(st)
    assert L.dsm_status_string(99) == b"unknown status"
    h = C.c_void_p()
    assert L.dsm_problem_create(None, C.byref(h)) == dsm.ERR_ARG
    assert b"desc" in L.dsm_last_error()
    assert L.dsm_problem_create(None, None) == dsm.ERR_ARG
    assert L.dsm_problem_destroy(None) == dsm.ERR_ARG
    assert L.dsm_fold_check(None, 1, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_eval_full(None, 1, None, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_eval_partial(None, 1, None, 1, None, None, None, None, None, None, None, None, None,
                              None) == dsm.ERR_ARG
    assert L.dsm_rasterize_owner(None, None, None, None, None) == dsm.ERR_ARG


def _desc(dims=(8, 8, 8), mesh=(3, 3, 3)):
    img = np.zeros(dims[::-1], np.float32)
    d = dsm.ProblemDesc()
    d.dims[:] = dims
    d.spacing_mm[:] = (1, 1, 1)
    d.moving = d.fixed = img.ctypes.data
    d.mesh[:] = mesh
    d.empty_tau = 0.1
    d.max_solutions, d.max_fos, d.max_fos_points = 4, 4, 1
    return d, img


@pytest.mark.parametrize("field,value,status", [
    ("dims", (513, 8, 8), dsm.ERR_DOMAIN), ("dims", (1, 8, 8), dsm.ERR_DOMAIN),
    ("mesh", (1, 3, 3), dsm.ERR_DOMAIN), ("mesh", (200, 3, 3), dsm.ERR_DOMAIN),
    ("spacing_mm", (0, 1, 1), dsm.ERR_ARG), ("max_solutions", 0, dsm.ERR_ARG),
])
def test_create_validation_before_device(field, value, status):
    d, img = _desc()
    if isinstance(value, tuple):
        getattr(d, field)[:] = value
    else:
        setattr(d, field, value)
    h = C.c_void_p()
    assert dsm.lib().dsm_problem_create(C.byref(d), C.byref(h)) == status
    assert not h.value


def test_guidance_validation():
    d, img = _desc()
    g = np.array([[100.0, 1.0, 1.0]], np.float32)  # outside the image
    c = np.zeros(1, np.int32)
    d.n_guid_moving = d.n_guid_fixed = 1
    d.guid_moving = d.guid_fixed = g.ctypes.data
    d.corr_moving = d.corr_fixed = c.ctypes.data
    h = C.c_void_p()
    assert dsm.lib().dsm_problem_create(C.byref(d), C.byref(h)) == dsm.ERR_DOMAIN
    g2 = np.array([[1.001, 1.0, 1.0]], np.float32)  # off the lattice
    d.guid_moving = d.guid_fixed = g2.ctypes.data
    assert dsm.lib().dsm_problem_create(C.byref(d), C.byref(h)) == dsm.ERR_DOMAIN
    g3 = np.array([[1.0, 1.0, 1.0]], np.float32)
    c2 = np.ones(1, np.int32)  # correspondence 0 on the source, 1 on the target
    d.guid_moving = d.guid_fixed = g3.ctypes.data
    d.corr_fixed = c2.ctypes.data
    assert dsm.lib().dsm_problem_create(C.byref(d), C.byref(h)) == dsm.ERR_ARG


@pytest.mark.parametrize("mesh,dims", [((3, 3, 3), (32, 32, 32)), ((5, 4, 3), (33, 17, 9)),
                                       ((10, 10, 6), (512, 512, 100)), ((2, 2, 2), (2, 2, 2)),
                                       ((6, 6, 6), (64, 64, 64))])
def test_host_topology_equals_oracle(mesh, dims):
    tp = dsm.mesh_topology(mesh, dims)
    z = np.zeros(dims[::-1], np.float32)
    rp = ref.Problem(z, z, mesh)
    assert (tp["P"], tp["T"], tp["E"], tp["max_star"]) == (rp.P, rp.T, rp.E, rp.max_star)
    np.testing.assert_array_equal(tp["tets"], rp.tets())
    off, st = rp.star()
    np.testing.assert_array_equal(tp["star_off"], off)
    np.testing.assert_array_equal(tp["star"], st)
    np.testing.assert_array_equal(tp["identity"], rp.identity())
    np.testing.assert_array_equal(tp["identity"], W.regular_grid(dims, mesh))


def test_distribution_arguments_checked_on_host():
    """A sampler launch never reads a distribution of the wrong dtype or size."""
    import torch
    ok = (torch.zeros((2, 3, 6), dtype=torch.float64), torch.zeros((2, 3, 21), dtype=torch.float64),
          torch.ones((2, 3), dtype=torch.float32))
    dsm._check_dist(*ok, torch.zeros(5, dtype=torch.int32), 5, 6, 6, 21)
    with pytest.raises(ValueError):
        dsm._check_dist(ok[0].float(), ok[1], ok[2], None, 5, 6, 6, 21)
    with pytest.raises(ValueError):
        dsm._check_dist(ok[0], ok[1][:1], ok[2], None, 5, 6, 6, 21)
    with pytest.raises(ValueError):
        dsm._check_dist(*ok, torch.zeros(4, dtype=torch.int32), 5, 6, 6, 21)
    with pytest.raises(ValueError):
        dsm.cluster_objectives(torch.zeros((4, 3), dtype=torch.float32), torch.zeros(2, dtype=torch.int32), 2)


def test_new_entry_points_validate_on_the_host():
    """Argument errors of the transformation, clustering, donor, variance-scaling
    and sampling entry points are reported before any device work."""
    L = dsm.lib()
    assert L.dsm_transform(None, 1, None, None, None, None) == dsm.ERR_ARG
    # clustering: k outside [1, 16], negative sizes, selection above capacity
    assert L.dsm_cluster_objectives(4, None, 2, None, 0, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_cluster_objectives(4, None, 2, None, 17, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_cluster_objectives(-1, None, 2, None, 2, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_cluster_objectives(4, None, 1025, None, 2, None, None, None, None) == dsm.ERR_CAPACITY
    assert L.dsm_cluster_objectives(4, None, 2, None, 2, None, None, None, None) == dsm.ERR_ARG  # null buffers
    assert L.dsm_cluster_objectives(0, None, 0, None, 2, None, None, None, None) == dsm.OK  # nothing to write
    # variance scaling: 6 or 24 variables only, at least one cluster
    assert L.dsm_improvement_ratio(4, 2, None, None, None, 1, None, None, None, 7, None, None) == dsm.ERR_ARG
    assert L.dsm_improvement_ratio(4, 2, None, None, None, 0, None, None, None, 6, None, None) == dsm.ERR_ARG
    assert L.dsm_improvement_ratio(4, 2, None, None, None, 1, None, None, None, 6, None, None) == dsm.ERR_ARG
    assert L.dsm_improvement_ratio(4, 0, None, None, None, 1, None, None, None, 24, None, None) == dsm.OK
    assert L.dsm_copy_from_donor(None, 4, None, 3, None, None, None, None) == dsm.ERR_ARG
    assert L.dsm_sample_elements(None, 4, None, 1, None, None, None, None, None, 1, None, None, None, 2.0, 0, 0,
                                 None, None, None) == dsm.ERR_ARG
    assert L.dsm_sample_estimated(None, 4, None, 1, None, 1, None, None, None, 1, None, None, None, 2.0, 0, 0,
                                  None, None, None) == dsm.ERR_ARG


def test_tuning_settings_validate_on_the_host():
    """The work-split and row-order settings and their autotuners reject a null
    problem (and the getters report it) before any device work."""
    L = dsm.lib()
    assert L.dsm_set_part_chunk(None, 4) == dsm.ERR_ARG
    assert L.dsm_get_part_chunk(None) == 0
    assert L.dsm_set_row_order(None, 0) == dsm.ERR_ARG
    assert L.dsm_get_row_order(None) == -1
    assert L.dsm_autotune_chunk(None, 1, None, 1, None, None, None, None, 0, None, None, None) == dsm.ERR_ARG
    assert L.dsm_autotune_row_order(None, 1, None, 1, None, None, None, None, None, None) == dsm.ERR_ARG
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "dsm.h")).read()
    defs = dict(re.findall(r"#define (DSM_ROWS_\w+) (\d+)", hdr))
    assert int(defs["DSM_ROWS_BY_SLICE"]) == dsm.Problem.ROWS_BY_SLICE == 0
    assert int(defs["DSM_ROWS_BY_SLICE_PAIR"]) == dsm.Problem.ROWS_BY_SLICE_PAIR == 1
