"""A minimal multi-objective population optimiser on top of the GPU evaluator,
used to measure what learned candidate screening gains.

Each generation visits the 8 index-parity classes of grid points (points of one
class share no tetrahedron, so their partial changes are independent,
Sec. 2.2).  Per class every solution proposes one candidate per point (plain)
or K candidates of which the surrogate picks one and decides whether to
evaluate it exactly (screened); exact partial evaluation, acceptance (feasible
and improving: Pareto improvement or not dominated by the elitist archive) and
the update of coordinates, term cache and objectives all run in the library's
kernels.  The elitist archive (non-dominated objective vectors) is merged on
the device after every generation (on the host when its solutions are kept
too); the hypervolume is computed on the host.

Candidates are isotropic Gaussian moves around the current position
(``sampler="isotropic"``), or (``sampler="estimated"``) samples of a normal
distribution per point estimated on the selected solutions, as RV-GOMEA's
partial changes draw them: each generation selects the ``tau`` fraction of the
population with the fewest dominating solutions (ties: smallest sum of range-
normalised objectives), estimates per FOS element the mean and full covariance
of its coordinates on the GPU (6 per point; the 4 points of a tetrahedron
element jointly), and samples N(mean, c L L^T) with a multiplier c per point
(per cube for tetrahedron elements) that grows by 1/0.9 after a generation in
which the element's change was accepted by some solution and shrinks by 0.9
otherwise (within [0.05, 10]).
Clustering, anticipated mean shift and the full multiplier schedule of
RV-GOMEA are not built.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import dsm


def parity_classes(mesh):
    """Point indices of the 8 index-parity classes, as int32 arrays."""
    nx, ny, nz = (int(n) for n in mesh)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cls = ((i & 1) + 2 * (j & 1) + 4 * (k & 1)).ravel()
    return [np.nonzero(cls == c)[0].astype(np.int32) for c in range(8)]


def cube_classes(mesh):
    """Cube indices of the 27 classes of equal (i, j, k) mod 3.  The stars of
    the corners of two cubes of one class share no tetrahedron, so changes to
    one tetrahedron per cube of a class are independent."""
    nx, ny, nz = (int(n) - 1 for n in mesh)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cls = ((i % 3) + 3 * (j % 3) + 9 * (k % 3)).ravel()
    return [c for c in (np.nonzero(cls == q)[0].astype(np.int64) for q in range(27)) if len(c)]


def nondominated(points):
    """Rows of `points` (minimisation) not dominated by another row; duplicates kept once."""
    pts = np.unique(np.asarray(points, dtype=np.float64), axis=0)
    if len(pts) == 0:
        return pts
    keep = np.ones(len(pts), dtype=bool)
    for b in range(0, len(pts), 1024):  # rows b.. against all rows, in blocks
        blk = pts[b:b + 1024]
        le = np.all(pts[None, :, :] <= blk[:, None, :], axis=2)
        lt = np.any(pts[None, :, :] < blk[:, None, :], axis=2)
        keep[b:b + 1024] = ~np.any(le & lt, axis=1)
    return pts[keep]


def merge_archive(archive, new):
    """Non-dominated rows of archive (itself non-dominated) and new points."""
    new = nondominated(new)
    if len(archive) == 0:
        return new
    arch = np.asarray(archive, dtype=np.float64)
    # archive rows dominated by a new point, new points dominated by (or equal to) an archive row
    le = np.all(new[None, :, :] <= arch[:, None, :], axis=2)
    lt = np.any(new[None, :, :] < arch[:, None, :], axis=2)
    arch_keep = ~np.any(le & lt, axis=1)
    le2 = np.all(arch[None, :, :] <= new[:, None, :], axis=2)
    new_keep = ~np.any(le2, axis=1)
    out = np.concatenate([arch[arch_keep], new[new_keep]])
    return out[np.lexsort(out.T[::-1])]


# The full RV-GOMEA configuration (estimated distributions per cluster of the
# selection, anticipated mean shift, forced improvements, standard-deviation-
# ratio multipliers), the best measured one on both FOS; pass as
# Optimiser(problem, X, fos=..., **RV_GOMEA) or run(..., **RV_GOMEA).
RV_GOMEA = dict(sampler="estimated", clusters=5, ams=True, forced_improvements=True, multiplier_schedule="sdr")


def hypervolume(points, ref):
    """Exact 3-D hypervolume dominated by `points` and bounded by `ref`
    (minimisation): slices along the third objective, each a 2-D union area."""
    ref = np.asarray(ref, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64)
    pts = pts[np.all(pts < ref, axis=1)]
    if len(pts) == 0:
        return 0.0
    pts = pts[np.argsort(pts[:, 2], kind="stable")]
    zs = np.append(pts[:, 2], ref[2])
    vol = 0.0
    for s in range(len(pts)):
        dz = zs[s + 1] - zs[s]
        if dz <= 0:
            continue
        sl = pts[:s + 1, :2]
        sl = sl[np.argsort(sl[:, 0], kind="stable")]
        widths = np.diff(np.append(sl[:, 0], ref[0]))
        area = float(np.sum(widths * (ref[1] - np.minimum.accumulate(sl[:, 1]))))
        vol += area * dz
    return vol


@dataclass
class RunLog:
    hypervolume: list = field(default_factory=list)
    seconds: list = field(default_factory=list)        # optimisation time (monitoring excluded) after each generation
    exact_evals: list = field(default_factory=list)    # exact partial evaluations per generation
    accepted: list = field(default_factory=list)
    archive_size: list = field(default_factory=list)


class Optimiser:
    """Population optimiser state on the GPU for one problem.

    With ``graph=True`` each generation's 8 class steps (sample, screen,
    evaluate, accept) are captured once in a HIP graph and replayed: the sampler
    reads its counter from device memory and the elitist archive is a
    fixed-capacity device buffer padded with +inf rows, so a replay needs no
    host work.  Eager and graph generations give bit-identical results."""

    def __init__(self, problem, X, sigma=1.0, seed=1, K=4, graph=False, archive_capacity=1 << 14,
                 keep_solutions=False, sampler="isotropic", tau=0.35, fos="point", clusters=1, ams=False,
                 forced_improvements=False, nis_max=None, single_objective_clusters=False,
                 multiplier_schedule="simple"):
        import torch
        self.torch = torch
        self.p = problem
        self.X = X.clone()
        self.S = X.shape[0]
        self.sigma = float(sigma)
        self.seed = int(seed)
        self.K = int(K)
        dev = X.device
        if fos not in ("point", "tetrahedron"):
            raise ValueError(f"unknown FOS {fos!r}")
        self.fos = fos
        if fos == "point":
            self.classes = [torch.from_numpy(c).to(dev) for c in parity_classes(problem.mesh)]
            self.offs = [torch.arange(len(c) + 1, dtype=torch.int32, device=dev) for c in self.classes]
        else:
            # the paper's FOS (Sec. 2.2): per cube one of its 6 tetrahedra, drawn
            # anew every generation; classes of cubes 3 apart run in parallel
            if graph:
                raise ValueError("the tetrahedron FOS runs eagerly (its elements are drawn every generation)")
            self.cube_classes = cube_classes(problem.mesh)
            self.tets = np.asarray(problem.topology()["tets"], dtype=np.int32)
            # per class: its cubes and the element offsets (4 points each), on the device once
            self.cubes_dev = [torch.from_numpy(c).to(dev) for c in self.cube_classes]
            self.tet_offs = [torch.from_numpy((4 * np.arange(len(c) + 1)).astype(np.int32)).to(dev)
                             for c in self.cube_classes]
            self.generation_index = 0
            self.classes = None  # drawn per generation
            n_cubes = int(np.prod([int(n) - 1 for n in problem.mesh]))
            self.n_cubes = n_cubes
        self.cache = torch.empty((self.S, problem.T, 3), dtype=torch.float64, device=dev)
        self.terms_cand = torch.zeros_like(self.cache)
        obj, flags = problem.eval_full(self.X, tet_terms=self.cache)
        if int((flags != 0).sum().item()):
            raise ValueError("initial population is infeasible")
        self.obj = obj
        self.keep_solutions = bool(keep_solutions)
        self.capacity = int(archive_capacity)
        # elitist archive on the device (dsm_archive_merge): vectors in
        # lexicographic order padded with +inf rows (arch_dev, read by the
        # acceptance kernels), the count on the device, with keep_solutions
        # each row's solution as its payload; host copies are made on demand
        row_floats = int(np.prod(X.shape[1:])) if self.keep_solutions else 0
        self.A = dsm.Archive(self.capacity, m_max=self.S, row_floats=row_floats, device=dev)
        self.arch_dev = self.A.vec
        self._archive = None
        self._merge()
        self.ref = 1.1 * obj.cpu().numpy().max(axis=0)
        self.collect = None  # optional list receiving (features, part_old, part_new) of exact evaluations
        # sampler counter: generation g uses counters 8 g + 1 ... 8 g + 8
        self.counter_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.n_classes = 8 if fos == "point" else len(self.cube_classes)
        self.use_graph = bool(graph)
        self._graph = None
        self._graph_sur = None
        self._outs = None
        if sampler not in ("isotropic", "estimated"):
            raise ValueError(f"unknown sampler {sampler!r}")
        self.sampler = sampler
        self.k = int(clusters)
        if not 1 <= self.k <= 16 or (self.k > 1 and sampler != "estimated"):
            raise ValueError("clusters: 1 to 16, more than 1 only with the estimated sampler")
        self._assign = None  # cluster of every solution (device int32) when k > 1
        # MO-RV-GOMEA's single-objective clusters: a cluster whose mean is best in
        # objective o optimises o alone (per-solution objective in self._so, else -1)
        self.use_so = bool(single_objective_clusters)
        if self.use_so and self.k < 2:
            raise ValueError("single-objective clusters need at least 2 clusters")
        self._so = None
        # anticipated mean shift (RV-GOMEA): per generation half of the solutions
        # draw around mean + 2 c (mu_t - mu_{t-1}), mu the selection's point means
        self.use_ams = bool(ams)
        if self.use_ams and sampler != "estimated":
            raise ValueError("the anticipated mean shift needs the estimated sampler")
        # forced improvements (RV-GOMEA): a solution without an accepted change for
        # more than nis_max generations copies element values from a donor
        self.use_fi = bool(forced_improvements)
        if self.use_fi and graph:
            raise ValueError("forced improvements run eagerly (the donors' uniform draws come from the host)")
        self.nis_max = int(1 + np.floor(np.log10(self.S))) if nis_max is None else int(nis_max)
        self.nis = torch.zeros(self.S, dtype=torch.int32, device=dev)
        self._donor = None
        self._n_forced = torch.zeros(1, dtype=torch.int32, device=dev)    # solutions given a donor
        self._n_replaced = torch.zeros(1, dtype=torch.int32, device=dev)  # of which replaced by their donor
        self._fi_work = None
        self._gen = 0
        self._point_mean = None  # previous generation's point means (device float64 [P][6])
        self._shift_buf = None
        self._shift = None
        self._ams = None
        if sampler == "estimated":
            if self.use_graph:
                raise ValueError("the estimated sampler runs eagerly (its selection needs the current objectives)")
            self.tau = float(tau)
            # distribution multipliers per cluster and element (per cube for the tetrahedron FOS),
            # with the no-improvement stretches of the standard-deviation-ratio schedule
            if multiplier_schedule not in ("simple", "sdr"):
                raise ValueError(f"unknown multiplier schedule {multiplier_schedule!r}")
            self.schedule = multiplier_schedule
            if fos == "point":
                self.mult = [torch.ones((self.k, len(c)), dtype=torch.float32, device=dev) for c in self.classes]
                self.avs_nis = [torch.zeros((self.k, len(c)), dtype=torch.int32, device=dev) for c in self.classes]
            else:
                self.mult_cube = torch.ones((self.k, self.n_cubes), dtype=torch.float32, device=dev)
                self.avs_nis_cube = torch.zeros((self.k, self.n_cubes), dtype=torch.int32, device=dev)
            self._dist = None

    @property
    def counter(self):
        return int(self.counter_dev.item())

    def _merge(self):
        """Merges the population's objective vectors (and solutions) into the archive."""
        self.A.merge(self.obj, rows=self.X.reshape(self.S, -1) if self.keep_solutions else None)

    @property
    def n_arch(self):
        """Rows of the elitist archive (reads the device count)."""
        if int(self.A.overflow.item()):
            raise ValueError(f"the archive would exceed its capacity of {self.capacity} rows")
        return self.A.n

    @property
    def arch_X_dev(self):
        """With keep_solutions: the solutions of the archive rows (device, [capacity][2][P][3]), else None."""
        return None if self.A.rows is None else self.A.rows.view((self.capacity,) + tuple(self.X.shape[1:]))

    @property
    def archive(self):
        """The elitist archive's objective vectors (host, lexicographic order)."""
        if self._archive is None:
            self._archive = self.arch_dev[:self.n_arch].cpu().numpy()
        return self._archive

    @property
    def archive_X(self):
        """With keep_solutions: the solution of every archive row (host copy), else None."""
        return None if self.arch_X_dev is None else self.arch_X_dev[:self.n_arch].cpu().numpy()

    def _tet_steps(self, surrogate):
        """One generation of the paper's FOS: per class of cubes, one random
        tetrahedron per cube, its 4 points sampled together (isotropic, or from
        the element's jointly estimated distribution with a per-cube
        multiplier), evaluated and accepted."""
        torch = self.torch
        if surrogate is not None or self.collect is not None:
            raise ValueError("screening and training-row collection support single-point elements only")
        dev = self.X.device
        rng = np.random.default_rng([self.seed, self.generation_index])
        self.generation_index += 1
        members = self._cluster() if self.sampler == "estimated" else None
        # this generation's tetrahedron of every cube, uploaded in one copy
        drawn = [self.tets[6 * cubes + rng.integers(0, 6, size=len(cubes))].reshape(-1) for cubes in self.cube_classes]
        start = np.concatenate([[0], np.cumsum([len(d) for d in drawn])])
        pts_all = torch.from_numpy(np.concatenate(drawn).astype(np.int32)).to(dev)
        outs = []
        for c, cubes in enumerate(self.cube_classes):
            pts = pts_all[start[c]:start[c + 1]]
            off = self.tet_offs[c]
            cubes_d = self.cubes_dev[c]
            if self.sampler == "isotropic":
                cand = self.p.sample_candidates(self.X, pts, 1, self.sigma, self.seed, c + 1, counter_dev=self.counter_dev)
                self._force(pts, cand)
            else:
                est = [self.p.estimate_elements(self.X, m, off, pts) for m in members]
                mean = torch.stack([e[0] for e in est]).contiguous()
                chol = torch.stack([e[1] for e in est]).contiguous()
                mult = self.mult_cube[:, cubes_d].contiguous()
                cand = self.p.sample_elements(self.X, off, pts, mean, chol, mult, self.seed, c + 1,
                                              counter_dev=self.counter_dev, cluster=self._assign, shift=self._shift,
                                              ams=self._ams)
                self._force(pts, cand)
            old, new, flags, _ = self.p.eval_partial(self.X, off, pts, cand, tet_terms_in=self.cache,
                                                     tet_terms_new=self.terms_cand)
            acc = torch.empty((self.S, len(cubes)), dtype=torch.uint8, device=dev)
            self.p.accept_elements(self.X, off, pts, cand, old, new, flags, self.terms_cand, self.cache, self.obj,
                                   archive=self.arch_dev, accepted=acc, single_objective=self._so)
            if self.sampler == "estimated" and self.schedule == "sdr":
                sdr = dsm.improvement_ratio(off, cand, acc, mean, chol, cluster=self._assign)
                m, nis = self.mult_cube[:, cubes_d].contiguous(), self.avs_nis_cube[:, cubes_d].contiguous()
                dsm.avs_update(m, nis, sdr.contiguous(), 25 + 24)
                self.mult_cube[:, cubes_d] = m
                self.avs_nis_cube[:, cubes_d] = nis
            elif self.sampler == "estimated":
                m = self.mult_cube[:, cubes_d].contiguous()
                dsm.multiplier_step(acc, m, cluster=self._assign)
                self.mult_cube[:, cubes_d] = m
            outs.append((None, acc, cand, old, new, flags))
        self.counter_dev += self.n_classes
        return outs

    def _steps(self, surrogate):
        """The 8 class steps of one generation, enqueued on the current stream
        without host synchronisation; returns per class (mask or None, accepted)."""
        torch = self.torch
        if self.fos == "tetrahedron":
            return self._tet_steps(surrogate)
        outs = []
        for c, (pts, off) in enumerate(zip(self.classes, self.offs)):
            F = pts.shape[0]
            if surrogate is None:
                cand = self._sample(c, pts, 1)
                self._force(pts, cand)
                mask = None
            else:
                if self.use_fi:
                    raise ValueError("forced improvements do not combine with surrogate screening")
                candK = self._sample(c, pts, self.K)
                _, mask, _, cand = surrogate.screen(self.p, self.X, pts, candK, obj=self.obj, archive=self.arch_dev)
            old, new, flags, _ = self.p.eval_partial(self.X, off, pts, cand, tet_terms_in=self.cache,
                                                     tet_terms_new=self.terms_cand, mask=mask)
            if self.collect is not None:
                feats = dsm.Surrogate.features(self.p, self.X, pts, cand.reshape(self.S, F, 1, 2, 3))
                ok = (flags == 0).reshape(-1)
                self.collect.append((feats[ok], old.reshape(-1, 3)[ok], new.reshape(-1, 3)[ok]))
            acc = torch.empty((self.S, F), dtype=torch.uint8, device=self.X.device)
            self.p.accept(self.X, pts, cand, old, new, flags, self.terms_cand, self.cache, self.obj,
                          archive=self.arch_dev, accepted=acc, single_objective=self._so)
            outs.append((mask, acc, cand, old, new, flags))
        self.counter_dev += 8
        return outs

    def _sample(self, c, pts, K):
        if self.sampler == "isotropic":
            return self.p.sample_candidates(self.X, pts, K, self.sigma, self.seed, c + 1, counter_dev=self.counter_dev)
        mean, chol = self._dist[c]
        return self.p.sample_estimated(self.X, pts, K, mean, chol, self.mult[c], self.seed, c + 1,
                                       counter_dev=self.counter_dev, cluster=self._assign, shift=self._shift,
                                       ams=self._ams)

    def _cluster(self):
        """Selection, and with k > 1 clusters its balanced k-leader-means
        clustering in objective space (MO-RV-GOMEA): the member lists whose
        distributions are estimated, one per cluster; every solution samples
        from its nearest cluster (self._assign)."""
        sel = self.select()
        if self.use_ams:
            all_pts = self.torch.arange(self.p.P, dtype=self.torch.int32, device=self.X.device)
            mean = self.p.estimate_distributions(self.X, sel, all_pts)[0]
            has_prev = self._point_mean is not None
            if not has_prev:
                self._point_mean = self.torch.empty_like(mean)
                self._shift_buf = self.torch.empty_like(mean)
            dsm.ams_shift(mean, self._point_mean, self._shift_buf, has_prev=has_prev)
            self._shift = self._shift_buf if has_prev else None
            half = np.random.default_rng([self.seed, self._gen, 7]).permutation(self.S) < self.S // 2
            self._ams = self.torch.from_numpy(half.astype(np.uint8)).to(self.X.device)
        if self.k == 1:
            return [sel]
        members, self._assign, means = dsm.cluster_objectives(self.obj, sel, self.k)
        if self.use_so:
            # objective o takes the cluster with the lowest mean in o among those
            # not yet taken (in objective order), so each gets its own while k >= 3
            self._so = dsm.single_objective_clusters(means, self._assign)
        return [members[j] for j in range(self.k)]

    def _dominated_by(self):
        """Number of population members dominating each solution (device int32, dsm_select)."""
        cnt = self.torch.empty(self.S, dtype=self.torch.int32, device=self.X.device)
        dsm.select(self.obj, 0, dominated_by=cnt)
        return cnt

    def _force(self, pts, cand):
        """Forced improvements: the flagged solutions' candidates become their
        donors' current values at pts."""
        if self._donor is not None:
            self.p.copy_from_donor(self.X, pts, self._donor, cand)

    def _draw_donors(self):
        """Solutions whose no-improvement stretch exceeds nis_max get a donor: a
        random member of the population that no member dominates
        (dsm_draw_donors, with uniform draws from the optimiser's generator)."""
        torch = self.torch
        u = np.random.default_rng([self.seed, self._gen, 11]).random(self.S, dtype=np.float32)
        self._donor = dsm.draw_donors(self.nis, self.nis_max, self._dominated_by(),
                                      torch.from_numpy(u).to(self.X.device), n_forced=self._n_forced)

    @property
    def fi_forced(self):
        """Solutions given a donor, summed over generations."""
        return int(self._n_forced.item())

    def _after_forcing(self, outs):
        """Updates the no-improvement stretches; a forced solution that accepted
        no change is replaced by its donor (coordinates, objectives, term cache)
        (dsm_mark_improved, dsm_forced_replace)."""
        torch = self.torch
        dev = self.X.device
        improved = torch.zeros(self.S, dtype=torch.uint8, device=dev)
        for _, acc, *_ in outs:
            dsm.mark_improved(acc, improved)
        if self._fi_work is None:
            self._fi_work = torch.empty(dsm.lib().dsm_forced_work_bytes(self.p._h, self.S), dtype=torch.uint8,
                                        device=dev)
            self._no_donor = torch.full((self.S,), -1, dtype=torch.int32, device=dev)
        donor = self._donor if self._donor is not None else self._no_donor
        self.p.forced_replace(self.X, self.obj, self.cache, donor, improved, self.nis, n_replaced=self._n_replaced,
                              work=self._fi_work)
        self._donor = None

    @property
    def fi_replaced(self):
        """Forced solutions replaced by their donors, summed over generations."""
        return int(self._n_replaced.item())

    def select(self):
        """Indices (int32, device) of the tau fraction of the population with the
        fewest dominating solutions; ties by the smallest sum of objectives
        normalised to the population's range (dsm_select)."""
        n = max(1, int(round(self.tau * self.S)))
        return dsm.select(self.obj, n)

    def generation(self, surrogate=None, log=None):
        """One generation over all 8 parity classes; returns (exact evaluations, accepted)."""
        torch = self.torch
        if self.use_fi:
            self._draw_donors()
        if self.sampler == "estimated" and self.fos == "point":
            members = self._cluster()
            self._dist = []
            for pts in self.classes:
                est = [self.p.estimate_distributions(self.X, m, pts) for m in members]
                self._dist.append((torch.stack([e[0] for e in est]).contiguous(),
                                   torch.stack([e[1] for e in est]).contiguous()))
        if self.use_graph and self.collect is None:
            if self._graph is None or self._graph_sur is not surrogate:
                # warm up once on a side stream, then capture
                s = torch.cuda.Stream()
                s.wait_stream(torch.cuda.current_stream())
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    self._outs = self._steps(surrogate)
                self._graph, self._graph_sur = g, surrogate
                # capture recorded the work without running it
            self._graph.replay()
            outs = self._outs
        else:
            outs = self._steps(surrogate)
        if self.sampler == "estimated" and self.fos == "point":
            for c, (_, acc, cand, *_) in enumerate(outs):
                if self.schedule == "sdr":
                    mean, chol = self._dist[c]
                    sdr = dsm.improvement_ratio(self.offs[c], cand, acc, mean, chol, cluster=self._assign)
                    dsm.avs_update(self.mult[c], self.avs_nis[c], sdr, 25 + 6)
                    continue
                dsm.multiplier_step(acc, self.mult[c], cluster=self._assign)
        if self.use_fi:
            self._after_forcing(outs)
        counts = torch.stack([acc.sum(dtype=torch.int64) for _, acc, *_ in outs] +
                             [mask.sum(dtype=torch.int64) for mask, *_ in outs if mask is not None]).cpu().numpy()
        n_acc = int(counts[:len(outs)].sum())
        masked = iter(counts[len(outs):])
        n_exact = sum(self.S * acc.shape[1] if mask is None else int(next(masked)) for mask, acc, *_ in outs)
        self._gen += 1
        self._merge()
        self._archive = None
        return n_exact, n_acc

    def hypervolume(self):
        return hypervolume(self.archive, self.ref)


def train_surrogate(collected, seed=7, steps=2000, batch=4096, max_rows=1 << 20):
    """A surrogate trained on collected (features, part_old, part_new) rows."""
    import torch
    feats = torch.cat([c[0] for c in collected])
    old = torch.cat([c[1] for c in collected]).contiguous()
    new = torch.cat([c[2] for c in collected]).contiguous()
    sur = dsm.Surrogate(seed=seed, max_rows=max_rows, max_batch=batch)
    sur.fit_scaling(feats, sur.pack(part_old=old, part_new=new)[2])  # raw deltas new - old
    fb, tg, _ = sur.pack(feats, old, new)
    losses = sur.train(fb, tg, steps=steps, batch=batch)
    return sur, losses, feats.shape[0]


def run(problem, X, generations, sigma=1.0, seed=1, surrogate=None, train_generations=0, train_steps=2000,
        K=4, target_hv=None, log_every=0, graph=False, sampler="isotropic", tau=0.35, fos="point", clusters=1,
        ams=False, forced_improvements=False, nis_max=None, single_objective_clusters=False,
        multiplier_schedule="simple"):
    """Runs `generations` generations; with `train_generations` > 0 the first
    ones are plain and collect training rows, a surrogate is then trained and
    the remaining generations are screened.  Returns (RunLog, optimiser, surrogate)."""
    import torch
    opt = Optimiser(problem, X, sigma=sigma, seed=seed, K=K, graph=graph, sampler=sampler, tau=tau, fos=fos,
                    clusters=clusters, ams=ams, forced_improvements=forced_improvements, nis_max=nis_max,
                    single_objective_clusters=single_objective_clusters, multiplier_schedule=multiplier_schedule)
    log = RunLog()
    t_opt = 0.0  # optimisation time; the hypervolume monitoring is not counted
    sur = surrogate
    if train_generations > 0:
        opt.collect = []
    for g in range(generations):
        t0 = time.perf_counter()
        use = sur if (train_generations == 0 or g >= train_generations) else None
        n_exact, n_acc = opt.generation(surrogate=use)
        if train_generations > 0 and g + 1 == train_generations:
            sur, _, _ = train_surrogate(opt.collect, steps=train_steps,
                                        max_rows=max(1 << 16, opt.S * max(len(c) for c in opt.classes) * K))
            opt.collect = None
        torch.cuda.synchronize()
        t_opt += time.perf_counter() - t0
        log.seconds.append(t_opt)
        log.hypervolume.append(opt.hypervolume())
        log.exact_evals.append(n_exact)
        log.accepted.append(n_acc)
        log.archive_size.append(len(opt.archive))
        if log_every and (g + 1) % log_every == 0:
            print(f"[optimiser] gen {g + 1}: hv {log.hypervolume[-1]:.6g} exact {n_exact} accepted {n_acc} "
                  f"archive {len(opt.archive)} t {log.seconds[-1]:.2f}s", flush=True)
        if target_hv is not None and log.hypervolume[-1] >= target_hv:
            break
    return log, opt, sur


def seed_finer(opt, problem_fine, S_fine, seed=0, rounds=64):
    """Sec. 2.4: a random sample (with replacement when the approximation set is
    smaller) of S_fine solutions of the coarse run's approximation set, refined
    to the finer mesh on the GPU.  Refined solutions that fail the finer
    problem's constraints are replaced by further draws; if `rounds` rounds of
    draws leave places open, the whole approximation set is refined once and
    the rest is drawn from its feasible members (with replacement when they
    are fewer).  Returns the device population and the number of draws
    rejected."""
    import torch
    pool = opt.archive_X
    if pool is None:
        raise ValueError("the coarse optimiser must keep its archive solutions (keep_solutions=True)")
    rng = np.random.default_rng(seed)
    dev = opt.X.device
    out, rejected = [], 0
    need = S_fine
    for _ in range(rounds):
        idx = rng.choice(len(pool), size=need, replace=len(pool) < need)
        Xf = dsm.refine_population(opt.p.mesh, torch.from_numpy(np.ascontiguousarray(pool[idx])).to(dev))
        ok = (problem_fine.fold_check(Xf) == 0).cpu().numpy()
        rejected += int((~ok).sum())
        out.append(Xf[torch.from_numpy(ok).to(dev)])
        need = S_fine - sum(x.shape[0] for x in out)
        if need == 0:
            break
    if need:
        feasible = []
        for b in range(0, len(pool), 4096):
            Xb = dsm.refine_population(opt.p.mesh, torch.from_numpy(np.ascontiguousarray(pool[b:b + 4096])).to(dev))
            feasible.append(b + np.nonzero((problem_fine.fold_check(Xb) == 0).cpu().numpy())[0])
        feasible = np.concatenate(feasible)
        if len(feasible) == 0:
            raise RuntimeError("no solution of the approximation set stays feasible when refined")
        idx = rng.choice(feasible, size=need, replace=len(feasible) < need)
        out.append(dsm.refine_population(opt.p.mesh, torch.from_numpy(np.ascontiguousarray(pool[idx])).to(dev)))
    return torch.cat(out)[:S_fine].contiguous(), rejected
