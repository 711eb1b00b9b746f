/*
 * dsm.h -- C ABI of libdsm: GPU (gfx950) evaluation of the objectives and
 * constraints of multi-objective dual simplex-mesh deformable registration
 * (Andreadis, Bosman, Alderliesten, "Multi-Objective Dual Simplex-Mesh Based
 * Deformable Image Registration for 3D Medical Images -- Proof of Concept").
 *
 * A problem holds a source ("moving") and a target ("fixed") image of equal
 * dimensions and two coupled tetrahedral meshes of the same topology, one per
 * image (Sec. 2.1: dual-dynamic grid model; each cube of 8 grid points split
 * into 6 tetrahedra, cubes mirrored in 2x2x2 groups).  A solution is the
 * coordinates of all points of both meshes; a population of S solutions is
 * evaluated at once, in full or partially per FOS element (Sec. 2.2, 2.3).
 *
 * Conventions shared by every entry point
 *   - Images are float32 [Dz][Dy][Dx], x fastest.  Voxel (i,j,k) has its centre
 *     at (i,j,k) in voxel units; each mesh spans the box [-0.5, D-0.5].
 *   - Grid point (i,j,k) has index i + nx*(j + ny*k).  Grid 0 is the source
 *     (moving) grid, grid 1 the target (fixed) grid.
 *   - Coordinates are float32 voxel units on the 1/128-voxel lattice:
 *     (x + 0.5) * 128 must be an integer in [0, 128*D].  Off-lattice,
 *     out-of-box or non-finite values are reported as flag bits, never read as
 *     addresses.
 *   - A population X is float32 [S][2][P][3] (solution, grid, point, xyz).
 *   - "dev" pointers are device memory of the current HIP device, owned by the
 *     caller and kept alive until the work enqueued on `stream` has finished;
 *     "host" pointers are read during the call only.  The library never frees
 *     caller memory.
 *   - Every evaluation call only enqueues work on `stream` (a hipStream_t;
 *     NULL = the null stream) and returns: no host synchronisation, no
 *     allocation after dsm_problem_create, so the calls can be captured in a
 *     HIP graph.  Calls on one problem must not run concurrently on different
 *     streams (they share the problem's workspace).
 *   - Sizes of zero (S = 0, F = 0, no jobs) are valid: the call enqueues nothing
 *     and returns DSM_OK, and the pointers of the empty buffers may be NULL.
 *   - Errors: every function returns a dsm_status; nothing throws across the
 *     ABI.  Host-detectable errors (null pointers, sizes, capacities) are
 *     returned before anything is enqueued.  Errors in device-resident values
 *     become flag bits of the affected solution; objectives of flagged entries
 *     are unspecified.  dsm_last_error() gives a thread-local message.
 */
#ifndef DSM_H
#define DSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dsm_status;
#define DSM_OK 0
#define DSM_ERR_ARG 1         /* null pointer, bad shape or size */
#define DSM_ERR_CAPACITY 2    /* S / F / FOS size above the create-time maximum */
#define DSM_ERR_DOMAIN 3      /* geometry outside what the exact predicates support */
#define DSM_ERR_DEVICE 4      /* HIP runtime error (no device, launch failure) */
#define DSM_ERR_NOMEM 5       /* device allocation failed at create */
#define DSM_ERR_UNSUPPORTED 6

/* Constraint flag bits of a solution or candidate (Sec. 2.3.4: no grid
 * folding; border points stay on their border).  Folding is tested exactly:
 * a tetrahedron is folded iff its orientation determinant is <= 0. */
#define DSM_FLAG_INV_MOVING 1u  /* a tetrahedron of the source grid is inverted or flat */
#define DSM_FLAG_INV_FIXED 2u   /* a tetrahedron of the target grid is inverted or flat */
#define DSM_FLAG_BORDER 4u      /* a border point left its border plane */
#define DSM_FLAG_DOMAIN 8u      /* a coordinate lies outside the image box */
#define DSM_FLAG_LATTICE 16u    /* a coordinate is not on the 1/128-voxel lattice */
#define DSM_FLAG_NONFINITE 32u  /* a coordinate is NaN or infinite */
#define DSM_FLAG_BAD_FOS 64u    /* FOS element malformed (point index, size) */
#define DSM_FLAG_SKIPPED 128u   /* not evaluated: masked out by the caller */

const char* dsm_status_string(dsm_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* dsm_last_error(void);

typedef struct dsm_problem dsm_problem;

typedef struct {
  int32_t dims[3];          /* Dx, Dy, Dz: 2 <= D <= 512 */
  float spacing_mm[3];      /* voxel spacing, > 0 */
  const float* moving;      /* host [Dz][Dy][Dx] source image (copied) */
  const float* fixed;       /* host [Dz][Dy][Dx] target image (copied) */
  int32_t mesh[3];          /* points per axis nx, ny, nz: 2 <= n <= 129 */
  float empty_tau;          /* a voxel is empty (black) iff its value <= tau (Sec. 2.3.1) */
  int32_t n_guid_moving;    /* guidance points on the source image (Sec. 2.3.3), may be 0 */
  int32_t n_guid_fixed;     /* guidance points on the target image */
  const float* guid_moving; /* host [n][3] voxel units, on the lattice, within [0, D-1] */
  const float* guid_fixed;
  const int32_t* corr_moving; /* host [n] correspondence id of each point */
  const int32_t* corr_fixed;
  int32_t max_solutions;    /* largest S any later call passes */
  int32_t max_fos;          /* largest F */
  int32_t max_fos_points;   /* largest number of points in one FOS element */
} dsm_problem_desc;

typedef struct {
  int32_t P, T, E;      /* points per grid, tetrahedra (6 per cube), unique edges */
  int32_t max_star;     /* most tetrahedra incident to one point */
  int64_t V;            /* voxels per image */
  int32_t max_affected; /* capacity of one FOS element's affected set */
  double norm[3];       /* normalisers: 1/(V_fixed+V_moving), 1/(E+4T), 1/(n_guid_moving+n_guid_fixed) or 0 */
  int32_t pitch;        /* row pitch (elements) of the device image layout; see dsm_problem_set_pitch */
} dsm_problem_info;

/* Copies the images and guidance to the current device, builds the topology
 * (Sec. 2.1), the per-point stars (Sec. 2.2) and the workspace for the given
 * capacities.  Errors: DSM_ERR_ARG for null/invalid fields, DSM_ERR_DOMAIN for
 * dims/mesh outside the supported range or guidance off the lattice/box,
 * DSM_ERR_DEVICE / DSM_ERR_NOMEM from the runtime.  *out is NULL on error. */
dsm_status dsm_problem_create(const dsm_problem_desc* desc, dsm_problem** out);
dsm_status dsm_problem_destroy(dsm_problem* p);
dsm_status dsm_problem_query(const dsm_problem* p, dsm_problem_info* out);

/* Host copies of the topology: tets host [T][4] (positively oriented on the
 * undeformed grid), star_off host [P+1] and star host [4T] (tetrahedra incident
 * to each point, ascending), identity host [P][3] (undeformed grid on the
 * lattice).  Any output may be NULL. */
dsm_status dsm_problem_topology(const dsm_problem* p, int32_t* tets, int32_t* star_off, int32_t* star,
                                float* identity);

/* Host-only variant of the above for a mesh without a problem (no device
 * needed): counts host [4] = {P, T, E, max_star}; tets host [T][4];
 * star_off host [P+1]; star host [4T]; identity host [P][3] for an image of
 * dims (Dx, Dy, Dz).  Any output may be NULL; query counts first to size them. */
dsm_status dsm_mesh_topology(const int32_t mesh[3], const int32_t dims[3], int32_t* counts, int32_t* tets,
                             int32_t* star_off, int32_t* star, float* identity);

/* Sec. 2.3.4 constraint check of whole solutions.
 * X dev [S][2][P][3]; flags dev [S] (OR of DSM_FLAG_* over all points and all
 * tetrahedra of both grids); first_bad_tet dev [S] or NULL: lowest folded
 * tetrahedron id, -1 if none. */
dsm_status dsm_fold_check(dsm_problem* p, int32_t S, const float* X, uint32_t* flags, int32_t* first_bad_tet,
                          void* stream);

/* Sec. 2.3: full evaluation of S solutions.
 * obj dev [S][3] float64: dissimilarity (Sec. 2.3.1, forward + backward, divided
 * by V_fixed + V_moving), deformation (Sec. 2.3.2, divided by E + 4T),
 * guidance (Sec. 2.3.3, divided by the number of guidance points).
 * flags dev [S] as dsm_fold_check.  tet_terms dev [S][T][3] float64 or NULL:
 * the un-normalised per-tetrahedron terms (the decomposition of Sec. 2.3 that
 * partial evaluation relies on); pass it to dsm_eval_partial as the cache. */
dsm_status dsm_eval_full(dsm_problem* p, int32_t S, const float* X, double* obj, uint32_t* flags, double* tet_terms,
                         void* stream);

/* Sec. 2.2-2.3: partial evaluation of every (solution, FOS element) pair.
 * FOS element f holds points fos_pts[fos_off[f] .. fos_off[f+1]) (dev int32,
 * fos_off dev [F+1]); its candidate coordinates, in both grids, are
 * cand dev [S][fos_off[F]][2][3].  The affected tetrahedra are the union of the
 * stars of the element's points.  Outputs, all dev:
 *   part_new [S][F][3] float64: normalised objective sums over the affected
 *     tetrahedra with the candidate coordinates;
 *   part_old [S][F][3] float64: the same sums for the current coordinates, from
 *     tet_terms_in [S][T][3] (as written by dsm_eval_full) if non-NULL, else
 *     recomputed; so full(new) = full(old) - part_old + part_new;
 *   flags [S][F]: constraint bits over the affected tetrahedra and their
 *     vertices with the candidate applied;
 *   tet_terms_new [S][T][3] or NULL: candidate terms of the affected
 *     tetrahedra written in place (other entries untouched); only meaningful
 *     when the elements' affected sets are pairwise disjoint;
 *   voxel_count [S][F] uint32 or NULL: voxel samples taken for the candidate.
 * Errors: DSM_ERR_CAPACITY if S or F exceeds the create-time maximum; a
 * malformed element (point out of range, more than max_fos_points points)
 * sets DSM_FLAG_BAD_FOS for that element. */
dsm_status dsm_eval_partial(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                            const int32_t* fos_pts, const float* cand, const double* tet_terms_in, double* part_old,
                            double* part_new, uint32_t* flags, double* tet_terms_new, uint32_t* voxel_count,
                            void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * partial evaluation as dsm_eval_partial, with identical results, whose
 * workspace (affected sets, element order, per-tetrahedron swept sums,
 * per-chunk flags and voxel counts) lives in a fixed array of
 * DSM_SCRATCH_BYTES per device, held from the first call on a device until
 * the process ends, instead of the problem's create-time workspace; S and F
 * are therefore not bounded by max_solutions / max_fos.  The call allocates
 * nothing and only enqueues on `stream`.  Every call on one device shares that
 * device's array and leaves its contents behind (nothing in it needs to start
 * at zero): calls that overlap on one device race, across problems, streams
 * and threads alike, so serialise them (one stream, or events).  The problem
 * must live on the current device.  Workspace bytes: 256-byte aligned regions
 * of 4 F maxA + 8 F + 8 S F nver maxA + 8 S F ceil(maxA / 8), with nver = 1
 * if tet_terms_in is given, else 2, and maxA = dsm_problem_info.max_affected.
 * Errors: DSM_ERR_CAPACITY if that exceeds DSM_SCRATCH_BYTES (split the
 * population into calls of fewer solutions); DSM_ERR_ARG for null pointers or
 * a problem of another device; DSM_ERR_DEVICE. */
#define DSM_SCRATCH_BYTES (64u << 20)
dsm_status dsm_eval_partial_noalloc(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                    const int32_t* fos_pts, const float* cand, const double* tet_terms_in,
                                    double* part_old, double* part_new, uint32_t* flags, double* tet_terms_new,
                                    uint32_t* voxel_count, void* stream);

/* dsm_eval_partial restricted to the (solution, element) pairs whose entry in
 * mask dev [S][F] (uint8) is non-zero; the other pairs cost a workgroup launch
 * only, get flags = DSM_FLAG_SKIPPED, zero partial sums and no term writes.
 * mask NULL evaluates every pair. */
dsm_status dsm_eval_partial_masked(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                   const int32_t* fos_pts, const float* cand, const uint8_t* mask,
                                   const double* tet_terms_in, double* part_old, double* part_new, uint32_t* flags,
                                   double* tet_terms_new, uint32_t* voxel_count, void* stream);

/* Several registration problems in one fused launch (one workgroup list over
 * every job's (solution, element) pairs).  A batch object owns the device job
 * table (max_jobs entries) and a pinned staging copy; it is created once. */
typedef struct dsm_batch dsm_batch;
typedef struct {
  dsm_problem* problem;         /* distinct problems within one call (they own the workspaces) */
  int32_t S;
  const float* X;               /* as dsm_eval_partial_masked, per job */
  int32_t F;
  const int32_t* fos_off;
  const int32_t* fos_pts;
  const float* cand;
  const uint8_t* mask;          /* may be NULL */
  const double* tet_terms_in;   /* may be NULL (current terms recomputed) */
  double* part_old;
  double* part_new;
  uint32_t* flags;
  double* tet_terms_new;        /* may be NULL */
  uint32_t* voxel_count;        /* may be NULL */
} dsm_partial_job;

dsm_status dsm_batch_create(int32_t max_jobs, dsm_batch** out);
dsm_status dsm_batch_destroy(dsm_batch* b);
/* Enqueues the partial evaluation of every job (results identical to one
 * dsm_eval_partial_masked call per job).  Errors: DSM_ERR_ARG (null, repeated
 * problem), DSM_ERR_CAPACITY (n_jobs > max_jobs or a job above its problem's
 * capacities).  Waits on the host only for the previous call's job-table copy. */
dsm_status dsm_eval_partial_batch(dsm_batch* b, int32_t n_jobs, const dsm_partial_job* jobs, void* stream);

/* The same fused evaluation split into a set-up call and an enqueue-only call,
 * so that a generation over several problems (e.g. both pyramid levels of
 * uneven problems) can be captured in a HIP graph and replayed.
 * dsm_batch_set_jobs validates the jobs as dsm_eval_partial_batch does and
 * stores their job table on the device (synchronously: it waits for the device
 * to be idle, so call it before any capture); every pointer in the jobs is
 * kept and must stay valid while the configuration is used.  The caller
 * changes inputs between runs by writing into the same buffers.
 * dsm_batch_run enqueues the affected-set, ordering, sweep and finishing
 * kernels of the stored configuration on `stream`: no allocation, no copy, no
 * host wait.  Results are identical to dsm_eval_partial_batch on the same
 * jobs.  dsm_eval_partial_batch and dsm_batch_set_jobs use separate device
 * tables; a new dsm_batch_set_jobs replaces the stored configuration.  Errors:
 * as dsm_eval_partial_batch; dsm_batch_run without a configuration is a
 * no-op. */
dsm_status dsm_batch_set_jobs(dsm_batch* b, int32_t n_jobs, const dsm_partial_job* jobs);
dsm_status dsm_batch_run(dsm_batch* b, void* stream);

/* Device image layout.  The sampled images are stored on the device with a
 * replicated one-voxel border, z-pairs interleaved, in rows of `pitch`
 * elements (pitch >= Dx + 2).  The pitch changes no result, only speed: the
 * trilinear gathers of one wave touch several rows at once, and some row
 * strides make them collide in the memory pipeline.  dsm_problem_set_pitch
 * re-packs the images for `pitch` (0 = the built-in default); it allocates and
 * synchronises the device, so call it at setup, not during capture.  Errors:
 * DSM_ERR_ARG for a pitch below Dx + 2, above 4 (Dx + 2) + 64, or an image
 * above 2 GiB. */
dsm_status dsm_problem_set_pitch(dsm_problem* p, int32_t pitch);

/* Autotuning of the layout for one partial-evaluation workload (the same
 * arguments as dsm_eval_partial, dev pointers): for each of the n_pitch host
 * candidates `pitches` (n_pitch 0: a built-in list around the default),
 * re-packs the images, runs the partial evaluation twice on the null stream and
 * records the second run's time in ms_out host [n_pitch] (or [6] for the
 * built-in list; may be NULL); the fastest pitch is kept and returned in
 * *best (may be NULL).  Setup-time call: allocates temporary outputs and
 * synchronises. */
dsm_status dsm_autotune_pitch(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                              const int32_t* fos_pts, const float* cand, const double* tet_terms_in, int32_t n_pitch,
                              const int32_t* pitches, float* ms_out, int32_t* best);

/* Work split of the partial evaluation.  Each workgroup of a partial
 * evaluation sweeps one chunk of `chunk` affected tetrahedra of one (element,
 * solution) pair, both directions; the chunk changes no voxel set, flag or
 * count, only the speed (smaller chunks give more, shorter workgroups) and
 * the rounding of the dissimilarity: the waves' per-lane compensated FP32
 * sums follow the work split (relative differences of order 1e-9 for element
 * sums, up to about 1e-7 for single tetrahedra; at most 4 x 2^-24).
 * dsm_set_part_chunk sets it for later partial evaluations of p (default 8);
 * it neither allocates nor synchronises, but a stored batch configuration
 * keeps the chunk it was stored with.  Errors: DSM_ERR_ARG for a chunk
 * outside [4, 8].  dsm_get_part_chunk returns the current chunk (0 for a null
 * problem). */
dsm_status dsm_set_part_chunk(dsm_problem* p, int32_t chunk);
int32_t dsm_get_part_chunk(const dsm_problem* p);

/* Autotuning of the chunk for one partial-evaluation workload, like
 * dsm_autotune_pitch: for each of the n_chunk host candidates `chunks`
 * (n_chunk 0: 4, 5, 6, 7, 8) runs the partial evaluation twice on the null
 * stream and records the second run's time in ms_out host [n_chunk] (or [5];
 * may be NULL); the fastest chunk is kept and returned in *best (may be NULL).
 * Setup-time call: allocates temporary outputs and synchronises.  Errors as
 * dsm_set_part_chunk for a candidate, as dsm_eval_partial for the rest. */
dsm_status dsm_autotune_chunk(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                              const int32_t* fos_pts, const float* cand, const double* tet_terms_in, int32_t n_chunk,
                              const int32_t* chunks, float* ms_out, int32_t* best);

/* Order of the voxel rows that the sweep of the objectives' dissimilarity
 * term (Sec. 2.3.1) visits within a tetrahedron.  DSM_ROWS_BY_SLICE (the
 * default): y-major within each voxel slice z.  DSM_ROWS_BY_SLICE_PAIR: slices
 * taken in pairs (z, z + 1) whose rows alternate, (y, z), (y, z + 1),
 * (y + 1, z), ..., so the two rows of one y read the same elements of the own
 * image (which holds the values at z and z + 1 side by side): fewer cache
 * lines per sample on tetrahedra with long rows, more candidate rows to build
 * on small ones.  The order changes no voxel set, flag or count, only the speed
 * and the rounding of the dissimilarity (as for the chunk); it applies to full and partial evaluations of p, and a
 * stored batch configuration keeps the order it was stored with.
 * dsm_set_row_order neither allocates nor synchronises.  Errors: DSM_ERR_ARG
 * for another value.  dsm_get_row_order returns the current order (-1 for a
 * null problem). */
#define DSM_ROWS_BY_SLICE 0
#define DSM_ROWS_BY_SLICE_PAIR 1
dsm_status dsm_set_row_order(dsm_problem* p, int32_t order);
int32_t dsm_get_row_order(const dsm_problem* p);

/* Autotuning of the row order for one partial-evaluation workload, like
 * dsm_autotune_chunk: runs the partial evaluation twice on the null stream
 * with each order (DSM_ROWS_BY_SLICE, then DSM_ROWS_BY_SLICE_PAIR) and records
 * the second run's time in ms_out host [2] (may be NULL); the faster order is
 * kept and returned in *best (may be NULL).  Setup-time call: allocates
 * temporary outputs and synchronises.  Errors as dsm_eval_partial. */
dsm_status dsm_autotune_row_order(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                  const int32_t* fos_pts, const float* cand, const double* tet_terms_in,
                                  float* ms_out, int32_t* best);

/* Test hook for Sec. 2.3.1 rasterisation: owner dev [Dz][Dy][Dx] int32 receives
 * the id of the tetrahedron of grid coordinates Xgrid dev [P][3] whose exact
 * voxel set contains each voxel (-1 if none); overlap dev [1] int32 counts
 * voxels claimed more than once.  With a feasible mesh every voxel is owned
 * exactly once. */
dsm_status dsm_rasterize_owner(dsm_problem* p, const float* Xgrid, int32_t* owner, int32_t* overlap, void* stream);

/* The registration result (Sec. 2.1: corresponding tetrahedra of the two
 * grids define a piecewise-affine map; Sec. 3, Fig. 2 shows it as a
 * transformed source image and a deformation vector field).  For one solution
 * X dev [2][P][3] (the layout of one entry of a population) and every voxel v
 * of image `own` (0 source, 1 target), x(v) is the point the map sends v's
 * centre to in the other image: v is located in its tetrahedron of grid `own`
 * by the exact voxel sets of the objectives and mapped with FP64 barycentric
 * coordinates.  Writes, each output optional (NULL):
 *   dvf    dev [Dz][Dy][Dx][3] f32, x(v) - v in voxel units (x, y, z);
 *   warped dev [Dz][Dy][Dx] f32, the other image sampled at x(v) (trilinear,
 *          clamped to the box): for own = 1 the transformed source image.
 * Voxels in no tetrahedron, which a feasible solution cannot leave, are NaN;
 * for a solution that folds the outputs are undefined.  Enqueued on `stream`;
 * no allocation.  Errors: DSM_ERR_ARG (null problem or X, own not 0 or 1),
 * DSM_ERR_DEVICE. */
dsm_status dsm_transform(dsm_problem* p, int32_t own, const float* X, float* dvf, float* warped, void* stream);

/* Measurement support.  dsm_problem_timing(p, capacity) with capacity > 0
 * creates `capacity` pairs of HIP events; each following dsm_eval_full /
 * dsm_eval_partial call records one pair around its voxel-sweep kernel on the
 * call's stream (until the pairs run out).  capacity 0 disables timing and
 * frees the events.  Not for use inside HIP graph capture.
 * dsm_problem_timing_read waits for the recorded events, writes the sweep
 * durations in milliseconds to ms host [max_n] in call order, their number to
 * *n, and rewinds the pairs for reuse.  Errors: DSM_ERR_ARG (null, negative),
 * DSM_ERR_DEVICE. */
dsm_status dsm_problem_timing(dsm_problem* p, int32_t capacity);
dsm_status dsm_problem_timing_read(dsm_problem* p, float* ms, int32_t max_n, int32_t* n);

/* ---------------------------------------------------------------------------
 * Learned pre-screening of partial-evaluation candidates (single-point FOS
 * elements).  Not part of the paper's method: a small MLP 192 -> 128 -> 128 ->
 * 3 (ReLU) predicts the three objective deltas of a candidate from local
 * features and is trained on the deltas that dsm_eval_partial computes
 * exactly; the exact evaluation still decides every accepted change.
 * Matrix products run as BF16 matrix-core instructions with FP32 accumulation;
 * master weights and Adam state are FP32.
 *
 * Feature row of candidate k of element f (single point p) of solution s,
 * float32 [192]:
 *   [0, 6)     candidate minus current position of p (grid 0 xyz, grid 1 xyz);
 *   [6, 162)   for each of the 26 lattice neighbours q = p + o, o in
 *              {-1,0,1}^3 without 0 (dz, dy, dx order, dx fastest), grid 0 then
 *              grid 1, xyz: (X[q] - candidate) - (U[q] - U[p]) with U the
 *              undeformed grid; 0 where q does not exist;
 *   [162, 188) source image at (grid-0 candidate + h o) minus target image at
 *              (grid-1 candidate + h o), clamped trilinear, h = half the
 *              undeformed cube extent per axis;
 *   [188, 192) 0.
 * Network inputs are the rows standardised with the fitted scaling and rounded
 * to BF16; outputs are standardised deltas.
 * ------------------------------------------------------------------------- */
#define DSM_SUR_FEATURES 192
#define DSM_SUR_HIDDEN 128
#define DSM_SUR_OUTPUTS 3
#define DSM_SUR_NPARAMS 43280 /* W1[128][192] b1[128] W2[128][128] b2[128] W3[16][128] b3[16]; rows 3..15 of W3 and b3 unused (0) */

typedef struct dsm_surrogate dsm_surrogate;
typedef struct {
  uint64_t seed;     /* weight initialisation and minibatch sampling */
  float lr, beta1, beta2, eps; /* Adam */
  int32_t max_rows;  /* largest S*F*K passed to dsm_surrogate_screen */
  int32_t max_batch; /* largest minibatch / gradient batch (multiple of 32) */
} dsm_surrogate_desc;

dsm_status dsm_surrogate_create(const dsm_surrogate_desc* desc, dsm_surrogate** out);
dsm_status dsm_surrogate_destroy(dsm_surrogate* s);
const char* dsm_surrogate_last_error(void);
/* FP32 master parameters, host [DSM_SUR_NPARAMS]: set != 0 writes them (and
 * refreshes the BF16 copies, synchronously), else reads them. */
dsm_status dsm_surrogate_params(dsm_surrogate* s, float* host, int32_t set);
/* Fits the input / output standardisation to N feature rows feats dev
 * [N][192] and raw deltas dev [N][3] (column mean and 1/std; constant columns
 * get 1/std = 1).  Synchronises the stream. */
dsm_status dsm_surrogate_fit_scaling(dsm_surrogate* s, int32_t N, const float* feats, const float* deltas, void* stream);
/* Host copies of the fitted scaling (any output may be NULL). */
dsm_status dsm_surrogate_get_scaling(dsm_surrogate* s, float* in_mean, float* in_rstd, float* out_mean, float* out_rstd);
/* Sets the scaling from host [192], [192], [3], [3] arrays (e.g. those of
 * another network, for comparisons at equal standardisation); synchronous. */
dsm_status dsm_surrogate_set_scaling(dsm_surrogate* s, const float* in_mean, const float* in_rstd, const float* out_mean,
                                     const float* out_rstd);
/* Raw feature rows feats dev [S*F*K][192] for candidates cand dev
 * [S][F][K][2][3] of single-point elements fos_pts dev [F] of solutions X. */
dsm_status dsm_surrogate_features(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                  const float* cand, float* feats, void* stream);
/* The rows of dsm_surrogate_features, standardised with the surrogate's input
 * statistics and rounded to BF16 in one pass: feats_bf16 dev [S*F*K][192] is
 * bit for bit what dsm_surrogate_pack makes of the FP32 rows (the screening
 * path; no FP32 rows are written). */
dsm_status dsm_surrogate_features_packed(dsm_surrogate* s, dsm_problem* p, int32_t S, const float* X, int32_t F,
                                         const int32_t* fos_pts, int32_t K, const float* cand, uint16_t* feats_bf16,
                                         void* stream);
/* Standardises N rows: feats dev [N][192] -> feats_bf16 dev [N][192] (bits of
 * BF16), and deltas part_new - part_old (dev [N][3] float64) -> targets dev
 * [N][3] (standardised) and raw_deltas dev [N][3]; any pair may be NULL. */
dsm_status dsm_surrogate_pack(dsm_surrogate* s, int32_t N, const float* feats, uint16_t* feats_bf16,
                              const double* part_old, const double* part_new, float* targets, float* raw_deltas,
                              void* stream);
/* Network outputs (standardised) pred dev [N][3] for BF16 rows. */
dsm_status dsm_surrogate_forward(dsm_surrogate* s, int32_t N, const uint16_t* feats_bf16, float* pred, void* stream);
/* Gradient of the mean squared error (1/N sum_rows mean_outputs (y - t)^2)
 * over all N <= max_batch rows, without an update: grad dev [DSM_SUR_NPARAMS]
 * in the parameter layout, loss dev [1] or NULL. */
dsm_status dsm_surrogate_gradient(dsm_surrogate* s, int32_t N, const uint16_t* feats_bf16, const float* targets,
                                  float* grad, float* loss, void* stream);
/* `steps` Adam steps on minibatches of `batch` rows drawn (counter-based, with
 * replacement) from the N rows; loss dev [steps] or NULL receives each
 * minibatch loss before its update. */
dsm_status dsm_surrogate_train(dsm_surrogate* s, int32_t N, const uint16_t* feats_bf16, const float* targets,
                               int32_t steps, int32_t batch, float* loss, void* stream);
/* Screens K candidates cand dev [S][F][K][2][3] of single-point elements:
 * pick dev [S][F] = the candidate with the best predicted Pareto rank among the
 * K (ties: smallest sum of standardised predictions); run_exact dev [S][F] = 1
 * iff its predicted delta is accepted by the rule of dsm_accept (with obj dev
 * [S][3] and an archive dev [n_archive][3], +inf rows ending it; without them only changes that
 * improve an objective and worsen none pass).  pred dev
 * [S][F][K][3] (raw predicted deltas) and cand_pick dev [S][F][2][3] (the
 * picked candidates) may be NULL.  Errors: DSM_ERR_CAPACITY if S*F*K > max_rows. */
dsm_status dsm_surrogate_screen(dsm_surrogate* s, dsm_problem* p, int32_t S, const float* X, int32_t F,
                                const int32_t* fos_pts, int32_t K, const float* cand, const double* obj,
                                int32_t n_archive, const double* archive, float* pred, int32_t* pick,
                                uint8_t* run_exact, float* cand_pick, void* stream);

/* ---------------------------------------------------------------------------
 * Generation steps of a population optimiser (single-point FOS elements).
 * ------------------------------------------------------------------------- */

/* cand dev [S][F][K][2][3]: the current position of point fos_pts[f] (dev [F])
 * in both grids plus N(0, sigma) voxels on its free (non-border) axes, clamped to
 * the image box and rounded to the 1/128-voxel lattice.  The normal deviates
 * come from a counter-based generator keyed by (seed, counter, element index):
 * equal arguments give equal candidates.  counter_dev dev [1] or NULL: when
 * given, the counter is counter + *counter_dev, read when the kernel runs (a
 * captured HIP graph then draws new candidates on every replay once the
 * caller advances *counter_dev on the device). */
dsm_status dsm_sample_candidates(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                 float sigma, uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                                 void* stream);

/* Distribution estimation of RV-GOMEA, the optimiser Sec. 2.2 builds on: its
 * partial changes draw a FOS element's variables from a normal distribution
 * estimated on selected solutions.  For single-point elements fos_pts dev [F]
 * the variables are the point's 6 coordinates (source x y z, target x y z);
 * coordinates pinned to the box are not variables.  Writes mean dev [F][6]
 * (float64) over the solutions sel dev [n_sel] of X dev [S][2][P][3] (indices
 * outside [0, S) are skipped) and chol dev [F][21] (float64): the lower
 * Cholesky factor, row r holding columns 0..r, of the maximum-likelihood
 * covariance (divisor: the number of solutions used) of the free coordinates;
 * pinned rows and columns are 0, and a non-positive pivot (rank-deficient
 * selection) gives a zero column.  An element with no valid solution or an
 * invalid point gets zeros.  Errors: DSM_ERR_ARG (null pointers, negative
 * sizes). */
dsm_status dsm_estimate_distributions(dsm_problem* p, int32_t S, const float* X, int32_t n_sel, const int32_t* sel,
                                      int32_t F, const int32_t* fos_pts, double* mean, double* chol, void* stream);

/* Candidates cand dev [S][F][K][2][3] drawn from the estimated distributions:
 * mean + sqrt(mult[f]) L z on the free coordinates of point fos_pts[f], z
 * standard normal from the same counter-based generator as
 * dsm_sample_candidates (6 draws per candidate; counter + *counter_dev when
 * counter_dev is given); pinned coordinates keep the solution's value; the
 * result is clamped to the image box and rounded to the 1/128-voxel lattice
 * (half to even).  mult dev [F] (float) are the distribution multipliers.  An
 * invalid point gives NaN candidates (flagged non-finite by the evaluator).
 * Clusters (MO-RV-GOMEA, Sec. 2.2): with n_clusters distributions per element,
 * mean [n_clusters][F][6], chol [n_clusters][F][21] and mult [n_clusters][F],
 * solution s draws from those of cluster dev [S] entry cluster[s]; a cluster
 * index outside [0, n_clusters) gives NaN candidates.  cluster NULL: every
 * solution uses the first (n_clusters 1 for a single distribution).
 * Anticipated mean shift (RV-GOMEA): with shift dev [P][6] float64 (per grid
 * point, source x y z then target x y z) and ams dev [S] uint8, a solution
 * with ams[s] != 0 draws around mean + delta * mult * shift[p] on the free
 * coordinates (delta is 2 in RV-GOMEA); shift NULL: no shift (ams unused).
 * Errors: DSM_ERR_ARG (also n_clusters < 1, or shift without ams). */
dsm_status dsm_sample_estimated(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                const double* mean, const double* chol, const float* mult, int32_t n_clusters,
                                const int32_t* cluster, const double* shift, const uint8_t* ams, double delta,
                                uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                                void* stream);

/* dsm_estimate_distributions for elements of up to 4 points (e.g. the paper's
 * per-cube tetrahedra), jointly: the variables of element f are the
 * coordinates of its points fos_pts[fos_off[f] .. fos_off[f+1]), 6 per point
 * in order (source x y z, target x y z).  mean dev [F][24] and chol dev
 * [F][300] (float64; row r of the lower factor holds columns 0..r) over the
 * solutions sel dev [n_sel] of X (indices outside [0, S) skipped); rows and
 * columns of pinned coordinates and of unused variables are 0.  Elements with
 * no point, more than 4 points, an invalid point or malformed offsets get
 * zeros.  Errors: DSM_ERR_ARG. */
dsm_status dsm_estimate_elements(dsm_problem* p, int32_t S, const float* X, int32_t n_sel, const int32_t* sel, int32_t F,
                                 const int32_t* fos_off, const int32_t* fos_pts, double* mean, double* chol,
                                 void* stream);

/* Candidates cand dev [S][fos_off[F]][2][3] (the layout of dsm_eval_partial)
 * drawn per solution and element from N(mean, mult[f] L L^T) on the element's
 * free variables (24 counter-based standard normal draws per solution and
 * element); pinned coordinates keep the solution's value; clamped to the box
 * and rounded to the lattice.  Elements rejected by dsm_estimate_elements get
 * NaN candidates (flagged non-finite by the evaluator); elements with
 * malformed offsets are not written.  Clusters (n_clusters, cluster) and the
 * anticipated mean shift (shift dev [P][6], ams dev [S], delta) as for
 * dsm_sample_estimated, with the shift of each of the element's points.
 * Errors: DSM_ERR_ARG. */
dsm_status dsm_sample_elements(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                               const int32_t* fos_pts, const double* mean, const double* chol, const float* mult,
                               int32_t n_clusters, const int32_t* cluster, const double* shift, const uint8_t* ams,
                               double delta, uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                               void* stream);

/* Forced improvements (RV-GOMEA, on which the optimisation of Sec. 2.2
 * builds): for every solution s whose donor dev [S] entry donor[s] lies in
 * [0, S), the candidate of each listed point fos_pts dev [n_pts] becomes the
 * donor solution's current coordinates in both grids: cand dev
 * [S][n_pts][2][3] (the layout of dsm_eval_partial; for CSR elements n_pts =
 * fos_off[F]).  Other solutions' candidates, and points outside [0, P), are
 * left unchanged.  Errors: DSM_ERR_ARG. */
dsm_status dsm_copy_from_donor(dsm_problem* p, int32_t S, const float* X, int32_t n_pts, const int32_t* fos_pts,
                               const int32_t* donor, float* cand, void* stream);

/* Adaptive variance scaling (AMaLGaM's standard-deviation ratio, used by
 * RV-GOMEA, on which the optimisation of Sec. 2.2 builds): for every cluster j
 * and element f (points fos_pts[fos_off[f] .. fos_off[f+1]), fos_off dev
 * [F+1]; single points: fos_off = 0, 1, ..., F), the mean of the candidates
 * cand dev [S][fos_off[F]][2][3] that were accepted (accepted dev [S][F]
 * uint8) by solutions of cluster j (cluster dev [S] int32, NULL: all in
 * cluster 0) is compared with the distribution mean dev [n_clusters][F][n_vars]
 * variable by variable, in units of the variable's standard deviation from
 * chol dev [n_clusters][F][n_vars (n_vars + 1) / 2] (packed lower rows);
 * sdr dev [n_clusters][F] f64 receives the largest ratio, or -1 where no
 * candidate was accepted (and for malformed elements).  Variables with zero
 * deviation (pinned) are skipped.  n_vars is 6 (single points) or 24
 * (elements of up to 4 points).  Errors: DSM_ERR_ARG. */
dsm_status dsm_improvement_ratio(int32_t S, int32_t F, const int32_t* fos_off, const float* cand,
                                 const uint8_t* accepted, int32_t n_clusters, const int32_t* cluster,
                                 const double* mean, const double* chol, int32_t n_vars, double* sdr, void* stream);

/* Balanced k-leader-means clustering of selected solutions in objective space
 * (MO-RV-GOMEA, on which the optimisation of Sec. 2.2 builds): per generation
 * one distribution per cluster and FOS element is estimated from the cluster's
 * members, and each solution draws from its nearest cluster.  obj dev [S][3]
 * f64 (finite), sel dev [n_sel] (indices outside [0, S) dropped, n valid
 * remain), 1 <= k <= 16, n_sel <= 1024.  Steps: objectives normalised per
 * objective to [0, 1] over the selection (zero range: divide by 1); leaders by
 * farthest-first traversal from the largest normalised first objective; k-means
 * from the leaders until no assignment changes (at most 50 rounds); cluster j
 * = the c = min(n, ceil(2n/k)) selected solutions nearest to mean j, nearest
 * first; ties to the lower selection position or cluster index; every sum in
 * selection order, so the result is reproducible bit for bit.  Outputs:
 * members dev [k][cmax] population indices with cmax = min(n_sel,
 * ceil(2 n_sel / k)) (entries past c are -1); assign dev [S] nearest cluster of
 * every solution; means dev [k][3] normalised means (may be NULL).  With n < k
 * every member and assignment is -1 and the means NaN.  One workgroup on
 * `stream`; no allocation.  Errors: DSM_ERR_ARG (sizes, k, null pointers),
 * DSM_ERR_CAPACITY (n_sel > 1024), DSM_ERR_DEVICE. */
dsm_status dsm_cluster_objectives(int32_t S, const double* obj, int32_t n_sel, const int32_t* sel, int32_t k,
                                  int32_t* members, int32_t* assign, double* means, void* stream);

/* Sec. 2.4 grid refinement for multi-resolution runs: each cube of both grids
 * is split into 8 cubes by points at the middle of every cube edge, the middle
 * of every face and the cube centre (face middles and centres are means of the
 * corners; a deformed face need not be planar), rounded to the 1/128-voxel
 * lattice half to even.  Xc dev [S][2][Pc][3] on a mesh of mesh_coarse host [3]
 * points per axis -> Xf dev [S][2][Pf][3] on (2 nx - 1, 2 ny - 1, 2 nz - 1)
 * points.  Feasibility of the result is not assumed: check it with
 * dsm_fold_check on the finer problem.  Errors: DSM_ERR_ARG (null pointers,
 * S < 0), DSM_ERR_DOMAIN (mesh outside [2, 129] per axis). */
dsm_status dsm_refine_population(const int32_t* mesh_coarse, int32_t S, const float* Xc, float* Xf, void* stream);

/* Sec. 2.2: accepts the partial changes of one evaluated batch of single-point
 * elements whose affected tetrahedra are pairwise disjoint (e.g. points of one
 * index-parity class) and applies them together.  A change is accepted iff its
 * flags are 0 and its delta (part_new - part_old, dev [S][F][3]) improves one
 * objective without worsening another, or improves one objective and the new
 * objective vector obj[s] + delta is not dominated by any of the n_archive
 * vectors archive dev [n][3]; a row whose first value is +inf ends the archive
 * (a fixed-capacity archive padded with +inf rows can be captured in a graph).  Accepted changes write cand dev [S][F][2][3] into
 * X dev [S][2][P][3] and copy the candidate terms of the point's star from
 * terms_cand dev [S][T][3] (as written by dsm_eval_partial(_masked)) into
 * terms_cache dev [S][T][3]; obj dev [S][3] is then recomputed from the cache.
 * single_objective dev [S] int32 or NULL: a solution with entry o in {0, 1, 2}
 * (a member of MO-RV-GOMEA's single-objective cluster for objective o) accepts
 * a feasible change iff it lowers objective o; other entries use the rule
 * above.  accepted dev [S][F] (uint8) or NULL. */
dsm_status dsm_accept(dsm_problem* p, int32_t S, float* X, int32_t F, const int32_t* fos_pts, const float* cand,
                      const double* part_old, const double* part_new, const uint32_t* flags, const double* terms_cand,
                      double* terms_cache, double* obj, int32_t n_archive, const double* archive,
                      const int32_t* single_objective, uint8_t* accepted, void* stream);

/* dsm_accept for elements of any number of points (e.g. the paper's per-cube
 * tetrahedron elements, Sec. 2.2): element f has the points
 * fos_pts[fos_off[f] .. fos_off[f+1]) and its candidate coordinates are
 * cand dev [S][fos_off[F]][2][3], the layout of dsm_eval_partial.  The
 * elements of one call must have pairwise disjoint affected tetrahedra.  An
 * accepted change writes all of its points and copies the candidate terms of
 * the union of their stars; single_objective as for dsm_accept. */
dsm_status dsm_accept_elements(dsm_problem* p, int32_t S, float* X, int32_t F, const int32_t* fos_off,
                               const int32_t* fos_pts, const float* cand, const double* part_old,
                               const double* part_new, const uint32_t* flags, const double* terms_cand,
                               double* terms_cache, double* obj, int32_t n_archive, const double* archive,
                               const int32_t* single_objective, uint8_t* accepted, void* stream);

/* ---------------------------------------------------------------------------
 * Generation bookkeeping on the device.  All enqueue on `stream` only; sizes
 * that live on the device (the archive's row count) are read by the kernels,
 * so the calls can be captured in a HIP graph.  Workspaces are caller-owned
 * device memory of the size the matching *_work_bytes function returns.
 * ------------------------------------------------------------------------- */

/* Bytes of workspace for dsm_archive_merge (host function, no device). */
size_t dsm_archive_work_bytes(int32_t capacity, int32_t m, int32_t row_floats);

/* Sec. 2.4 (the approximation set the finer run is seeded from): merges m
 * objective vectors points dev [m][3] float64 into the elitist archive.  The
 * archive is archive dev [capacity][3] float64 holding *n_archive (dev int32)
 * rows that are mutually non-dominated, distinct and in lexicographic order,
 * +inf in every later row, as this call leaves them (start from *n_archive = 0
 * or any such set).  Of the archive rows then the points, in that order, a
 * vector is kept iff no vector of either dominates it (minimisation) and no
 * earlier one equals it; the kept vectors are written back in lexicographic
 * order, later rows set to +inf, and *n_archive updated.  With row_floats > 0
 * every vector carries a payload row (e.g. its solution): archive_rows dev
 * [capacity][row_floats] moves with the archive, point_rows dev
 * [m][row_floats] are the points' rows.  If more than `capacity` vectors would
 * be kept, nothing changes and *overflow (dev int32, may be NULL) is set to 1,
 * else to 0.  work: dev, dsm_archive_work_bytes(capacity, m, row_floats)
 * bytes.  Errors: DSM_ERR_ARG (sizes, null pointers), DSM_ERR_DEVICE. */
dsm_status dsm_archive_merge(int32_t capacity, double* archive, int32_t* n_archive, int32_t m, const double* points,
                             int32_t row_floats, float* archive_rows, const float* point_rows, void* work,
                             int32_t* overflow, void* stream);

/* Sec. 2.2 selection for the distributions of the partial changes: the n_sel
 * of the S solutions (obj dev [S][3] float64) with the fewest population
 * members dominating them, ties by the smallest sum, in objective order, of
 * the objectives normalised to the population's range (divisor at least
 * 1e-300), then by index; sel dev [n_sel] int32 in that order.
 * dominated_by dev [S] int32 or NULL receives every solution's count.  One
 * workgroup.  Errors: DSM_ERR_ARG (n_sel outside [0, S], null pointers),
 * DSM_ERR_CAPACITY (S > 8192), DSM_ERR_DEVICE. */
dsm_status dsm_select(int32_t S, const double* obj, int32_t n_sel, int32_t* sel, int32_t* dominated_by, void* stream);

/* Adaptive variance scaling of the distribution multipliers (AMaLGaM's rule,
 * used by RV-GOMEA, Sec. 2.2), n independent distributions, float32: with
 * sdr dev [n] float64 (the standard-deviation ratio of the accepted changes,
 * < 0 where none was accepted, as dsm_improvement_ratio writes it), after an
 * improvement the multiplier is at least 1 and is divided by eta if sdr > 1,
 * and the no-improvement stretch nis restarts at 0; otherwise the stretch
 * grows by 1 while the multiplier is at most 1, the multiplier is multiplied
 * by eta if it is above 1 or the stretch reached nis_max, and reset to 1 if
 * it fell below 1 while the stretch is shorter than nis_max.  The result is
 * clamped to [lo, hi].  mult dev [n] float32 and nis dev [n] int32 are updated
 * in place.  Errors: DSM_ERR_ARG (eta outside (0, 1), lo not in (0, hi], null
 * pointers), DSM_ERR_DEVICE. */
dsm_status dsm_avs_update(int32_t n, float* mult, int32_t* nis, const double* sdr, int32_t nis_max, float eta, float lo,
                          float hi, void* stream);

/* The simple multiplier schedule of the distributions (a simplification of
 * the adaptive variance scaling above): for every cluster j < k and element
 * f, the multiplier mult dev [k][F] float32 is divided by eta (at most hi) if
 * some solution s of cluster j (cluster dev [S] int32; with k = 1 every
 * solution, and cluster may be NULL) had element f accepted (accepted dev
 * [S][F] uint8, as dsm_accept writes it), else multiplied by eta (at least
 * lo).  Errors: DSM_ERR_ARG, DSM_ERR_DEVICE. */
dsm_status dsm_multiplier_step(int32_t k, int32_t F, int32_t S, const uint8_t* accepted, const int32_t* cluster,
                               float* mult, float eta, float lo, float hi, void* stream);

/* improved dev [S] uint8 is set to 1 where some entry of accepted dev [S][F]
 * (as dsm_accept writes it) is non-zero; other entries are left as they are
 * (clear it once per generation, then call once per class step). */
dsm_status dsm_mark_improved(int32_t S, int32_t F, const uint8_t* accepted, uint8_t* improved, void* stream);

/* Bytes of workspace for dsm_forced_replace (host function). */
size_t dsm_forced_work_bytes(const dsm_problem* p, int32_t S);

/* Forced improvements (RV-GOMEA, Sec. 2.2) at the end of a generation: a
 * solution's no-improvement stretch nis dev [S] int32 restarts at 0 if
 * improved dev [S] uint8 is set and grows by 1 otherwise; a solution with a
 * donor (donor dev [S] int32 >= 0, -1 = none) that accepted nothing takes the
 * donor's coordinates X dev [S][2][P][3], objectives obj dev [S][3] and term
 * cache dev [S][T][3] as they were before this call (chains of donors read
 * the old rows); every solution with a donor restarts its stretch.
 * n_replaced dev [1] int32 or NULL is increased by the number replaced.
 * work: dev, dsm_forced_work_bytes(p, S) bytes.  Errors: DSM_ERR_ARG,
 * DSM_ERR_DEVICE. */
dsm_status dsm_forced_replace(dsm_problem* p, int32_t S, float* X, double* obj, double* cache, const int32_t* donor,
                              const uint8_t* improved, int32_t* nis, void* work, int32_t* n_replaced, void* stream);

/* RV-GOMEA's anticipated mean shift (Sec. 2.2 builds on RV-GOMEA; the
 * samplers add 2 c times it for half of the population): shift dev [n]
 * float64 = mean - prev, then prev dev [n] = mean (mean dev [n], e.g. the
 * selection's point means [P][6] of dsm_estimate_distributions); with
 * has_prev = 0 (first generation) only prev = mean, and shift may be NULL.
 * Errors: DSM_ERR_ARG, DSM_ERR_DEVICE. */
dsm_status dsm_ams_shift(int32_t n, const double* mean, double* prev, double* shift, int32_t has_prev, void* stream);

/* MO-RV-GOMEA's single-objective clusters (the optimiser Sec. 2.2 builds
 * on): of k clusters with objective means means dev [k][3] float64 (as
 * dsm_cluster_objectives writes them), objective o = 0, 1, 2 (while o < k)
 * takes the cluster, not yet taken, with the lowest mean in o (the lowest
 * index among equal means; a NaN mean is never lower).  so dev [S] int32
 * receives the objective of solution s's cluster assign dev [S] int32, or -1.
 * Errors: DSM_ERR_ARG (k outside [1, 16]), DSM_ERR_DEVICE. */
dsm_status dsm_single_objective_clusters(int32_t k, const double* means, int32_t S, const int32_t* assign, int32_t* so,
                                         void* stream);

/* RV-GOMEA's forced-improvement donors: every solution whose no-improvement
 * stretch nis dev [S] int32 exceeds nis_max gets donor dev [S] int32 = the
 * entry at min(floor(u[s] n), n - 1) of the ascending list of the n solutions
 * that no member dominates (dominated_by == 0, dominated_by dev [S] int32 as
 * dsm_select writes it), u dev [S] float32 uniform draws in [0, 1) made by the
 * caller (computed in float32); all other solutions get -1.  n_forced dev [1]
 * int32 or NULL is increased by the number of donors given.  Errors:
 * DSM_ERR_ARG, DSM_ERR_CAPACITY (S > 8192), DSM_ERR_DEVICE. */
dsm_status dsm_draw_donors(int32_t S, const int32_t* nis, int32_t nis_max, const int32_t* dominated_by, const float* u,
                           int32_t* donor, int32_t* n_forced, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DSM_H */
