// C ABI of libdsm: argument validation, problem setup and launch sequencing.
// Every evaluation entry point validates host-visible arguments, then only
// enqueues kernels on the caller's stream (no synchronisation, no allocation).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dsm_internal.h"

using namespace dsm;


namespace {

thread_local std::string g_err;

dsm_status fail(dsm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

dsm_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? DSM_ERR_NOMEM : DSM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * count);
}

void release(dsm_problem* p) {
  if (!p) return;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  void* bufs[] = {p->d_img, p->d_raw, p->d_tets, p->d_tet_w, p->d_star_off, p->d_star, p->d_gpt, p->d_gcorr,
                  p->d_aff, p->d_aff_cnt, p->d_order, p->d_terms, p->d_simws, p->d_ident, p->d_cflags, p->d_ccount};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
}

// (Re)builds the bordered images for row pitch `pitch` (0 = default) and
// points the kernels' problem description at them.  Synchronous.
hipError_t repack(dsm_problem* p, int pitch) {
  const BorderedLayout bl = bordered_layout(p->dims[0], p->dims[1], p->dims[2], pitch);
  const size_t stride = 2 * (size_t)bl.elements();
  hipError_t e = hipSuccess;
  if (stride != p->img_stride) {
    if (p->d_img) (void)hipFree(p->d_img);
    p->d_img = nullptr;
    p->img_stride = 0;
    if ((e = dev_alloc(&p->d_img, 2 * stride)) != hipSuccess) return e;
  }
  p->img_stride = stride;
  for (int g = 0; g < 2; ++g)
    if ((e = launch_pack_bordered(p->d_raw + g * p->V, p->d_img + g * stride, p->dims[0], p->dims[1], p->dims[2], bl,
                                  nullptr)) != hipSuccess)
      return e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  p->pitch = bl.px;
  DevProblem& dv = p->dev;
  dv.img[0] = p->d_img;
  dv.img[1] = p->d_img + stride;
  dv.img_bytes = (int)(sizeof(float) * stride);
  dv.ex = bl.px;
  dv.exy = bl.px * bl.py;
  return hipSuccess;
}

// next free timing pair, or nulls
void timing_pair(dsm_problem* p, hipEvent_t& b, hipEvent_t& e) {
  b = e = nullptr;
  if (p->ev_used * 2 + 1 < (int)p->ev.size()) {
    b = p->ev[2 * p->ev_used];
    e = p->ev[2 * p->ev_used + 1];
    p->ev_used++;
  }
}

bool on_lattice(float x, int D, double& u) {
  if (!isfinite(x)) return false;
  u = ((double)x + 0.5) * kLat;
  return u == floor(u) && u >= 0.0 && u <= kLat * D;
}

}  // namespace

namespace dsm {
dsm_status set_error(dsm_status st, const char* msg) {
  g_err = msg ? msg : "";
  return st;
}
void clear_error() { g_err.clear(); }
}  // namespace dsm

extern "C" {

const char* dsm_status_string(dsm_status s) {
  switch (s) {
    case DSM_OK: return "ok";
    case DSM_ERR_ARG: return "invalid argument";
    case DSM_ERR_CAPACITY: return "capacity exceeded";
    case DSM_ERR_DOMAIN: return "geometry outside the supported domain";
    case DSM_ERR_DEVICE: return "device error";
    case DSM_ERR_NOMEM: return "out of device memory";
    case DSM_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* dsm_last_error(void) { return g_err.c_str(); }

dsm_status dsm_problem_create(const dsm_problem_desc* d, dsm_problem** out) {
  g_err.clear();
  if (!out) return fail(DSM_ERR_ARG, "out is null");
  *out = nullptr;
  if (!d) return fail(DSM_ERR_ARG, "desc is null");
  if (!d->moving || !d->fixed) return fail(DSM_ERR_ARG, "image pointer is null");
  for (int a = 0; a < 3; ++a) {
    if (d->dims[a] < 2 || d->dims[a] > 512)
      return fail(DSM_ERR_DOMAIN, "dims[%d] = %d outside [2, 512] (exact lattice predicates need 128*D <= 2^16)", a,
                  d->dims[a]);
    if (d->mesh[a] < 2 || d->mesh[a] > 129) return fail(DSM_ERR_DOMAIN, "mesh[%d] = %d outside [2, 129]", a, d->mesh[a]);
    if (!(d->spacing_mm[a] > 0.0f) || !isfinite(d->spacing_mm[a]))
      return fail(DSM_ERR_ARG, "spacing_mm[%d] must be positive and finite", a);
  }
  if (!isfinite(d->empty_tau)) return fail(DSM_ERR_ARG, "empty_tau must be finite");
  if (d->n_guid_moving < 0 || d->n_guid_fixed < 0) return fail(DSM_ERR_ARG, "negative guidance count");
  if ((d->n_guid_moving > 0 && (!d->guid_moving || !d->corr_moving)) ||
      (d->n_guid_fixed > 0 && (!d->guid_fixed || !d->corr_fixed)))
    return fail(DSM_ERR_ARG, "guidance pointer is null");
  if (d->max_solutions < 1 || d->max_fos < 0 || d->max_fos_points < 0)
    return fail(DSM_ERR_ARG, "capacities must be max_solutions >= 1, max_fos >= 0, max_fos_points >= 0");
  if (d->max_fos > 0 && d->max_fos_points < 1) return fail(DSM_ERR_ARG, "max_fos_points must be >= 1 when max_fos > 0");

  auto* p = new dsm_problem();
  for (int a = 0; a < 3; ++a) {
    p->dims[a] = d->dims[a];
    p->mesh[a] = d->mesh[a];
  }
  if (!build_topology(p->mesh, p->topo)) {
    release(p);
    return fail(DSM_ERR_ARG, "bad mesh");
  }
  p->V = (int64_t)d->dims[0] * d->dims[1] * d->dims[2];
  p->max_S = d->max_solutions;
  p->max_F = d->max_fos;
  p->max_pts = d->max_fos_points;
  p->maxA = std::max(1, std::min(p->topo.T, std::max(1, p->max_pts) * p->topo.max_star));
  p->identity.resize(3 * (size_t)p->topo.P);
  identity_grid(p->mesh, p->dims, p->identity.data());

  // guidance points: lattice integers, within the voxel-centre range [0, D-1]
  const int ng[2] = {d->n_guid_moving, d->n_guid_fixed};
  const float* gsrc[2] = {d->guid_moving, d->guid_fixed};
  const int32_t* csrc[2] = {d->corr_moving, d->corr_fixed};
  std::vector<double> gl;
  std::vector<int> gc;
  for (int g = 0; g < 2; ++g)
    for (int i = 0; i < ng[g]; ++i) {
      for (int a = 0; a < 3; ++a) {
        double u;
        const float x = gsrc[g][3 * (size_t)i + a];
        if (!on_lattice(x, d->dims[a], u) || x < 0.0f || x > (float)(d->dims[a] - 1)) {
          release(p);
          return fail(DSM_ERR_DOMAIN, "guidance point %d of image %d is off the lattice or outside [0, D-1]", i, g);
        }
        gl.push_back(u);
      }
      gc.push_back(csrc[g][i]);
    }
  // every correspondence must have a point on both images
  for (int g = 0; g < 2; ++g)
    for (int i = 0; i < ng[g]; ++i) {
      const int c = csrc[g][i];
      bool found = false;
      for (int j = 0; j < ng[1 - g] && !found; ++j) found = csrc[1 - g][j] == c;
      if (!found) {
        release(p);
        return fail(DSM_ERR_ARG, "correspondence %d has points on one image only", c);
      }
    }

  hipError_t e;
  if ((e = hipGetDevice(&p->device)) != hipSuccess) {
    release(p);
    return hip_fail(e, "hipGetDevice");
  }
  const HostTopology& tp = p->topo;
#define DSM_TRY(expr, what)  \
  if ((e = (expr)) != hipSuccess) { \
    release(p);              \
    return hip_fail(e, what); \
  }
  // images as given, then packed on the device into the bordered z-pair layout
  DSM_TRY(dev_alloc(&p->d_raw, 2 * (size_t)p->V), "hipMalloc images");
  DSM_TRY(hipMemcpy(p->d_raw, d->moving, sizeof(float) * p->V, hipMemcpyHostToDevice), "copy images");
  DSM_TRY(hipMemcpy(p->d_raw + p->V, d->fixed, sizeof(float) * p->V, hipMemcpyHostToDevice), "copy images");
  DSM_TRY(repack(p, 0), "pack images");
  DSM_TRY(dev_alloc(&p->d_tets, tp.tets.size()), "hipMalloc tets");
  DSM_TRY(hipMemcpy(p->d_tets, tp.tets.data(), sizeof(int) * tp.tets.size(), hipMemcpyHostToDevice), "copy tets");
  DSM_TRY(dev_alloc(&p->d_tet_w, tp.tet_w.size()), "hipMalloc weights");
  DSM_TRY(hipMemcpy(p->d_tet_w, tp.tet_w.data(), sizeof(double) * tp.tet_w.size(), hipMemcpyHostToDevice), "copy weights");
  DSM_TRY(dev_alloc(&p->d_star_off, tp.star_off.size()), "hipMalloc star_off");
  DSM_TRY(hipMemcpy(p->d_star_off, tp.star_off.data(), sizeof(int) * tp.star_off.size(), hipMemcpyHostToDevice),
          "copy star_off");
  DSM_TRY(dev_alloc(&p->d_star, tp.star.size()), "hipMalloc star");
  DSM_TRY(hipMemcpy(p->d_star, tp.star.data(), sizeof(int) * tp.star.size(), hipMemcpyHostToDevice), "copy star");
  DSM_TRY(dev_alloc(&p->d_gpt, gl.size()), "hipMalloc guidance");
  if (!gl.empty())
    DSM_TRY(hipMemcpy(p->d_gpt, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice), "copy guidance");
  DSM_TRY(dev_alloc(&p->d_gcorr, gc.size()), "hipMalloc correspondences");
  if (!gc.empty())
    DSM_TRY(hipMemcpy(p->d_gcorr, gc.data(), sizeof(int) * gc.size(), hipMemcpyHostToDevice), "copy correspondences");
  DSM_TRY(dev_alloc(&p->d_aff, (size_t)std::max(1, p->max_F) * p->maxA), "hipMalloc affected sets");
  DSM_TRY(dev_alloc(&p->d_aff_cnt, (size_t)std::max(1, p->max_F)), "hipMalloc affected counts");
  DSM_TRY(dev_alloc(&p->d_order, (size_t)std::max(1, p->max_F)), "hipMalloc element order");
  DSM_TRY(dev_alloc(&p->d_terms, (size_t)p->max_S * tp.T * 3), "hipMalloc term workspace");
  DSM_TRY(dev_alloc(&p->d_ident, p->identity.size()), "hipMalloc undeformed grid");
  DSM_TRY(hipMemcpy(p->d_ident, p->identity.data(), sizeof(float) * p->identity.size(), hipMemcpyHostToDevice),
          "copy undeformed grid");
  {
    const size_t full_groups = (size_t)(tp.T + kFullChunk - 1) / kFullChunk;
    p->simws_len = std::max((size_t)p->max_S * std::max(1, p->max_F) * 2 * p->maxA,
                            (size_t)p->max_S * full_groups * kFullChunk);
  }
  DSM_TRY(dev_alloc(&p->d_simws, p->simws_len), "hipMalloc sweep workspace");
  p->nchunk = (p->maxA + p->part_chunk - 1) / p->part_chunk;
  {
    const size_t nc = (size_t)p->max_S * std::max(1, p->max_F) * ((p->maxA + kMinPartChunk - 1) / kMinPartChunk);
    DSM_TRY(dev_alloc(&p->d_cflags, nc), "hipMalloc chunk flags");
    DSM_TRY(dev_alloc(&p->d_ccount, nc), "hipMalloc chunk counts");
  }
#undef DSM_TRY

  DevProblem& dv = p->dev;
  for (int a = 0; a < 3; ++a) {
    dv.D[a] = p->dims[a];
    dv.n[a] = p->mesh[a];
    dv.sp[a] = d->spacing_mm[a];
  }
  dv.DxDy = p->dims[0] * p->dims[1];
  dv.tau = d->empty_tau;
  dv.P = tp.P;
  dv.T = tp.T;
  dv.tets = (const int4*)p->d_tets;
  dv.tet_w = p->d_tet_w;
  dv.star_off = p->d_star_off;
  dv.star = p->d_star;
  dv.ng[0] = ng[0];
  dv.ng[1] = ng[1];
  dv.gpt[0] = p->d_gpt;
  dv.gpt[1] = p->d_gpt + 3 * (size_t)ng[0];
  dv.gcorr[0] = p->d_gcorr;
  dv.gcorr[1] = p->d_gcorr + ng[0];
  dv.norm[0] = 1.0 / (2.0 * (double)p->V);
  dv.norm[1] = 1.0 / (double)(tp.E + 4 * tp.T);
  dv.norm[2] = (ng[0] + ng[1]) > 0 ? 1.0 / (double)(ng[0] + ng[1]) : 0.0;

  // the evaluation kernel's dynamic LDS must fit one workgroup
  const size_t lds = eval_lds_bytes(kMaxChunk, 2);
  if (lds > 64 * 1024) {
    release(p);
    return fail(DSM_ERR_CAPACITY, "max_fos_points too large: affected set of %d tetrahedra needs %zu B of LDS", p->maxA,
                lds);
  }
  *out = p;
  return DSM_OK;
}

dsm_status dsm_problem_destroy(dsm_problem* p) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "problem is null");
  release(p);
  return DSM_OK;
}

dsm_status dsm_problem_query(const dsm_problem* p, dsm_problem_info* out) {
  g_err.clear();
  if (!p || !out) return fail(DSM_ERR_ARG, "null argument");
  out->P = p->topo.P;
  out->T = p->topo.T;
  out->E = p->topo.E;
  out->max_star = p->topo.max_star;
  out->V = p->V;
  out->max_affected = p->maxA;
  for (int c = 0; c < 3; ++c) out->norm[c] = p->dev.norm[c];
  out->pitch = p->pitch;
  return DSM_OK;
}

dsm_status dsm_problem_set_pitch(dsm_problem* p, int32_t pitch) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "problem is null");
  if (pitch != 0 && !pitch_ok(p->dims[0], p->dims[1], p->dims[2], pitch))
    return fail(DSM_ERR_ARG, "pitch %d outside [Dx + 2, 4 (Dx + 2) + 64] or image above 2 GiB", pitch);
  const hipError_t e = repack(p, pitch);
  return e == hipSuccess ? DSM_OK : hip_fail(e, "re-pack images");
}

dsm_status dsm_problem_topology(const dsm_problem* p, int32_t* tets, int32_t* star_off, int32_t* star,
                                float* identity) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "problem is null");
  if (tets) memcpy(tets, p->topo.tets.data(), sizeof(int) * p->topo.tets.size());
  if (star_off) memcpy(star_off, p->topo.star_off.data(), sizeof(int) * p->topo.star_off.size());
  if (star) memcpy(star, p->topo.star.data(), sizeof(int) * p->topo.star.size());
  if (identity) memcpy(identity, p->identity.data(), sizeof(float) * p->identity.size());
  return DSM_OK;
}

dsm_status dsm_mesh_topology(const int32_t mesh[3], const int32_t dims[3], int32_t* counts, int32_t* tets,
                             int32_t* star_off, int32_t* star, float* identity) {
  g_err.clear();
  if (!mesh) return fail(DSM_ERR_ARG, "mesh is null");
  const int m[3] = {mesh[0], mesh[1], mesh[2]};
  for (int a = 0; a < 3; ++a)
    if (m[a] < 2 || m[a] > 129) return fail(DSM_ERR_DOMAIN, "mesh[%d] = %d outside [2, 129]", a, m[a]);
  HostTopology tp;
  if (!build_topology(m, tp)) return fail(DSM_ERR_ARG, "bad mesh");
  if (counts) {
    counts[0] = tp.P;
    counts[1] = tp.T;
    counts[2] = tp.E;
    counts[3] = tp.max_star;
  }
  if (tets) memcpy(tets, tp.tets.data(), sizeof(int) * tp.tets.size());
  if (star_off) memcpy(star_off, tp.star_off.data(), sizeof(int) * tp.star_off.size());
  if (star) memcpy(star, tp.star.data(), sizeof(int) * tp.star.size());
  if (identity) {
    if (!dims) return fail(DSM_ERR_ARG, "dims is null");
    const int d[3] = {dims[0], dims[1], dims[2]};
    for (int a = 0; a < 3; ++a)
      if (d[a] < 2 || d[a] > 512) return fail(DSM_ERR_DOMAIN, "dims[%d] = %d outside [2, 512]", a, d[a]);
    identity_grid(m, d, identity);
  }
  return DSM_OK;
}

dsm_status dsm_fold_check(dsm_problem* p, int32_t S, const float* X, uint32_t* flags, int32_t* first_bad_tet,
                          void* stream) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "null argument");
  if (S < 0) return fail(DSM_ERR_ARG, "S < 0");
  if (S == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !flags) return fail(DSM_ERR_ARG, "null argument");
  const hipError_t e = launch_fold(p->dev, S, X, flags, first_bad_tet, (hipStream_t)stream);
  return e == hipSuccess ? DSM_OK : hip_fail(e, "fold check launch");
}

dsm_status dsm_eval_full(dsm_problem* p, int32_t S, const float* X, double* obj, uint32_t* flags, double* tet_terms,
                         void* stream) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "null argument");
  if (S < 0) return fail(DSM_ERR_ARG, "S < 0");
  if (S == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !obj || !flags) return fail(DSM_ERR_ARG, "null argument");
  if (S > p->max_S) return fail(DSM_ERR_CAPACITY, "S = %d exceeds max_solutions = %d", S, p->max_S);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_fold(p->dev, S, X, flags, nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "fold check launch");
  EvalArgs a{};
  a.pr = p->dev;
  a.S = S;
  a.G = (p->topo.T + kFullChunk - 1) / kFullChunk;
  a.partial = 0;
  a.X = X;
  a.maxA = kFullChunk;
  a.nver = 1;
  a.terms_out = tet_terms ? tet_terms : p->d_terms;
  a.simws = p->d_simws;
  a.row_pairs = p->row_order;
  hipEvent_t eb, ee;
  timing_pair(p, eb, ee);
  if ((e = launch_eval(a, eb, ee, st)) != hipSuccess) return hip_fail(e, "evaluation launch");
  if ((e = launch_full_reduce(p->dev, S, a.terms_out, obj, st)) != hipSuccess) return hip_fail(e, "reduce launch");
  return DSM_OK;
}

dsm_status dsm_eval_partial_masked(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                   const int32_t* fos_pts, const float* cand, const uint8_t* mask,
                                   const double* tet_terms_in, double* part_old,
                            double* part_new, uint32_t* flags, double* tet_terms_new, uint32_t* voxel_count,
                            void* stream) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "null argument");
  if (S < 0 || F < 0) return fail(DSM_ERR_ARG, "negative S or F");
  if (S > p->max_S) return fail(DSM_ERR_CAPACITY, "S = %d exceeds max_solutions = %d", S, p->max_S);
  if (F > p->max_F) return fail(DSM_ERR_CAPACITY, "F = %d exceeds max_fos = %d", F, p->max_F);
  if (S == 0 || F == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_off || !fos_pts || !cand || !part_old || !part_new || !flags)
    return fail(DSM_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_affected(p->dev, F, fos_off, fos_pts, p->max_pts, p->maxA, p->d_aff, p->d_aff_cnt, st);
  if (e == hipSuccess && F <= kOrderMax) e = launch_order(F, p->d_aff_cnt, p->d_order, st);
  if (e != hipSuccess) return hip_fail(e, "affected-set launch");
  EvalArgs a{};
  a.pr = p->dev;
  a.S = S;
  a.G = F;
  a.partial = 1;
  a.X = X;
  a.fos_off = fos_off;
  a.fos_pts = fos_pts;
  a.cand = cand;
  a.aff = p->d_aff;
  a.aff_cnt = p->d_aff_cnt;
  a.order = F <= kOrderMax ? p->d_order : nullptr;
  a.maxA = p->maxA;
  a.nver = tet_terms_in ? 1 : 2;
  a.terms_in = tet_terms_in;
  a.part_old = part_old;
  a.part_new = part_new;
  a.flags = flags;
  a.terms_out = tet_terms_new;
  a.vcount = voxel_count;
  a.mask = mask;
  a.simws = p->d_simws;
  a.pchunk = p->part_chunk;
  a.row_pairs = p->row_order;
  a.nchunk = p->nchunk;
  a.cflags = p->d_cflags;
  a.ccount = p->d_ccount;
  hipEvent_t eb, ee;
  timing_pair(p, eb, ee);
  if ((e = launch_eval(a, eb, ee, st)) != hipSuccess) return hip_fail(e, "evaluation launch");
  return DSM_OK;
}

dsm_status dsm_eval_partial(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                            const int32_t* fos_pts, const float* cand, const double* tet_terms_in, double* part_old,
                            double* part_new, uint32_t* flags, double* tet_terms_new, uint32_t* voxel_count,
                            void* stream) {
  return dsm_eval_partial_masked(p, S, X, F, fos_off, fos_pts, cand, nullptr, tet_terms_in, part_old, part_new, flags,
                                 tet_terms_new, voxel_count, stream);
}

}  // extern "C"

namespace {
// Shared driver of the setup-time autotuners: for each candidate k, apply(k)
// changes one setting of p, then the partial evaluation runs twice on the null
// stream and the second run is timed; the fastest candidate is applied again
// at the end and returned in *best_k (an index into the candidates).
template <class Apply>
dsm_status autotune(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                    const int32_t* fos_pts, const float* cand, const double* tet_terms_in, int n, Apply apply,
                    float* ms_out, int* best_k) {
  double *old = nullptr, *nw = nullptr;
  uint32_t* fl = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  dsm_status st = DSM_OK;
  float best_ms = INFINITY;
  int best = -1;
  if ((e = dev_alloc(&old, (size_t)S * F * 3)) != hipSuccess || (e = dev_alloc(&nw, (size_t)S * F * 3)) != hipSuccess ||
      (e = dev_alloc(&fl, (size_t)S * F)) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
      (e = hipEventCreate(&e1)) != hipSuccess) {
    st = hip_fail(e, "autotune buffers");
  }
  for (int k = 0; st == DSM_OK && k < n; ++k) {
    if ((st = apply(k)) != DSM_OK) break;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == DSM_OK; ++rep) {  // the first run warms caches and code
      (void)hipEventRecord(e0, nullptr);
      st = dsm_eval_partial(p, S, X, F, fos_off, fos_pts, cand, tet_terms_in, old, nw, fl, nullptr, nullptr, nullptr);
      (void)hipEventRecord(e1, nullptr);
      if (st == DSM_OK && (e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "autotune run");
      if (st == DSM_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    }
    if (st != DSM_OK) break;
    if (ms_out) ms_out[k] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = k;
    }
  }
  if (st == DSM_OK && best >= 0) st = apply(best);
  if (st == DSM_OK) *best_k = best;
  if (old) (void)hipFree(old);
  if (nw) (void)hipFree(nw);
  if (fl) (void)hipFree(fl);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}
}  // namespace

extern "C" {

dsm_status dsm_autotune_pitch(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                              const int32_t* fos_pts, const float* cand, const double* tet_terms_in, int32_t n_pitch,
                              const int32_t* pitches, float* ms_out, int32_t* best) {
  g_err.clear();
  if (!p || !X || !fos_off || !fos_pts || !cand || n_pitch < 0 || (n_pitch > 0 && !pitches)) return fail(DSM_ERR_ARG, "null argument");
  if (S <= 0 || F <= 0) return fail(DSM_ERR_ARG, "S and F must be positive");
  std::vector<int> cands;
  if (n_pitch > 0) {
    cands.assign(pitches, pitches + n_pitch);
  } else {  // default candidates: the default pitch and the next pitches of each class mod 16 elements
    const int d0 = default_pitch(p->dims[0]);
    for (int k : {0, 4, 8, 16, 24, 56}) cands.push_back(d0 + k);
  }
  for (int c : cands)
    if (c != 0 && !pitch_ok(p->dims[0], p->dims[1], p->dims[2], c)) return fail(DSM_ERR_ARG, "pitch %d not accepted", c);
  int k = -1;
  const dsm_status st = autotune(p, S, X, F, fos_off, fos_pts, cand, tet_terms_in, (int)cands.size(), [&](int i) {
    const hipError_t e = repack(p, cands[i]);
    return e == hipSuccess ? DSM_OK : hip_fail(e, "re-pack images");
  }, ms_out, &k);
  if (st == DSM_OK && best) *best = p->pitch;
  return st;
}

dsm_status dsm_set_part_chunk(dsm_problem* p, int32_t chunk) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "null argument");
  if (chunk < kMinPartChunk || chunk > kMaxPartChunk)
    return fail(DSM_ERR_ARG, "chunk %d outside [%d, %d]", chunk, kMinPartChunk, kMaxPartChunk);
  p->part_chunk = chunk;
  p->nchunk = (p->maxA + chunk - 1) / chunk;
  return DSM_OK;
}

int32_t dsm_get_part_chunk(const dsm_problem* p) { return p ? p->part_chunk : 0; }

dsm_status dsm_autotune_chunk(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                              const int32_t* fos_pts, const float* cand, const double* tet_terms_in, int32_t n_chunk,
                              const int32_t* chunks, float* ms_out, int32_t* best) {
  g_err.clear();
  if (!p || !X || !fos_off || !fos_pts || !cand || n_chunk < 0 || (n_chunk > 0 && !chunks)) return fail(DSM_ERR_ARG, "null argument");
  if (S <= 0 || F <= 0) return fail(DSM_ERR_ARG, "S and F must be positive");
  std::vector<int> cands;
  if (n_chunk > 0)
    cands.assign(chunks, chunks + n_chunk);
  else
    for (int c = kMinPartChunk; c <= kMaxPartChunk; ++c) cands.push_back(c);
  for (int c : cands)
    if (c < kMinPartChunk || c > kMaxPartChunk) return fail(DSM_ERR_ARG, "chunk %d outside [%d, %d]", c, kMinPartChunk, kMaxPartChunk);
  int k = -1;
  const dsm_status st = autotune(p, S, X, F, fos_off, fos_pts, cand, tet_terms_in, (int)cands.size(),
                                 [&](int i) { return dsm_set_part_chunk(p, cands[i]); }, ms_out, &k);
  if (st == DSM_OK && best) *best = p->part_chunk;
  return st;
}

dsm_status dsm_set_row_order(dsm_problem* p, int32_t order) {
  g_err.clear();
  if (!p) return fail(DSM_ERR_ARG, "null argument");
  if (order != DSM_ROWS_BY_SLICE && order != DSM_ROWS_BY_SLICE_PAIR) return fail(DSM_ERR_ARG, "row order %d unknown", order);
  p->row_order = order;
  return DSM_OK;
}

int32_t dsm_get_row_order(const dsm_problem* p) { return p ? p->row_order : -1; }

dsm_status dsm_autotune_row_order(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                  const int32_t* fos_pts, const float* cand, const double* tet_terms_in,
                                  float* ms_out, int32_t* best) {
  g_err.clear();
  if (!p || !X || !fos_off || !fos_pts || !cand) return fail(DSM_ERR_ARG, "null argument");
  if (S <= 0 || F <= 0) return fail(DSM_ERR_ARG, "S and F must be positive");
  const int orders[2] = {DSM_ROWS_BY_SLICE, DSM_ROWS_BY_SLICE_PAIR};
  int k = -1;
  const dsm_status st = autotune(p, S, X, F, fos_off, fos_pts, cand, tet_terms_in, 2,
                                 [&](int i) { return dsm_set_row_order(p, orders[i]); }, ms_out, &k);
  if (st == DSM_OK && best) *best = p->row_order;
  return st;
}

}  // extern "C"

// What the affected-set and ordering launches of one stored job need.
struct BatchSetJob {
  DevProblem pr;
  int F, max_pts, maxA;
  const int* fos_off;
  const int* fos_pts;
  int* aff;
  int* aff_cnt;
  int* order;  // null: no ordering launch
};

struct dsm_batch {
  int max_jobs = 0;
  EvalArgs* d_jobs = nullptr;
  int* d_off = nullptr;
  EvalArgs* h_jobs = nullptr;  // pinned staging
  int* h_off = nullptr;
  hipEvent_t copied = nullptr;
  bool pending = false;
  // configuration stored by dsm_batch_set_jobs
  EvalArgs* d_set_jobs = nullptr;
  int* d_set_off = nullptr;
  std::vector<BatchSetJob> set;
  int set_n = 0, set_per_xcd = 0, set_total_finish = 0, set_rows = 0;
  size_t set_lds = 0;
};

namespace {

// Row orders of a batch's jobs for launch_eval_batch: 0 all by slice, 1 all
// by slice pair, 2 both.
int batch_rows(const std::vector<EvalArgs>& args) {
  bool by_slice = false, by_pair = false;
  for (const EvalArgs& a : args)
    if (a.S > 0 && a.G > 0) (a.row_pairs ? by_pair : by_slice) = true;
  return by_slice && by_pair ? 2 : (by_pair ? 1 : 0);
}

// Validates the jobs and fills their evaluation arguments, the per-XCD slot
// offsets of the sweep (a job of n workgroups takes ceil(n / 8) slots on each
// of the 8 XCDs) and the workgroup offsets of the finishing kernel.
dsm_status batch_tables(const dsm_batch* b, int n_jobs, const dsm_partial_job* jobs, std::vector<EvalArgs>& args,
                        std::vector<int>& off, std::vector<int>& foff, size_t& lds) {
  if (!b || (n_jobs > 0 && !jobs) || n_jobs < 0) return fail(DSM_ERR_ARG, "null argument");
  if (n_jobs > b->max_jobs) return fail(DSM_ERR_CAPACITY, "n_jobs = %d exceeds max_jobs = %d", n_jobs, b->max_jobs);
  args.assign(n_jobs, EvalArgs{});
  off.assign(n_jobs + 1, 0);
  foff.assign(n_jobs + 1, 0);
  lds = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const dsm_partial_job& q = jobs[j];
    dsm_problem* p = q.problem;
    if (!p || !q.X || !q.fos_off || !q.fos_pts || !q.cand || !q.part_old || !q.part_new || !q.flags)
      return fail(DSM_ERR_ARG, "job %d: null argument", j);
    for (int k = 0; k < j; ++k)
      if (jobs[k].problem == p) return fail(DSM_ERR_ARG, "job %d repeats the problem of job %d", j, k);
    if (q.S < 0 || q.F < 0) return fail(DSM_ERR_ARG, "job %d: negative S or F", j);
    if (q.S > p->max_S || q.F > p->max_F) return fail(DSM_ERR_CAPACITY, "job %d: S or F above the problem's capacity", j);
    EvalArgs& a = args[j];
    a.pr = p->dev;
    a.S = q.S;
    a.G = q.F;
    a.partial = 1;
    a.X = q.X;
    a.fos_off = q.fos_off;
    a.fos_pts = q.fos_pts;
    a.cand = q.cand;
    a.aff = p->d_aff;
    a.aff_cnt = p->d_aff_cnt;
    a.order = q.F <= kOrderMax ? p->d_order : nullptr;
    a.maxA = p->maxA;
    a.nver = q.tet_terms_in ? 1 : 2;
    a.terms_in = q.tet_terms_in;
    a.part_old = q.part_old;
    a.part_new = q.part_new;
    a.flags = q.flags;
    a.terms_out = q.tet_terms_new;
    a.vcount = q.voxel_count;
    a.mask = q.mask;
    a.simws = p->d_simws;
    a.pchunk = p->part_chunk;
    a.row_pairs = p->row_order;
    a.nchunk = p->nchunk;
    a.cflags = p->d_cflags;
    a.ccount = p->d_ccount;
    off[j + 1] = off[j] + (q.S * q.F * a.nchunk + 7) / 8;
    foff[j + 1] = foff[j] + (q.S * q.F + kFinishPairs - 1) / kFinishPairs;
    lds = std::max(lds, eval_lds_bytes(kMaxChunk, a.nver));
  }
  return DSM_OK;
}

}  // namespace

extern "C" {

dsm_status dsm_batch_create(int32_t max_jobs, dsm_batch** out) {
  g_err.clear();
  if (!out || max_jobs < 1) return fail(DSM_ERR_ARG, "null out or max_jobs < 1");
  *out = nullptr;
  auto* b = new dsm_batch();
  b->max_jobs = max_jobs;
  hipError_t e = hipMalloc((void**)&b->d_jobs, sizeof(EvalArgs) * max_jobs);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_off, sizeof(int) * 2 * (max_jobs + 1));
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_jobs, sizeof(EvalArgs) * max_jobs, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_off, sizeof(int) * 2 * (max_jobs + 1), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
  if (e != hipSuccess) {
    dsm_batch_destroy(b);
    return hip_fail(e, "batch allocation");
  }
  *out = b;
  return DSM_OK;
}

dsm_status dsm_batch_destroy(dsm_batch* b) {
  g_err.clear();
  if (!b) return fail(DSM_ERR_ARG, "null batch");
  if (b->pending && b->copied) (void)hipEventSynchronize(b->copied);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_off) (void)hipFree(b->d_off);
  if (b->h_jobs) (void)hipHostFree(b->h_jobs);
  if (b->h_off) (void)hipHostFree(b->h_off);
  if (b->copied) (void)hipEventDestroy(b->copied);
  if (b->d_set_jobs) (void)hipFree(b->d_set_jobs);
  if (b->d_set_off) (void)hipFree(b->d_set_off);
  delete b;
  return DSM_OK;
}

dsm_status dsm_eval_partial_batch(dsm_batch* b, int32_t n_jobs, const dsm_partial_job* jobs, void* stream) {
  g_err.clear();
  std::vector<EvalArgs> args;
  std::vector<int> off, foff;
  size_t lds = 0;
  const dsm_status vs = batch_tables(b, n_jobs, jobs, args, off, foff, lds);
  if (vs != DSM_OK) return vs;
  if (n_jobs == 0 || off[n_jobs] == 0) return DSM_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int j = 0; j < n_jobs && e == hipSuccess; ++j)
    if (jobs[j].S > 0 && jobs[j].F > 0) {
      e = launch_affected(args[j].pr, jobs[j].F, jobs[j].fos_off, jobs[j].fos_pts, jobs[j].problem->max_pts,
                          args[j].maxA, args[j].aff ? jobs[j].problem->d_aff : nullptr, jobs[j].problem->d_aff_cnt, st);
      if (e == hipSuccess && args[j].order) e = launch_order(jobs[j].F, jobs[j].problem->d_aff_cnt, jobs[j].problem->d_order, st);
    }
  if (e != hipSuccess) return hip_fail(e, "affected-set launch");
  if (b->pending && (e = hipEventSynchronize(b->copied)) != hipSuccess) return hip_fail(e, "job table wait");
  memcpy(b->h_jobs, args.data(), sizeof(EvalArgs) * n_jobs);
  memcpy(b->h_off, off.data(), sizeof(int) * (n_jobs + 1));
  memcpy(b->h_off + (n_jobs + 1), foff.data(), sizeof(int) * (n_jobs + 1));
  e = hipMemcpyAsync(b->d_jobs, b->h_jobs, sizeof(EvalArgs) * n_jobs, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_off, b->h_off, sizeof(int) * 2 * (n_jobs + 1), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(b->copied, st);
  if (e != hipSuccess) return hip_fail(e, "job table copy");
  b->pending = true;
  if ((e = launch_eval_batch(b->d_jobs, b->d_off, n_jobs, off[n_jobs], foff[n_jobs], lds, batch_rows(args), st)) !=
      hipSuccess)
    return hip_fail(e, "batched evaluation launch");
  return DSM_OK;
}

dsm_status dsm_batch_set_jobs(dsm_batch* b, int32_t n_jobs, const dsm_partial_job* jobs) {
  g_err.clear();
  std::vector<EvalArgs> args;
  std::vector<int> off, foff;
  size_t lds = 0;
  const dsm_status vs = batch_tables(b, n_jobs, jobs, args, off, foff, lds);
  if (vs != DSM_OK) return vs;
  hipError_t e = hipSuccess;
  if (!b->d_set_jobs) {
    e = hipMalloc((void**)&b->d_set_jobs, sizeof(EvalArgs) * b->max_jobs);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_set_off, sizeof(int) * 2 * (b->max_jobs + 1));
    if (e != hipSuccess) return hip_fail(e, "batch configuration allocation");
  }
  // the previous configuration may still be in use by enqueued runs
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "device synchronisation");
  std::vector<int> both(off);
  both.insert(both.end(), foff.begin(), foff.end());
  if (n_jobs > 0) {
    e = hipMemcpy(b->d_set_jobs, args.data(), sizeof(EvalArgs) * n_jobs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_set_off, both.data(), sizeof(int) * both.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "job table copy");
  }
  b->set.clear();
  for (int j = 0; j < n_jobs; ++j) {
    const EvalArgs& a = args[j];
    if (a.S <= 0 || a.G <= 0) continue;
    dsm_problem* p = jobs[j].problem;
    b->set.push_back(BatchSetJob{a.pr, a.G, p->max_pts, a.maxA, a.fos_off, a.fos_pts, p->d_aff, p->d_aff_cnt,
                                 a.order ? p->d_order : nullptr});
  }
  b->set_per_xcd = n_jobs > 0 ? off[n_jobs] : 0;
  b->set_total_finish = n_jobs > 0 ? foff[n_jobs] : 0;
  b->set_lds = lds;
  b->set_rows = batch_rows(args);
  b->set_n = n_jobs;
  return DSM_OK;
}

dsm_status dsm_batch_run(dsm_batch* b, void* stream) {
  g_err.clear();
  if (!b) return fail(DSM_ERR_ARG, "null batch");
  if (b->set_per_xcd == 0) return DSM_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (const BatchSetJob& q : b->set) {
    e = launch_affected(q.pr, q.F, q.fos_off, q.fos_pts, q.max_pts, q.maxA, q.aff, q.aff_cnt, st);
    if (e == hipSuccess && q.order) e = launch_order(q.F, q.aff_cnt, q.order, st);
    if (e != hipSuccess) return hip_fail(e, "affected-set launch");
  }
  e = launch_eval_batch(b->d_set_jobs, b->d_set_off, b->set_n, b->set_per_xcd, b->set_total_finish, b->set_lds,
                        b->set_rows, st);
  return e == hipSuccess ? DSM_OK : hip_fail(e, "batched evaluation launch");
}

dsm_status dsm_problem_timing(dsm_problem* p, int32_t capacity) {
  g_err.clear();
  if (!p || capacity < 0) return fail(DSM_ERR_ARG, "null problem or negative capacity");
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->ev_used = 0;
  for (int i = 0; i < 2 * capacity; ++i) {
    hipEvent_t e;
    const hipError_t st = hipEventCreate(&e);
    if (st != hipSuccess) return hip_fail(st, "hipEventCreate");
    p->ev.push_back(e);
  }
  return DSM_OK;
}

dsm_status dsm_problem_timing_read(dsm_problem* p, float* ms, int32_t max_n, int32_t* n) {
  g_err.clear();
  if (!p || !n || (max_n > 0 && !ms) || max_n < 0) return fail(DSM_ERR_ARG, "null argument");
  const int k = std::min(p->ev_used, max_n);
  for (int i = 0; i < k; ++i) {
    hipError_t st = hipEventSynchronize(p->ev[2 * i + 1]);
    if (st == hipSuccess) st = hipEventElapsedTime(&ms[i], p->ev[2 * i], p->ev[2 * i + 1]);
    if (st != hipSuccess) return hip_fail(st, "timing events");
  }
  *n = k;
  p->ev_used = 0;
  return DSM_OK;
}

dsm_status dsm_transform(dsm_problem* p, int32_t own, const float* X, float* dvf, float* warped, void* stream) {
  g_err.clear();
  if (!p || !X) return fail(DSM_ERR_ARG, "null argument");
  if (own != 0 && own != 1) return fail(DSM_ERR_ARG, "own %d is not 0 or 1", own);
  const hipError_t e = launch_transform(p->dev, own, X, dvf, warped, (hipStream_t)stream);
  return e == hipSuccess ? DSM_OK : hip_fail(e, "transform launch");
}

dsm_status dsm_rasterize_owner(dsm_problem* p, const float* Xgrid, int32_t* owner, int32_t* overlap, void* stream) {
  g_err.clear();
  if (!p || !Xgrid || !owner || !overlap) return fail(DSM_ERR_ARG, "null argument");
  const hipError_t e = launch_owner(p->dev, Xgrid, owner, overlap, (hipStream_t)stream);
  return e == hipSuccess ? DSM_OK : hip_fail(e, "owner launch");
}

}  // extern "C"
