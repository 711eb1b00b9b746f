// Generation bookkeeping of the multi-objective optimiser on the device: the
// elitist archive (the approximation set of Sec. 2.4), the selection the
// distributions are estimated on, the adaptive multiplier step and the
// forced-improvement replacement (both from RV-GOMEA, which Sec. 2.2 builds
// on).  Every entry point only enqueues kernels: sizes that live on the device
// (the archive's row count) are read by the kernels, never by the host.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dsm_internal.h"

namespace dsm {
namespace {

constexpr int kMergeWG = 256;

__device__ __forceinline__ bool dominates3(const double* a, const double* b) {
  return a[0] <= b[0] && a[1] <= b[1] && a[2] <= b[2] && (a[0] < b[0] || a[1] < b[1] || a[2] < b[2]);
}
__device__ __forceinline__ bool equal3(const double* a, const double* b) {
  return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}
// a before b in lexicographic order
__device__ __forceinline__ bool lex_less(const double* a, const double* b) {
  return a[0] != b[0] ? a[0] < b[0] : (a[1] != b[1] ? a[1] < b[1] : a[2] < b[2]);
}

// Workspace of one merge (byte offsets, 256-aligned regions).
struct MergeWork {
  size_t keep_a, keep_n, pref_a, pos_a, pos_n, vec, rows, hdr, total;
};
__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
__host__ __device__ inline MergeWork merge_work(int cap, int m, int row_floats) {
  MergeWork w;
  size_t o = 0;
  w.keep_a = o;  // int [cap]: archive row kept
  o = al256(o + sizeof(int) * (size_t)cap);
  w.keep_n = o;  // int [m]: new point kept
  o = al256(o + sizeof(int) * (size_t)m);
  w.pref_a = o;  // int [cap + 1]: exclusive prefix of keep_a
  o = al256(o + sizeof(int) * ((size_t)cap + 1));
  w.pos_a = o;  // int [cap]: output position of archive row (-1 dropped)
  o = al256(o + sizeof(int) * (size_t)cap);
  w.pos_n = o;  // int [m]: output position of new point (-1 dropped)
  o = al256(o + sizeof(int) * (size_t)m);
  w.vec = o;  // double [cap][3]: merged vectors
  o = al256(o + sizeof(double) * 3 * (size_t)cap);
  w.rows = o;  // float [cap][row_floats]: merged payload
  o = al256(o + sizeof(float) * (size_t)cap * row_floats);
  w.hdr = o;  // int [2]: merged count, overflow
  o = al256(o + sizeof(int) * 2);
  w.total = o;
  return w;
}

// Archive row i (of n) is kept iff no new point dominates it (the archive's
// own rows are mutually non-dominated and distinct).
__global__ void k_merge_mark_archive(const double* __restrict__ arch, const int* __restrict__ n_arch, int cap, int m,
                                     const double* __restrict__ pts, int* __restrict__ keep_a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const int n = min(*n_arch, cap);
  int keep = 0;
  if (i < n) {
    keep = 1;
    const double* a = arch + 3 * (size_t)i;
    for (int j = 0; j < m && keep; ++j)
      if (dominates3(pts + 3 * (size_t)j, a)) keep = 0;
  }
  keep_a[i] = keep;
}

// New point j is kept iff no archive row dominates or equals it, no new point
// dominates it and no earlier new point equals it: one workgroup per point,
// its threads striding over the candidates.
__global__ __launch_bounds__(kMergeWG) void k_merge_mark_new(const double* __restrict__ arch,
                                                           const int* __restrict__ n_arch, int cap, int m,
                                                           const double* __restrict__ pts, int* __restrict__ keep_n) {
  __shared__ int drop;
  const int j = blockIdx.x, t = threadIdx.x;
  if (t == 0) drop = 0;
  __syncthreads();
  const int n = min(*n_arch, cap);
  const double* p = pts + 3 * (size_t)j;
  int d = 0;
  for (int i = t; i < n && !d; i += kMergeWG) {
    const double* a = arch + 3 * (size_t)i;
    d = dominates3(a, p) || equal3(a, p);
  }
  for (int k = t; k < m && !d; k += kMergeWG) {
    const double* q = pts + 3 * (size_t)k;
    d = dominates3(q, p) || (k < j && equal3(q, p));
  }
  if (d) atomicOr(&drop, 1);
  __syncthreads();
  if (t == 0) keep_n[j] = drop ? 0 : 1;
}

// Exclusive prefix of keep_a over [0, cap) by one workgroup.
__global__ __launch_bounds__(1024) void k_merge_prefix(const int* __restrict__ keep_a, int cap, int* __restrict__ pref_a) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (cap + 1023) / 1024;
  const int b = t * per, e = min(cap, b + per);
  int s = 0;
  for (int i = b; i < e; ++i) s += keep_a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = b; i < e; ++i) {
    pref_a[i] = run;
    run += keep_a[i];
  }
  if (t == 1023) pref_a[cap] = part[1023];
}

// Output positions: kept archive rows keep their order (they are sorted) and
// make room for the kept new points lexicographically below them; a kept new
// point goes after the kept archive rows and kept new points below it (the
// sorted archive is searched by bisection).  Kept vectors are distinct, so the
// positions are a permutation of [0, k).
__global__ void k_merge_positions(const double* __restrict__ arch, const int* __restrict__ n_arch, int cap, int m,
                                  const double* __restrict__ pts, const int* __restrict__ keep_a,
                                  const int* __restrict__ keep_n, const int* __restrict__ pref_a, int* __restrict__ pos_a,
                                  int* __restrict__ pos_n, int* __restrict__ hdr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = min(*n_arch, cap);
  if (e < cap) {
    int pos = -1;
    if (e < n && keep_a[e]) {
      const double* a = arch + 3 * (size_t)e;
      int below = 0;
      for (int j = 0; j < m; ++j) below += keep_n[j] && lex_less(pts + 3 * (size_t)j, a);
      pos = pref_a[e] + below;
    }
    pos_a[e] = pos;
  } else if (e < cap + m) {
    const int j = e - cap;
    int pos = -1;
    if (keep_n[j]) {
      const double* p = pts + 3 * (size_t)j;
      int lo = 0, hi = n;  // first archive row not below p
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lex_less(arch + 3 * (size_t)mid, p))
          lo = mid + 1;
        else
          hi = mid;
      }
      int below = pref_a[lo];
      for (int k = 0; k < m; ++k) below += keep_n[k] && lex_less(pts + 3 * (size_t)k, p);
      pos = below;
    }
    pos_n[j] = pos;
  } else if (e == cap + m) {
    int kn = 0;
    for (int j = 0; j < m; ++j) kn += keep_n[j];
    const int k = pref_a[cap] + kn;
    hdr[0] = k;
    hdr[1] = k > cap ? 1 : 0;
  }
}

// Scatter of the kept vectors and payload rows into the workspace, one thread
// per (source row, column); columns 0-2 are the vector, 3.. the payload.
__global__ void k_merge_scatter(const double* __restrict__ arch, const float* __restrict__ arch_rows, int cap, int m,
                                const double* __restrict__ pts, const float* __restrict__ pt_rows, int row_floats,
                                const int* __restrict__ pos_a, const int* __restrict__ pos_n,
                                const int* __restrict__ hdr, double* __restrict__ vec, float* __restrict__ rows) {
  if (hdr[1]) return;  // overflow: the archive stays as it was
  const int cols = 3 + row_floats;
  const int64_t total = (int64_t)(cap + m) * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e - (int64_t)r * cols);
    const int pos = r < cap ? pos_a[r] : pos_n[r - cap];
    if (pos < 0) continue;
    if (c < 3)
      vec[3 * (size_t)pos + c] = r < cap ? arch[3 * (size_t)r + c] : pts[3 * (size_t)(r - cap) + c];
    else
      rows[(size_t)pos * row_floats + (c - 3)] =
          r < cap ? arch_rows[(size_t)r * row_floats + (c - 3)] : pt_rows[(size_t)(r - cap) * row_floats + (c - 3)];
  }
}

// Copies the merged archive back: rows [0, k) from the workspace, +inf after;
// the count and the overflow flag.
__global__ void k_merge_copyback(double* __restrict__ arch, float* __restrict__ arch_rows, int cap, int row_floats,
                                 const double* __restrict__ vec, const float* __restrict__ rows,
                                 const int* __restrict__ hdr, int* __restrict__ n_arch, int* __restrict__ overflow) {
  const int k = hdr[0];
  const bool over = hdr[1] != 0;
  const int cols = 3 + row_floats;
  const int64_t total = (int64_t)cap * cols;
  const int64_t first = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (first == 0 && overflow) *overflow = over ? 1 : 0;
  if (over) return;
  for (int64_t e = first; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e - (int64_t)r * cols);
    if (c < 3)
      arch[3 * (size_t)r + c] = r < k ? vec[3 * (size_t)r + c] : INFINITY;
    else if (r < k)
      arch_rows[(size_t)r * row_floats + (c - 3)] = rows[(size_t)r * row_floats + (c - 3)];
  }
}

__global__ void k_merge_count(const int* __restrict__ hdr, int* __restrict__ n_arch) {
  if (threadIdx.x == 0 && !hdr[1]) *n_arch = hdr[0];
}

// Selection: one workgroup.  Range of every objective, dominated-by counts,
// keys count * 4 + normalised sum (the sum is below 4, so counts decide
// first), ranks by counting (ties by index), scatter of the first n_sel.
constexpr int kSelWG = 1024;
__global__ __launch_bounds__(kSelWG) void k_select(int S, const double* __restrict__ obj, int n_sel,
                                                   int* __restrict__ sel, int* __restrict__ dominated_by) {
  extern __shared__ double s_key[];  // [S]
  __shared__ double s_red[kSelWG / 64][6];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};  // lo xyz, hi xyz
  for (int i = t; i < S; i += kSelWG)
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], obj[3 * (size_t)i + c]);
      v[3 + c] = fmax(v[3 + c], obj[3 * (size_t)i + c]);
    }
  for (int off = 32; off >= 1; off >>= 1)
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], __shfl_xor(v[c], off, 64));
      v[3 + c] = fmax(v[3 + c], __shfl_xor(v[3 + c], off, 64));
    }
  if (lane == 0)
    for (int c = 0; c < 6; ++c) s_red[wave][c] = v[c];
  __syncthreads();
  double rl[3], range[3];
  for (int c = 0; c < 3; ++c) {
    double lo = s_red[0][c], hi = s_red[0][3 + c];
    for (int w = 1; w < kSelWG / 64; ++w) {
      lo = fmin(lo, s_red[w][c]);
      hi = fmax(hi, s_red[w][3 + c]);
    }
    rl[c] = lo;
    range[c] = fmax(hi - lo, 1e-300);
  }
  for (int i = t; i < S; i += kSelWG) {
    const double* o = obj + 3 * (size_t)i;
    int cnt = 0;
    for (int j = 0; j < S; ++j) cnt += dominates3(obj + 3 * (size_t)j, o);
    double nrm = 0.0;
    for (int c = 0; c < 3; ++c) nrm = nrm + (o[c] - rl[c]) / range[c];
    s_key[i] = (double)cnt * 4.0 + nrm;
    if (dominated_by) dominated_by[i] = cnt;
  }
  __syncthreads();
  for (int i = t; i < S; i += kSelWG) {
    const double k = s_key[i];
    int rank = 0;
    for (int j = 0; j < S; ++j) rank += s_key[j] < k || (s_key[j] == k && j < i);
    if (rank < n_sel) sel[rank] = i;
  }
}

// RV-GOMEA's anticipated mean shift: the change of the selection's point means
// since the previous generation; prev keeps the current means.
__global__ void k_ams_shift(int n, const double* __restrict__ mean, double* __restrict__ prev, double* __restrict__ shift,
                            int has_prev) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double m = mean[i];
    if (has_prev) shift[i] = m - prev[i];
    prev[i] = m;
  }
}

// MO-RV-GOMEA's single-objective clusters: objective o = 0, 1, 2 (while o < k)
// takes, of the clusters not yet taken, the one with the lowest mean in o (the
// lowest index among equal means); every solution gets its cluster's objective.
// Each workgroup derives the (at most kClusterMax) assignments itself.
__global__ void k_so_clusters(int k, const double* __restrict__ means, int S, const int* __restrict__ assign,
                              int* __restrict__ so) {
  __shared__ int of_cluster[kClusterMax];
  if (threadIdx.x == 0) {
    for (int j = 0; j < k; ++j) of_cluster[j] = -1;
    for (int o = 0; o < 3 && o < k; ++o) {
      int best = -1;
      double bv = 0.0;
      for (int j = 0; j < k; ++j)
        if (of_cluster[j] < 0 && (best < 0 || means[3 * j + o] < bv)) {
          best = j;
          bv = means[3 * j + o];
        }
      of_cluster[best] = o;  // o < k clusters are taken, so one is free
    }
  }
  __syncthreads();
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    const int a = assign[s];
    so[s] = a >= 0 && a < k ? of_cluster[a] : -1;
  }
}

// RV-GOMEA's forced-improvement donors, one workgroup: the solutions no member
// dominates, in ascending order (block-wide prefix), and every solution whose
// no-improvement stretch exceeds nis_max takes the list's entry at
// min(floor(u[s] n), n - 1).
__global__ __launch_bounds__(1024) void k_draw_donors(int S, const int* __restrict__ nis, int nis_max,
                                                      const int* __restrict__ dominated_by, const float* __restrict__ u,
                                                      int* __restrict__ donor, int* __restrict__ n_forced) {
  extern __shared__ int s_nd[];  // [S]
  __shared__ int part[1024];
  __shared__ int s_forced;
  const int t = threadIdx.x;
  const int per = (S + 1023) / 1024;
  const int b = min(S, t * per), e = min(S, b + per);
  int c = 0;
  for (int i = b; i < e; ++i) c += dominated_by[i] == 0;
  part[t] = c;
  if (t == 0) s_forced = 0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - c;
  for (int i = b; i < e; ++i)
    if (dominated_by[i] == 0) s_nd[run++] = i;
  const int n = part[1023];
  __syncthreads();
  int forced = 0;
  for (int s = t; s < S; s += 1024) {
    int d = -1;
    if (nis[s] > nis_max && n > 0) {
      d = s_nd[min(max((int)(u[s] * (float)n), 0), n - 1)];
      ++forced;
    }
    donor[s] = d;
  }
  if (forced) atomicAdd(&s_forced, forced);
  __syncthreads();
  if (t == 0 && n_forced) n_forced[0] += s_forced;
}

// AMaLGaM's adaptive variance scaling, one thread per distribution (float32).
__global__ void k_avs(int n, float* __restrict__ mult, int* __restrict__ nis, const double* __restrict__ sdr,
                      int nis_max, float eta, float lo, float hi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c = mult[i];
  const double r = sdr[i];
  float c1;
  int n1;
  if (r >= 0.0) {
    c1 = c < 1.f ? 1.f : c;
    if (r > 1.0) c1 = c1 / eta;
    n1 = 0;
  } else {
    n1 = c <= 1.f ? nis[i] + 1 : nis[i];
    c1 = c;
    if (c > 1.f || n1 >= nis_max) c1 = c * eta;
    if (c1 < 1.f && n1 < nis_max) c1 = 1.f;
  }
  mult[i] = fminf(fmaxf(c1, lo), hi);
  nis[i] = n1;
}

// The simple multiplier schedule: per (cluster j, element f), one thread
// scanning the solutions: a hit if a solution of cluster j (every solution
// without clusters) had element f accepted; the multiplier is divided by eta
// after a hit, else multiplied by it, within [lo, hi].
__global__ void k_multiplier_step(int k, int F, int S, const unsigned char* __restrict__ acc,
                                  const int* __restrict__ cluster, float* __restrict__ mult, float eta, float lo,
                                  float hi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * F) return;
  const int j = e / F, f = e - j * F;
  bool hit = false;
  for (int s = 0; s < S && !hit; ++s) hit = acc[(size_t)s * F + f] != 0 && (!cluster || cluster[s] == j);
  const float c = mult[e];
  mult[e] = hit ? fminf(c / eta, hi) : fmaxf(c * eta, lo);
}

// improved[s] |= some element of solution s was accepted.
__global__ void k_mark_improved(int S, int F, const unsigned char* __restrict__ acc, unsigned char* __restrict__ improved) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  unsigned char any = 0;
  for (int f = 0; f < F; ++f) any |= acc[(size_t)s * F + f];
  if (any) improved[s] = 1;
}

// Forced-improvement replacement, first pass: the donors' rows (coordinates,
// objectives, term cache) of the solutions to replace are staged, so that a
// donor replaced in the same step still gives its values from before it.
__global__ void k_forced_stage(int S, int row_x, int row_c, const float* __restrict__ X, const double* __restrict__ obj,
                               const double* __restrict__ cache, const int* __restrict__ donor,
                               const unsigned char* __restrict__ improved, float* __restrict__ wx,
                               double* __restrict__ wobj, double* __restrict__ wcache) {
  const int s = blockIdx.y;
  const int d = donor[s];
  if (d < 0 || d >= S || improved[s]) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < row_x + 3 + row_c; k += gridDim.x * blockDim.x) {
    if (k < row_x)
      wx[(size_t)s * row_x + k] = X[(size_t)d * row_x + k];
    else if (k < row_x + 3)
      wobj[3 * (size_t)s + (k - row_x)] = obj[3 * (size_t)d + (k - row_x)];
    else
      wcache[(size_t)s * row_c + (k - row_x - 3)] = cache[(size_t)d * row_c + (k - row_x - 3)];
  }
}

// Second pass: the staged rows are written; the stretches are updated.
__global__ void k_forced_apply(int S, int row_x, int row_c, float* __restrict__ X, double* __restrict__ obj,
                               double* __restrict__ cache, const int* __restrict__ donor,
                               const unsigned char* __restrict__ improved, const float* __restrict__ wx,
                               const double* __restrict__ wobj, const double* __restrict__ wcache,
                               int* __restrict__ nis, int* __restrict__ n_replaced) {
  const int s = blockIdx.y;
  const int d = donor[s];
  const bool replace = d >= 0 && d < S && !improved[s];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nis[s] = (improved[s] || d >= 0) ? 0 : nis[s] + 1;
    if (replace && n_replaced) atomicAdd(n_replaced, 1);
  }
  if (!replace) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < row_x + 3 + row_c; k += gridDim.x * blockDim.x) {
    if (k < row_x)
      X[(size_t)s * row_x + k] = wx[(size_t)s * row_x + k];
    else if (k < row_x + 3)
      obj[3 * (size_t)s + (k - row_x)] = wobj[3 * (size_t)s + (k - row_x)];
    else
      cache[(size_t)s * row_c + (k - row_x - 3)] = wcache[(size_t)s * row_c + (k - row_x - 3)];
  }
}

}  // namespace
}  // namespace dsm

using namespace dsm;

extern "C" {

size_t dsm_archive_work_bytes(int32_t capacity, int32_t m, int32_t row_floats) {
  if (capacity < 1 || m < 0 || row_floats < 0) return 0;
  return merge_work(capacity, m, row_floats).total;
}

dsm_status dsm_archive_merge(int32_t capacity, double* archive, int32_t* n_archive, int32_t m, const double* points,
                             int32_t row_floats, float* archive_rows, const float* point_rows, void* work,
                             int32_t* overflow, void* stream) {
  if (capacity < 1 || m < 0 || row_floats < 0) return DSM_ERR_ARG;
  if (!archive || !n_archive || !work || (m > 0 && !points)) return DSM_ERR_ARG;
  if (row_floats > 0 && (!archive_rows || (m > 0 && !point_rows))) return DSM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const MergeWork w = merge_work(capacity, m, row_floats);
  unsigned char* base = (unsigned char*)work;
  int* keep_a = (int*)(base + w.keep_a);
  int* keep_n = (int*)(base + w.keep_n);
  int* pref_a = (int*)(base + w.pref_a);
  int* pos_a = (int*)(base + w.pos_a);
  int* pos_n = (int*)(base + w.pos_n);
  double* vec = (double*)(base + w.vec);
  float* rows = (float*)(base + w.rows);
  int* hdr = (int*)(base + w.hdr);
  k_merge_mark_archive<<<(capacity + 255) / 256, 256, 0, st>>>(archive, n_archive, capacity, m, points, keep_a);
  if (m > 0) k_merge_mark_new<<<m, kMergeWG, 0, st>>>(archive, n_archive, capacity, m, points, keep_n);
  k_merge_prefix<<<1, 1024, 0, st>>>(keep_a, capacity, pref_a);
  k_merge_positions<<<(capacity + m + 1 + 255) / 256, 256, 0, st>>>(archive, n_archive, capacity, m, points, keep_a,
                                                                   keep_n, pref_a, pos_a, pos_n, hdr);
  const int64_t sc = (int64_t)(capacity + m) * (3 + row_floats), cb = (int64_t)capacity * (3 + row_floats);
  k_merge_scatter<<<(unsigned)std::min<int64_t>((sc + 255) / 256, 16384), 256, 0, st>>>(
      archive, archive_rows, capacity, m, points, point_rows, row_floats, pos_a, pos_n, hdr, vec, rows);
  k_merge_copyback<<<(unsigned)std::min<int64_t>((cb + 255) / 256, 16384), 256, 0, st>>>(
      archive, archive_rows, capacity, row_floats, vec, rows, hdr, n_archive, overflow);
  k_merge_count<<<1, 64, 0, st>>>(hdr, n_archive);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_select(int32_t S, const double* obj, int32_t n_sel, int32_t* sel, int32_t* dominated_by, void* stream) {
  if (S < 0 || n_sel < 0 || n_sel > S) return DSM_ERR_ARG;
  if (S > 8192) return DSM_ERR_CAPACITY;
  if (S == 0) return DSM_OK;
  if (!obj || (n_sel > 0 && !sel)) return DSM_ERR_ARG;
  k_select<<<1, kSelWG, sizeof(double) * S, (hipStream_t)stream>>>(S, obj, n_sel, sel, dominated_by);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_avs_update(int32_t n, float* mult, int32_t* nis, const double* sdr, int32_t nis_max, float eta, float lo,
                          float hi, void* stream) {
  if (n < 0 || !(eta > 0.f && eta < 1.f) || !(lo > 0.f && lo <= hi)) return DSM_ERR_ARG;
  if (n == 0) return DSM_OK;
  if (!mult || !nis || !sdr) return DSM_ERR_ARG;
  k_avs<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(n, mult, nis, sdr, nis_max, eta, lo, hi);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_multiplier_step(int32_t k, int32_t F, int32_t S, const uint8_t* accepted, const int32_t* cluster,
                               float* mult, float eta, float lo, float hi, void* stream) {
  if (k < 1 || F < 0 || S < 0 || !(eta > 0.f && eta < 1.f) || !(lo > 0.f && lo <= hi)) return DSM_ERR_ARG;
  if (F == 0) return DSM_OK;
  if (!mult || (S > 0 && !accepted) || (k > 1 && !cluster)) return DSM_ERR_ARG;
  k_multiplier_step<<<(k * F + 255) / 256, 256, 0, (hipStream_t)stream>>>(k, F, S, accepted, k > 1 ? cluster : nullptr,
                                                                        mult, eta, lo, hi);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_mark_improved(int32_t S, int32_t F, const uint8_t* accepted, uint8_t* improved, void* stream) {
  if (S < 0 || F < 0) return DSM_ERR_ARG;
  if (S == 0 || F == 0) return DSM_OK;
  if (!accepted || !improved) return DSM_ERR_ARG;
  k_mark_improved<<<(S + 255) / 256, 256, 0, (hipStream_t)stream>>>(S, F, accepted, improved);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_ams_shift(int32_t n, const double* mean, double* prev, double* shift, int32_t has_prev, void* stream) {
  if (n < 0) return DSM_ERR_ARG;
  if (n == 0) return DSM_OK;
  if (!mean || !prev || (has_prev && !shift)) return DSM_ERR_ARG;
  k_ams_shift<<<std::min(1024, (n + 255) / 256), 256, 0, (hipStream_t)stream>>>(n, mean, prev, shift, has_prev ? 1 : 0);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_single_objective_clusters(int32_t k, const double* means, int32_t S, const int32_t* assign, int32_t* so,
                                         void* stream) {
  if (k < 1 || k > kClusterMax || S < 0) return DSM_ERR_ARG;
  if (S == 0) return DSM_OK;
  if (!means || !assign || !so) return DSM_ERR_ARG;
  k_so_clusters<<<std::min(64, (S + 255) / 256), 256, 0, (hipStream_t)stream>>>(k, means, S, assign, so);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_draw_donors(int32_t S, const int32_t* nis, int32_t nis_max, const int32_t* dominated_by, const float* u,
                           int32_t* donor, int32_t* n_forced, void* stream) {
  if (S < 0) return DSM_ERR_ARG;
  if (S > 8192) return DSM_ERR_CAPACITY;
  if (S == 0) return DSM_OK;
  if (!nis || !dominated_by || !u || !donor) return DSM_ERR_ARG;
  k_draw_donors<<<1, 1024, sizeof(int) * S, (hipStream_t)stream>>>(S, nis, nis_max, dominated_by, u, donor, n_forced);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

size_t dsm_forced_work_bytes(const dsm_problem* p, int32_t S) {
  if (!p || S < 0) return 0;
  return (size_t)S * (sizeof(float) * 6 * p->topo.P + sizeof(double) * 3 + sizeof(double) * 3 * p->topo.T);
}

dsm_status dsm_forced_replace(dsm_problem* p, int32_t S, float* X, double* obj, double* cache, const int32_t* donor,
                              const uint8_t* improved, int32_t* nis, void* work, int32_t* n_replaced, void* stream) {
  if (!p || S < 0) return DSM_ERR_ARG;
  if (S == 0) return DSM_OK;
  if (!X || !obj || !cache || !donor || !improved || !nis || !work) return DSM_ERR_ARG;
  const int row_x = 6 * p->topo.P, row_c = 3 * p->topo.T;
  float* wx = (float*)work;
  double* wobj = (double*)(wx + (size_t)S * row_x);  // row_x = 6 P floats: 8-byte aligned
  double* wcache = wobj + 3 * (size_t)S;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)std::min(64, (row_x + 3 + row_c + 255) / 256), (unsigned)S);
  k_forced_stage<<<grid, 256, 0, st>>>(S, row_x, row_c, X, obj, cache, donor, improved, wx, wobj, wcache);
  k_forced_apply<<<grid, 256, 0, st>>>(S, row_x, row_c, X, obj, cache, donor, improved, wx, wobj, wcache, nis,
                                       n_replaced);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

}  // extern "C"
