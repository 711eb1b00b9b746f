// Generation step support for a population optimiser on top of the evaluator:
// a counter-based candidate sampler and the acceptance of partial changes.
//
// Sec. 2.2: each partial change is accepted only if it improves the solution;
// changes to FOS elements whose affected tetrahedra are disjoint (one colour
// class of single points: equal index parity on every axis) are independent, so
// all accepted changes of a class are applied together.  "Improves" is read in
// the multi-objective sense: the candidate is feasible and either Pareto-
// dominates the current solution or is not dominated by any member of the
// elitist archive.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <math.h>

#include "dsm_internal.h"

namespace dsm {
namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// standard normal from two counter-based uniforms (Box-Muller)
__device__ __forceinline__ double normal(unsigned long long seed, unsigned long long ctr) {
  const unsigned long long a = mix64(seed + 0x9e3779b97f4a7c15ull * (2 * ctr + 1));
  const unsigned long long b = mix64(seed + 0x9e3779b97f4a7c15ull * (2 * ctr + 2));
  const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// cand [S][F][K][2][3]: current position of single point pts[f] plus
// N(0, sigma) voxels on its free axes, clamped to the image box and rounded to
// the 1/128-voxel lattice (half to even).
__global__ void k_sample(DevProblem pr, int S, const float* __restrict__ X, int F, const int* __restrict__ pts, int K,
                         float sigma, unsigned long long seed, unsigned long long counter,
                         const unsigned long long* __restrict__ counter_dev, float* __restrict__ cand) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (counter_dev) counter += *counter_dev;
  const int64_t n = (int64_t)S * F * K * 6;
  if (e >= n) return;
  const int comp = (int)(e % 6);
  const int64_t row = e / 6;
  const int f = (int)((row / K) % F);
  const int s = (int)(row / ((int64_t)F * K));
  const int g = comp / 3, a = comp % 3;
  const int p = pts[f];
  if (p < 0 || p >= pr.P) {
    cand[e] = NAN;  // flagged as non-finite by the evaluator
    return;
  }
  const float x = X[(((size_t)s * 2 + g) * pr.P + p) * 3 + a];
  const int idx = a == 0 ? p % pr.n[0] : (a == 1 ? (p / pr.n[0]) % pr.n[1] : p / (pr.n[0] * pr.n[1]));
  const bool free_axis = idx > 0 && idx < pr.n[a] - 1;
  double v = x;
  if (free_axis) {
    v += sigma * normal(seed, counter * 0x100000000ull + (unsigned long long)e);
    v = fmin(fmax(v, -0.5), pr.D[a] - 0.5);
  }
  v = rint((v + 0.5) * kLat) / kLat - 0.5;
  cand[e] = (float)v;
}

// ------------------------------------------------ estimated distributions
// RV-GOMEA, on which Sec. 2.2 builds, draws the variables of a FOS element
// from a normal distribution estimated on selected solutions of the
// population.  For a single-point element the variables are the point's 6
// coordinates (source grid x y z, target grid x y z); coordinates pinned to
// the box (border points) are not variables.

constexpr int kPtTile = 128;  // selected solutions staged in LDS at a time

// Per element f: mean [F][6] of the point's coordinates over the solutions
// sel[0..n_sel) (indices outside [0, S) are skipped), and chol [F][21], the
// lower Cholesky factor (rows 0..5, row r holding columns 0..r) of their
// maximum-likelihood covariance (divisor: the number of solutions used)
// restricted to the free coordinates; pinned rows and columns are 0, and a
// pivot that is not positive (a rank-deficient selection) gives a zero
// column.  Sums run over sel in order, in FP64.
__global__ __launch_bounds__(64) void k_estimate(DevProblem pr, int S, const float* __restrict__ X, int n_sel,
                                                 const int* __restrict__ sel, int F, const int* __restrict__ pts,
                                                 double* __restrict__ mean, double* __restrict__ chol) {
  // one wave per point: the selected solutions' 6 coordinates are staged in LDS
  // tiles; lane c < 6 sums mean component c and lane e < 21 covariance entry e,
  // each over the selection in order
  __shared__ float s_x[kPtTile][6];
  __shared__ int s_ok[kPtTile];
  __shared__ double s_m[6];
  __shared__ double s_C[21];
  const int f = blockIdx.x, t = threadIdx.x;
  double* mu = mean + (size_t)f * 6;
  double* L = chol + (size_t)f * 21;
  if (t < 6) mu[t] = 0.0;
  if (t < 21) L[t] = 0.0;
  const int p = pts[f];
  if (p < 0 || p >= pr.P || n_sel < 1) return;
  const int idx[3] = {p % pr.n[0], (p / pr.n[0]) % pr.n[1], p / (pr.n[0] * pr.n[1])};
  bool fr[6];
  for (int c = 0; c < 6; ++c) fr[c] = idx[c % 3] > 0 && idx[c % 3] < pr.n[c % 3] - 1;
  int n = 0;
  for (int i = 0; i < n_sel; ++i) n += sel[i] >= 0 && sel[i] < S;
  if (n == 0) return;
  auto stage = [&](int i0) {
    const int rows = min(kPtTile, n_sel - i0);
    for (int q = t; q < rows * 6; q += 64) {
      const int i = q / 6, c = q % 6, si = sel[i0 + i];
      s_x[i][c] = si >= 0 && si < S ? X[(((size_t)si * 2 + c / 3) * pr.P + p) * 3 + c % 3] : 0.f;
    }
    for (int i = t; i < rows; i += 64) s_ok[i] = sel[i0 + i] >= 0 && sel[i0 + i] < S;
    __syncthreads();
    return rows;
  };
  double m = 0.0;
  for (int i0 = 0; i0 < n_sel; i0 += kPtTile) {
    const int rows = stage(i0);
    if (t < 6)
      for (int i = 0; i < rows; ++i)
        if (s_ok[i]) m += (double)s_x[i][t];
    __syncthreads();
  }
  if (t < 6) s_m[t] = m / n;
  __syncthreads();
  int r = 0;
  while (t < 21 && (r + 1) * (r + 2) / 2 <= t) ++r;
  const int c = t - r * (r + 1) / 2;
  double acc = 0.0;
  for (int i0 = 0; i0 < n_sel; i0 += kPtTile) {
    const int rows = stage(i0);
    if (t < 21)
      for (int i = 0; i < rows; ++i)
        if (s_ok[i]) {
          const double dr = fr[r] ? (double)s_x[i][r] - s_m[r] : 0.0;
          const double dc = fr[c] ? (double)s_x[i][c] - s_m[c] : 0.0;
          acc += dr * dc;
        }
    __syncthreads();
  }
  if (t < 21) s_C[t] = acc / n;
  __syncthreads();
  if (t != 0) return;
  double l[21] = {0};
  for (int r2 = 0; r2 < 6; ++r2)
    for (int c2 = 0; c2 <= r2; ++c2) {
      double v = s_C[r2 * (r2 + 1) / 2 + c2];
      for (int k = 0; k < c2; ++k) v -= l[r2 * (r2 + 1) / 2 + k] * l[c2 * (c2 + 1) / 2 + k];
      if (c2 == r2)
        l[r2 * (r2 + 1) / 2 + r2] = v > 0.0 ? sqrt(v) : 0.0;
      else {
        const double d = l[c2 * (c2 + 1) / 2 + c2];
        l[r2 * (r2 + 1) / 2 + c2] = d > 0.0 ? v / d : 0.0;
      }
    }
  for (int k = 0; k < 6; ++k) mu[k] = s_m[k];
  for (int k = 0; k < 21; ++k) L[k] = l[k];
}

// cand [S][F][K][2][3]: mean + sqrt(mult[f]) L z on the free coordinates of
// single point pts[f], z ~ N(0, I) from the counter-based generator (6 draws
// per candidate, counters as in k_sample); pinned coordinates keep the
// solution's value; clamped to the image box and rounded to the 1/128-voxel
// lattice (half to even).
__global__ void k_sample_est(DevProblem pr, int S, const float* __restrict__ X, int F, const int* __restrict__ pts, int K,
                             const double* __restrict__ mean, const double* __restrict__ chol,
                             const float* __restrict__ mult, int n_clusters, const int* __restrict__ cluster,
                             const double* __restrict__ shift, const unsigned char* __restrict__ ams, double delta,
                             unsigned long long seed, unsigned long long counter,
                             const unsigned long long* __restrict__ counter_dev, float* __restrict__ cand) {
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (counter_dev) counter += *counter_dev;
  if (row >= (int64_t)S * F * K) return;
  const int f = (int)((row / K) % F);
  const int s = (int)(row / ((int64_t)F * K));
  const int p = pts[f];
  float* out = cand + row * 6;
  const int cl = cluster ? cluster[s] : 0;
  if (p < 0 || p >= pr.P || cl < 0 || cl >= n_clusters) {
    for (int c = 0; c < 6; ++c) out[c] = NAN;  // flagged as non-finite by the evaluator
    return;
  }
  const size_t d = (size_t)cl * F + f;  // distribution of the solution's cluster
  const double* mu = mean + d * 6;
  const double* L = chol + d * 21;
  const double sc = sqrt((double)mult[d]);
  double z[6];
  for (int c = 0; c < 6; ++c) z[c] = normal(seed, counter * 0x100000000ull + (unsigned long long)(row * 6 + c));
  const int idx[3] = {p % pr.n[0], (p / pr.n[0]) % pr.n[1], p / (pr.n[0] * pr.n[1])};
  for (int c = 0; c < 6; ++c) {
    const int g = c / 3, a = c % 3;
    double v = X[(((size_t)s * 2 + g) * pr.P + p) * 3 + a];
    if (idx[a] > 0 && idx[a] < pr.n[a] - 1) {
      double w = 0.0;
      for (int t = 0; t <= c; ++t) w += L[c * (c + 1) / 2 + t] * z[t];
      double m = mu[c];
      if (shift && ams[s]) m += delta * (double)mult[d] * shift[(size_t)p * 6 + c];  // anticipated mean shift
      v = fmin(fmax(m + sc * w, -0.5), pr.D[a] - 0.5);
    }
    out[c] = (float)(rint((v + 0.5) * kLat) / kLat - 0.5);
  }
}

// Multi-point elements (such as the paper's per-cube tetrahedra): the
// variables of element f are the coordinates of its points
// fos_pts[fos_off[f] .. fos_off[f+1]) in order, 6 per point (source x y z,
// target x y z), at most kEstPoints points.  The distribution is estimated
// over all of them jointly (full covariance).
constexpr int kEstPoints = 4, kEstVars = 6 * kEstPoints, kEstTri = kEstVars * (kEstVars + 1) / 2;
constexpr int kEstTile = 128;  // selected solutions staged in LDS at a time

// One 64-thread workgroup per element: mean [F][kEstVars] and the lower
// Cholesky factor chol [F][kEstTri] (row r holding columns 0..r) of the
// maximum-likelihood covariance of the free variables over the solutions
// sel[0..n_sel) (indices outside [0, S) skipped); rows and columns of pinned
// coordinates, and of variables beyond 6 x (number of points), are 0; a
// non-positive pivot gives a zero column.  Elements with no point, more than
// kEstPoints points or an invalid point get zeros.
__global__ __launch_bounds__(64) void k_estimate_el(DevProblem pr, int S, const float* __restrict__ X, int n_sel,
                                                    const int* __restrict__ sel, int F, const int* __restrict__ off,
                                                    const int* __restrict__ pts, double* __restrict__ mean,
                                                    double* __restrict__ chol) {
  __shared__ double s_mu[kEstVars];
  __shared__ double s_C[kEstTri];
  __shared__ int s_valid;
  __shared__ float s_x[kEstTile][kEstVars];
  __shared__ int s_ok[kEstTile];
  const int f = blockIdx.x, t = threadIdx.x;
  double* mu = mean + (size_t)f * kEstVars;
  double* L = chol + (size_t)f * kEstTri;
  for (int i = t; i < kEstVars; i += 64) mu[i] = 0.0;
  for (int i = t; i < kEstTri; i += 64) L[i] = 0.0;
  const int b = off[f], np = off[f + 1] - b;
  if (t == 0) {
    int ok = b >= 0 && np >= 1 && np <= kEstPoints && b + np <= off[F];
    for (int k = 0; ok && k < np; ++k) ok = pts[b + k] >= 0 && pts[b + k] < pr.P;
    s_valid = ok;
  }
  __syncthreads();
  if (!s_valid) return;
  const int nv = 6 * np;
  int n = 0;  // solutions used
  for (int i = 0; i < n_sel; ++i) n += sel[i] >= 0 && sel[i] < S;
  if (n == 0) return;
  // variable v: point v / 6, coordinate v % 6; free unless pinned to the box
  auto is_free = [&](int v) {
    const int p = pts[b + v / 6], a = v % 3;
    const int idx = a == 0 ? p % pr.n[0] : (a == 1 ? (p / pr.n[0]) % pr.n[1] : p / (pr.n[0] * pr.n[1]));
    return idx > 0 && idx < pr.n[a] - 1;
  };
  // the selected solutions' coordinates, staged in LDS tiles of kEstTile rows;
  // every sum still runs over the selection in order
  auto stage = [&](int i0) {
    const int rows = min(kEstTile, n_sel - i0);
    for (int q = t; q < rows * nv; q += 64) {
      const int i = q / nv, v = q % nv;
      const int si = sel[i0 + i];
      float x = 0.f;
      if (si >= 0 && si < S) {
        const int p = pts[b + v / 6], c = v % 6;
        x = X[(((size_t)si * 2 + c / 3) * pr.P + p) * 3 + c % 3];
      }
      s_x[i][v] = x;
    }
    for (int i = t; i < rows; i += 64) s_ok[i] = sel[i0 + i] >= 0 && sel[i0 + i] < S;
    __syncthreads();
    return rows;
  };
  double m = 0.0;
  for (int i0 = 0; i0 < n_sel; i0 += kEstTile) {
    const int rows = stage(i0);
    if (t < nv)
      for (int i = 0; i < rows; ++i)
        if (s_ok[i]) m += (double)s_x[i][t];
    __syncthreads();
  }
  if (t < nv) s_mu[t] = m / n;
  __syncthreads();
  constexpr int kPer = (kEstTri + 63) / 64;  // covariance entries per thread
  const int ne = nv * (nv + 1) / 2;
  double acc[kPer];
  int er[kPer], ec[kPer];
  bool ef[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int e = t + 64 * k;
    int r = 0;
    if (e < ne)
      while ((r + 1) * (r + 2) / 2 <= e) ++r;
    er[k] = r;
    ec[k] = e - r * (r + 1) / 2;
    ef[k] = e < ne && is_free(r) && is_free(ec[k]);
    acc[k] = 0.0;
  }
  for (int i0 = 0; i0 < n_sel; i0 += kEstTile) {
    const int rows = stage(i0);
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (ef[k]) {
        const double mr = s_mu[er[k]], mc = s_mu[ec[k]];
        for (int i = 0; i < rows; ++i)
          if (s_ok[i]) acc[k] += ((double)s_x[i][er[k]] - mr) * ((double)s_x[i][ec[k]] - mc);
      }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (t + 64 * k < ne) s_C[t + 64 * k] = acc[k] / n;
  __syncthreads();
  if (t == 0) {  // in place: s_C becomes the factor
    for (int r = 0; r < nv; ++r)
      for (int c = 0; c <= r; ++c) {
        double v = s_C[r * (r + 1) / 2 + c];
        for (int k = 0; k < c; ++k) v -= s_C[r * (r + 1) / 2 + k] * s_C[c * (c + 1) / 2 + k];
        if (c == r)
          s_C[r * (r + 1) / 2 + r] = v > 0.0 ? sqrt(v) : 0.0;
        else {
          const double d = s_C[c * (c + 1) / 2 + c];
          s_C[r * (r + 1) / 2 + c] = d > 0.0 ? v / d : 0.0;
        }
      }
  }
  __syncthreads();
  if (t < nv) mu[t] = s_mu[t];
  for (int e = t; e < nv * (nv + 1) / 2; e += 64) L[e] = s_C[e];
}

// cand [S][fos_off[F]][2][3] for multi-point elements: mean + sqrt(mult[f]) L z
// on the element's free variables, z ~ N(0, I) (kEstVars draws per solution
// and element, counters as in k_sample); pinned coordinates keep the
// solution's value; clamped to the box and rounded to the lattice.  Elements
// that k_estimate_el rejects get NaN candidates.
__global__ void k_sample_el(DevProblem pr, int S, const float* __restrict__ X, int F, const int* __restrict__ off,
                            const int* __restrict__ pts, const double* __restrict__ mean,
                            const double* __restrict__ chol, const float* __restrict__ mult, int n_clusters,
                            const int* __restrict__ cluster, const double* __restrict__ shift,
                            const unsigned char* __restrict__ ams, double delta, unsigned long long seed, unsigned long long counter,
                            const unsigned long long* __restrict__ counter_dev, float* __restrict__ cand) {
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (counter_dev) counter += *counter_dev;
  if (row >= (int64_t)S * F) return;
  const int s = (int)(row / F), f = (int)(row % F);
  const int b = off[f], np = off[f + 1] - b, total = off[F];
  if (b < 0 || np < 0 || b + np > total) return;  // malformed offsets: nothing of this element to write
  const int cl = cluster ? cluster[s] : 0;
  bool ok = np >= 1 && np <= kEstPoints && cl >= 0 && cl < n_clusters;
  for (int k = 0; ok && k < np; ++k) ok = pts[b + k] >= 0 && pts[b + k] < pr.P;
  if (!ok) {
    for (int k = 0; k < np; ++k)
      for (int c = 0; c < 6; ++c) cand[((size_t)s * total + b + k) * 6 + c] = NAN;
    return;
  }
  const size_t d = (size_t)cl * F + f;  // distribution of the solution's cluster
  const double* mu = mean + d * kEstVars;
  const double* L = chol + d * kEstTri;
  const double sc = sqrt((double)mult[d]);
  double z[kEstVars];
  for (int v = 0; v < 6 * np; ++v) z[v] = normal(seed, counter * 0x100000000ull + (unsigned long long)(row * kEstVars + v));
  for (int v = 0; v < 6 * np; ++v) {
    const int p = pts[b + v / 6], c = v % 6, g = c / 3, a = c % 3;
    const int idx = a == 0 ? p % pr.n[0] : (a == 1 ? (p / pr.n[0]) % pr.n[1] : p / (pr.n[0] * pr.n[1]));
    double x = X[(((size_t)s * 2 + g) * pr.P + p) * 3 + a];
    if (idx > 0 && idx < pr.n[a] - 1) {
      double w = 0.0;
      for (int k = 0; k <= v; ++k) w += L[v * (v + 1) / 2 + k] * z[k];
      double m = mu[v];
      if (shift && ams[s]) m += delta * (double)mult[d] * shift[(size_t)p * 6 + c];  // anticipated mean shift
      x = fmin(fmax(m + sc * w, -0.5), pr.D[a] - 0.5);
    }
    cand[((size_t)s * total + b + v / 6) * 6 + c] = (float)(rint((x + 0.5) * kLat) / kLat - 0.5);
  }
}

// Accept / apply one colour class of single-point elements.
__global__ void k_accept(DevProblem pr, int S, float* __restrict__ X, int F, const int* __restrict__ off,
                         const int* __restrict__ pts, const float* __restrict__ cand, const double* __restrict__ part_old,
                         const double* __restrict__ part_new, const uint32_t* __restrict__ flags,
                         const double* __restrict__ terms_cand, double* __restrict__ cache,
                         const double* __restrict__ obj, int n_arch, const double* __restrict__ arch,
                         const int* __restrict__ single_objective, unsigned char* __restrict__ accepted) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * F) return;
  const int s = e / F, f = e % F;
  bool acc = flags[e] == 0u;
  if (acc) {
    double d[3], nv[3];
    bool le = true, lt = false;
    for (int o = 0; o < 3; ++o) {
      d[o] = part_new[(size_t)e * 3 + o] - part_old[(size_t)e * 3 + o];
      nv[o] = obj[(size_t)s * 3 + o] + d[o];
      le = le && d[o] <= 0.0;
      lt = lt || d[o] < 0.0;
    }
    acc = le && lt;
    const int so = single_objective ? single_objective[s] : -1;
    if (so >= 0 && so < 3) {
      acc = d[so] < 0.0;  // a single-objective cluster's member: improve that objective
    } else if (!acc && n_arch > 0) {
      bool dominated = false, improves = false;
      for (int o = 0; o < 3; ++o) improves = improves || d[o] < 0.0;
      for (int q = 0; q < n_arch && !dominated; ++q) {
        if (arch[(size_t)q * 3] == INFINITY) break;  // padding ends the archive
        bool ale = true, alt = false;
        for (int o = 0; o < 3; ++o) {
          ale = ale && arch[(size_t)q * 3 + o] <= nv[o];
          alt = alt || arch[(size_t)q * 3 + o] < nv[o];
        }
        dominated = ale && alt;
      }
      acc = improves && !dominated;
    }
  }
  if (accepted) accepted[e] = acc ? 1 : 0;
  if (!acc) return;
  // the element's points: pts[off[f] .. off[f+1]) with candidates at
  // [s][off[F]][2][3], or the single point pts[f] without off
  const int j0 = off ? off[f] : f, j1 = off ? off[f + 1] : f + 1, n = off ? off[F] : F;
  for (int j = j0; j < j1; ++j) {
    const int p = pts[j];
    if (p < 0 || p >= pr.P) continue;  // such elements are flagged by the evaluator
    for (int c = 0; c < 6; ++c)
      X[(((size_t)s * 2 + c / 3) * pr.P + p) * 3 + c % 3] = cand[((size_t)s * n + j) * 6 + c];
    for (int k = pr.star_off[p]; k < pr.star_off[p + 1]; ++k) {
      const size_t t = (size_t)s * pr.T + pr.star[k];
      for (int o = 0; o < 3; ++o) cache[t * 3 + o] = terms_cand[t * 3 + o];
    }
  }
}

// Sec. 2.4 grid refinement: fine point (I, J, K) of a 2n-1 grid is the mean of
// the coarse points whose indices are floor or ceil of (I/2, J/2, K/2): a
// coarse point, an edge middle, a face middle or a cube centre.  The mean of
// lattice integers (1, 2, 4 or 8 of them) is exact in FP64 and is rounded
// to the lattice half to even.  One thread per (solution, grid, fine point).
__global__ void k_refine(int nx, int ny, int nz, int S, const float* __restrict__ Xc, float* __restrict__ Xf) {
  const int fx = 2 * nx - 1, fy = 2 * ny - 1, fz = 2 * nz - 1;
  const int64_t Pc = (int64_t)nx * ny * nz, Pf = (int64_t)fx * fy * fz;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)S * 2 * Pf) return;
  const int64_t sg = e / Pf;
  const int f = (int)(e - sg * Pf);
  const int I = f % fx, J = (f / fx) % fy, K = f / (fx * fy);
  const int i0 = I >> 1, i1 = (I + 1) >> 1, j0 = J >> 1, j1 = (J + 1) >> 1, k0 = K >> 1, k1 = (K + 1) >> 1;
  const float* base = Xc + sg * Pc * 3;
  double u[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 8; ++c) {  // the 8 index combinations; repeated corners weigh equally
    const int i = (c & 1) ? i1 : i0, j = (c & 2) ? j1 : j0, k = (c & 4) ? k1 : k0;
    const float* x = base + ((int64_t)(k * ny + j) * nx + i) * 3;
    for (int d = 0; d < 3; ++d) u[d] += ((double)x[d] + 0.5) * kLat;
  }
  float* y = Xf + e * 3;
  for (int d = 0; d < 3; ++d) y[d] = (float)(rint(u[d] * 0.125) / kLat - 0.5);
}

// Forced improvements (RV-GOMEA): a solution s with donor[s] in [0, S) takes,
// for every listed point, the donor's current coordinates in both grids as its
// candidate (cand [S][n][2][3], the partial-evaluation layout); other
// solutions' candidates are left as they are.
__global__ void k_donor(int S, int P, const float* __restrict__ X, int n, const int* __restrict__ pts,
                        const int* __restrict__ donor, float* __restrict__ cand) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)S * n * 6) return;
  const int s = (int)(e / ((int64_t)n * 6));
  const int k = (int)((e / 6) % n), c = (int)(e % 6);
  const int d = donor[s], p = pts[k];
  if (d < 0 || d >= S || p < 0 || p >= P) return;
  cand[e] = X[(((size_t)d * 2 + c / 3) * P + p) * 3 + c % 3];
}

// Standard-deviation ratio of the improvements (AMaLGaM's adaptive variance
// scaling, used by RV-GOMEA): per (cluster j, element f) the mean of the
// accepted candidates of the cluster's solutions, compared with the
// distribution's mean variable by variable in units of the variable's standard
// deviation (sqrt of the row norm of L); the largest ratio, or -1 without an
// accepted candidate.  One wave per (cluster, element): the candidates are
// staged in LDS tiles and lane v sums variable v over the solutions in order.
constexpr int kSdrTile = 128;

__global__ __launch_bounds__(64) void k_sdr(int S, int F, const int* __restrict__ off, const float* __restrict__ cand,
                                            const unsigned char* __restrict__ accepted, int n_clusters,
                                            const int* __restrict__ cluster, const double* __restrict__ mean,
                                            const double* __restrict__ chol, int nvar, double* __restrict__ sdr) {
  __shared__ float s_x[kSdrTile][kEstVars];
  __shared__ int s_use[kSdrTile];
  const int e = blockIdx.x, lane = threadIdx.x;
  const int j = e / F, f = e % F;
  const int b = off[f], np = off[f + 1] - b, total = off[F];
  const int nv = 6 * np;
  if (b < 0 || np < 1 || nv > nvar || b + np > total) {
    if (lane == 0) sdr[e] = -1.0;
    return;
  }
  double sum = 0.0;
  int n = 0;
  for (int s0 = 0; s0 < S; s0 += kSdrTile) {
    const int rows = min(kSdrTile, S - s0);
    for (int i = lane; i < rows; i += 64) {
      const int s = s0 + i;
      s_use[i] = (cluster ? cluster[s] : 0) == j && accepted[(size_t)s * F + f];
    }
    __syncthreads();
    for (int q = lane; q < rows * nv; q += 64) {
      const int i = q / nv, v = q % nv;
      s_x[i][v] = s_use[i] ? cand[((size_t)(s0 + i) * total + b) * 6 + v] : 0.f;
    }
    __syncthreads();
    for (int i = 0; i < rows; ++i)
      if (s_use[i]) {
        if (lane < nv) sum += (double)s_x[i][lane];
        ++n;
      }
    __syncthreads();
  }
  if (n == 0) {
    if (lane == 0) sdr[e] = -1.0;
    return;
  }
  double r = 0.0;
  if (lane < nv) {
    const double* mu = mean + (size_t)e * nvar;
    const double* L = chol + (size_t)e * (nvar * (nvar + 1) / 2);
    double s2 = 0.0;
    for (int k = 0; k <= lane; ++k) s2 += L[lane * (lane + 1) / 2 + k] * L[lane * (lane + 1) / 2 + k];
    if (s2 > 0.0) r = fabs(sum / n - mu[lane]) / sqrt(s2);
  }
  for (int m = 32; m >= 1; m >>= 1) r = fmax(r, __shfl_xor(r, m, 64));  // the maximum does not depend on order
  if (lane == 0) sdr[e] = r;
}

// ---------------------------------------------------------------- clustering
// Balanced k-leader-means of the selected solutions in objective space (the
// clustering of MO-RV-GOMEA, on which the paper's optimiser builds, Sec. 2.2):
// normalisation over the selection, farthest-first leaders, k-means from the
// leaders, each cluster the c nearest selected solutions, every solution
// assigned to its nearest mean.  One workgroup; every floating-point step runs
// in a fixed order without contraction (sums in selection order by one thread
// per cluster and objective), so the result does not depend on the schedule.
constexpr int kClusterWG = 1024, kClusterWaves = kClusterWG / 64;

__device__ __forceinline__ double dist2(const double* a, const double* b) {
#pragma clang fp contract(off)
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}

__device__ __forceinline__ int nearest_mean(const double* y, const double (*mu)[3], int k) {
  int best = 0;
  double bd = dist2(y, mu[0]);
  for (int j = 1; j < k; ++j) {
    const double d = dist2(y, mu[j]);
    if (d < bd) {
      best = j;
      bd = d;
    }
  }
  return best;
}

// Index of the largest v[0..n) (lowest index among equals), for all threads.
__device__ int block_argmax(const double* v, int n, double* wv, int* wi, int* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double bv = -INFINITY;
  int bi = 0x7fffffff;
  for (int i = tid; i < n; i += kClusterWG)
    if (v[i] > bv) {  // increasing i: an equal later value never replaces
      bv = v[i];
      bi = i;
    }
  for (int m = 32; m >= 1; m >>= 1) {
    const double ov = __shfl_xor(bv, m);
    const int oi = __shfl_xor(bi, m);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    wv[wave] = bv;
    wi[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double b = wv[0];
    int i0 = wi[0];
    for (int w = 1; w < kClusterWaves; ++w)
      if (wv[w] > b || (wv[w] == b && wi[w] < i0)) {
        b = wv[w];
        i0 = wi[w];
      }
    *out = i0;
  }
  __syncthreads();
  return *out;
}

__global__ __launch_bounds__(kClusterWG) void k_cluster(int S, const double* __restrict__ obj, int n_sel,
                                                        const int* __restrict__ sel, int k, int cmax,
                                                        int* __restrict__ members, int* __restrict__ assign,
                                                        double* __restrict__ means_out) {
#pragma clang fp contract(off)
  __shared__ int s_idx[kClusterSelMax];
  __shared__ double s_Y[kClusterSelMax][3];
  __shared__ double s_d[kClusterSelMax];
  __shared__ int s_lab[kClusterSelMax];
  __shared__ double s_mu[kClusterMax][3];
  __shared__ int s_lead[kClusterMax];
  __shared__ double s_lo[3], s_rng[3];
  __shared__ double s_red[kClusterWaves][6];
  __shared__ int s_wcnt[kClusterWaves];
  __shared__ double s_wv[kClusterWaves];
  __shared__ int s_wi[kClusterWaves];
  __shared__ int s_n, s_arg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // valid selected solutions, compacted in selection order
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int base = 0; base < n_sel; base += kClusterWG) {
    const int i = base + tid;
    const int s = i < n_sel ? sel[i] : -1;
    const bool v = s >= 0 && s < S;
    const unsigned long long m = __ballot(v);
    const int pre = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (lane == 0) s_wcnt[wave] = __popcll(m);
    __syncthreads();
    int off = s_n;
    for (int w = 0; w < wave; ++w) off += s_wcnt[w];
    if (v) s_idx[off + pre] = s;
    __syncthreads();
    if (tid == 0) {
      int t = s_n;
      for (int w = 0; w < kClusterWaves; ++w) t += s_wcnt[w];
      s_n = t;
    }
    __syncthreads();
  }
  const int n = s_n;
  const int c = min(n, (2 * n + k - 1) / k);
  for (int e = tid; e < k * cmax; e += kClusterWG)
    if (n < k || e % cmax >= c) members[e] = -1;
  if (n < k) {
    for (int s = tid; s < S; s += kClusterWG) assign[s] = -1;
    if (means_out && tid < 3 * k) means_out[tid] = NAN;
    return;
  }
  // per-objective range over the selection (min and max are order-free)
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = tid; i < n; i += kClusterWG)
    for (int o = 0; o < 3; ++o) {
      const double x = obj[(size_t)s_idx[i] * 3 + o];
      lo[o] = fmin(lo[o], x);
      hi[o] = fmax(hi[o], x);
    }
  for (int m = 32; m >= 1; m >>= 1)
    for (int o = 0; o < 3; ++o) {
      lo[o] = fmin(lo[o], __shfl_xor(lo[o], m));
      hi[o] = fmax(hi[o], __shfl_xor(hi[o], m));
    }
  if (lane == 0)
    for (int o = 0; o < 3; ++o) {
      s_red[wave][o] = lo[o];
      s_red[wave][3 + o] = hi[o];
    }
  __syncthreads();
  if (tid < 3) {
    double a = s_red[0][tid], b = s_red[0][3 + tid];
    for (int w = 1; w < kClusterWaves; ++w) {
      a = fmin(a, s_red[w][tid]);
      b = fmax(b, s_red[w][3 + tid]);
    }
    s_lo[tid] = a;
    s_rng[tid] = b - a > 0.0 ? b - a : 1.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += kClusterWG)
    for (int o = 0; o < 3; ++o) s_Y[i][o] = (obj[(size_t)s_idx[i] * 3 + o] - s_lo[o]) / s_rng[o];
  __syncthreads();
  // farthest-first leaders
  for (int i = tid; i < n; i += kClusterWG) s_d[i] = s_Y[i][0];
  __syncthreads();
  int lead = block_argmax(s_d, n, s_wv, s_wi, &s_arg);
  if (tid == 0) s_lead[0] = lead;
  for (int i = tid; i < n; i += kClusterWG) s_d[i] = dist2(s_Y[i], s_Y[lead]);
  __syncthreads();
  for (int l = 1; l < k; ++l) {
    lead = block_argmax(s_d, n, s_wv, s_wi, &s_arg);
    if (tid == 0) s_lead[l] = lead;
    for (int i = tid; i < n; i += kClusterWG) s_d[i] = fmin(s_d[i], dist2(s_Y[i], s_Y[lead]));
    __syncthreads();
  }
  if (tid < 3 * k) s_mu[tid / 3][tid % 3] = s_Y[s_lead[tid / 3]][tid % 3];
  for (int i = tid; i < n; i += kClusterWG) s_lab[i] = -1;
  __syncthreads();
  // k-means from the leaders
  for (int it = 0; it < kClusterRounds; ++it) {
    int changed = 0;
    for (int i = tid; i < n; i += kClusterWG) {
      const int j = nearest_mean(s_Y[i], s_mu, k);
      changed |= j != s_lab[i];
      s_lab[i] = j;
    }
    if (!__syncthreads_or(changed)) break;
    if (tid < 3 * k) {
      const int j = tid / 3, o = tid % 3;
      double acc = 0.0;
      int cnt = 0;
      for (int i = 0; i < n; ++i)
        if (s_lab[i] == j) {
          acc += s_Y[i][o];
          ++cnt;
        }
      if (cnt) s_mu[j][o] = acc / cnt;
    }
    __syncthreads();
  }
  // cluster j: the c selected solutions nearest to mean j (rank by distance, then position)
  for (int j = 0; j < k; ++j) {
    for (int i = tid; i < n; i += kClusterWG) s_d[i] = dist2(s_Y[i], s_mu[j]);
    __syncthreads();
    for (int i = tid; i < n; i += kClusterWG) {
      const double di = s_d[i];
      int rank = 0;
      for (int m = 0; m < n; ++m) rank += s_d[m] < di || (s_d[m] == di && m < i);
      if (rank < c) members[(size_t)j * cmax + rank] = s_idx[i];
    }
    __syncthreads();
  }
  for (int s = tid; s < S; s += kClusterWG) {
    double y[3];
    for (int o = 0; o < 3; ++o) y[o] = (obj[(size_t)s * 3 + o] - s_lo[o]) / s_rng[o];
    assign[s] = nearest_mean(y, s_mu, k);
  }
  if (means_out && tid < 3 * k) means_out[tid] = s_mu[tid / 3][tid % 3];
}

}  // namespace
}  // namespace dsm

using namespace dsm;

extern "C" {

dsm_status dsm_sample_candidates(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                 float sigma, uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                                 void* stream) {
  if (!p || S < 0 || F < 0 || K < 1 || !(sigma >= 0.f)) return DSM_ERR_ARG;
  const int64_t n = (int64_t)S * F * K * 6;
  if (n == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_pts || !cand) return DSM_ERR_ARG;
  k_sample<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(p->dev, S, X, F, fos_pts, K, sigma, seed,
                                                                       counter, (const unsigned long long*)counter_dev,
                                                                       cand);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_estimate_distributions(dsm_problem* p, int32_t S, const float* X, int32_t n_sel, const int32_t* sel,
                                      int32_t F, const int32_t* fos_pts, double* mean, double* chol, void* stream) {
  if (!p || S < 0 || F < 0 || n_sel < 0) return DSM_ERR_ARG;
  if (F == 0) return DSM_OK;  // empty buffers may be null
  if (!fos_pts || !mean || !chol || (n_sel > 0 && (!X || !sel))) return DSM_ERR_ARG;
  k_estimate<<<(unsigned)F, 64, 0, (hipStream_t)stream>>>(p->dev, S, X, n_sel, sel, F, fos_pts, mean,
                                                                        chol);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_sample_estimated(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                const double* mean, const double* chol, const float* mult, int32_t n_clusters,
                                const int32_t* cluster, const double* shift, const uint8_t* ams, double delta,
                                uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                                void* stream) {
  if (!p || S < 0 || F < 0 || K < 1) return DSM_ERR_ARG;
  const int64_t n = (int64_t)S * F * K;
  if (n == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_pts || !mean || !chol || !mult || !cand || n_clusters < 1 || (shift && !ams)) return DSM_ERR_ARG;
  k_sample_est<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      p->dev, S, X, F, fos_pts, K, mean, chol, mult, n_clusters, cluster, shift, ams, delta, seed, counter,
      (const unsigned long long*)counter_dev, cand);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_estimate_elements(dsm_problem* p, int32_t S, const float* X, int32_t n_sel, const int32_t* sel, int32_t F,
                                 const int32_t* fos_off, const int32_t* fos_pts, double* mean, double* chol,
                                 void* stream) {
  if (!p || S < 0 || F < 0 || n_sel < 0) return DSM_ERR_ARG;
  if (F == 0) return DSM_OK;  // empty buffers may be null
  if (!fos_off || !fos_pts || !mean || !chol || (n_sel > 0 && (!X || !sel))) return DSM_ERR_ARG;
  k_estimate_el<<<(unsigned)F, 64, 0, (hipStream_t)stream>>>(p->dev, S, X, n_sel, sel, F, fos_off, fos_pts, mean, chol);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_sample_elements(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                               const int32_t* fos_pts, const double* mean, const double* chol, const float* mult,
                               int32_t n_clusters, const int32_t* cluster, const double* shift, const uint8_t* ams,
                               double delta, uint64_t seed, uint64_t counter, const uint64_t* counter_dev, float* cand,
                               void* stream) {
  if (!p || S < 0 || F < 0) return DSM_ERR_ARG;
  const int64_t n = (int64_t)S * F;
  if (n == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_off || !fos_pts || !mean || !chol || !mult || !cand || n_clusters < 1 || (shift && !ams))
    return DSM_ERR_ARG;
  k_sample_el<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      p->dev, S, X, F, fos_off, fos_pts, mean, chol, mult, n_clusters, cluster, shift, ams, delta, seed, counter,
      (const unsigned long long*)counter_dev, cand);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_cluster_objectives(int32_t S, const double* obj, int32_t n_sel, const int32_t* sel, int32_t k,
                                  int32_t* members, int32_t* assign, double* means, void* stream) {
  if (S < 0 || n_sel < 0 || k < 1 || k > kClusterMax) return DSM_ERR_ARG;
  if (n_sel > kClusterSelMax) return DSM_ERR_CAPACITY;
  const int cmax = std::min<int>(n_sel, (2 * n_sel + k - 1) / k);
  if ((S > 0 && (!obj || !assign)) || (n_sel > 0 && !sel) || (cmax > 0 && !members)) return DSM_ERR_ARG;
  if (S == 0 && cmax == 0 && !means) return DSM_OK;  // nothing to write
  k_cluster<<<1, kClusterWG, 0, (hipStream_t)stream>>>(S, obj, n_sel, sel, k, cmax, members, assign, means);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_refine_population(const int32_t* mesh_coarse, int32_t S, const float* Xc, float* Xf, void* stream) {
  if (!mesh_coarse || S < 0 || (S > 0 && (!Xc || !Xf))) return DSM_ERR_ARG;
  const int nx = mesh_coarse[0], ny = mesh_coarse[1], nz = mesh_coarse[2];
  if (nx < 2 || ny < 2 || nz < 2 || nx > 129 || ny > 129 || nz > 129) return DSM_ERR_DOMAIN;
  const int64_t n = (int64_t)S * 2 * (2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1);
  if (n == 0) return DSM_OK;
  k_refine<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(nx, ny, nz, S, Xc, Xf);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_accept(dsm_problem* p, int32_t S, float* X, int32_t F, const int32_t* fos_pts, const float* cand,
                      const double* part_old, const double* part_new, const uint32_t* flags, const double* terms_cand,
                      double* terms_cache, double* obj, int32_t n_archive, const double* archive,
                      const int32_t* single_objective, uint8_t* accepted, void* stream) {
  if (!p || S < 0 || F < 0 || n_archive < 0 || (n_archive > 0 && !archive) || S > p->max_S) return DSM_ERR_ARG;
  if (S == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !terms_cache || !obj || (F > 0 && (!fos_pts || !cand || !part_old || !part_new || !flags || !terms_cand)))
    return DSM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (F > 0)
    k_accept<<<(S * F + 255) / 256, 256, 0, st>>>(p->dev, S, X, F, nullptr, fos_pts, cand, part_old, part_new, flags,
                                                   terms_cand, terms_cache, obj, n_archive, archive, single_objective,
                                                   accepted);
  if (hipGetLastError() != hipSuccess) return DSM_ERR_DEVICE;
  return launch_full_reduce(p->dev, S, terms_cache, obj, st) == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_improvement_ratio(int32_t S, int32_t F, const int32_t* fos_off, const float* cand,
                                 const uint8_t* accepted, int32_t n_clusters, const int32_t* cluster,
                                 const double* mean, const double* chol, int32_t n_vars, double* sdr, void* stream) {
  if (S < 0 || F < 0 || n_clusters < 1 || (n_vars != 6 && n_vars != kEstVars)) return DSM_ERR_ARG;
  const int64_t n = (int64_t)n_clusters * F;
  if (n == 0) return DSM_OK;
  if (!fos_off || !mean || !chol || !sdr || (S > 0 && (!cand || !accepted))) return DSM_ERR_ARG;
  k_sdr<<<(unsigned)n, 64, 0, (hipStream_t)stream>>>(S, F, fos_off, cand, accepted, n_clusters, cluster, mean, chol,
                                                    n_vars, sdr);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_copy_from_donor(dsm_problem* p, int32_t S, const float* X, int32_t n_pts, const int32_t* fos_pts,
                               const int32_t* donor, float* cand, void* stream) {
  if (!p || S < 0 || n_pts < 0) return DSM_ERR_ARG;
  const int64_t n = (int64_t)S * n_pts * 6;
  if (n == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_pts || !donor || !cand) return DSM_ERR_ARG;
  k_donor<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(S, p->dev.P, X, n_pts, fos_pts, donor, cand);
  return hipGetLastError() == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

dsm_status dsm_accept_elements(dsm_problem* p, int32_t S, float* X, int32_t F, const int32_t* fos_off,
                               const int32_t* fos_pts, const float* cand, const double* part_old,
                               const double* part_new, const uint32_t* flags, const double* terms_cand,
                               double* terms_cache, double* obj, int32_t n_archive, const double* archive,
                               const int32_t* single_objective, uint8_t* accepted, void* stream) {
  if (!p || S < 0 || F < 0 || n_archive < 0 || (n_archive > 0 && !archive) || S > p->max_S) return DSM_ERR_ARG;
  if (S == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !terms_cache || !obj ||
      (F > 0 && (!fos_off || !fos_pts || !cand || !part_old || !part_new || !flags || !terms_cand)))
    return DSM_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (F > 0)
    k_accept<<<(S * F + 255) / 256, 256, 0, st>>>(p->dev, S, X, F, fos_off, fos_pts, cand, part_old, part_new, flags,
                                                   terms_cand, terms_cache, obj, n_archive, archive, single_objective,
                                                   accepted);
  if (hipGetLastError() != hipSuccess) return DSM_ERR_DEVICE;
  return launch_full_reduce(p->dev, S, terms_cache, obj, st) == hipSuccess ? DSM_OK : DSM_ERR_DEVICE;
}

}  // extern "C"
