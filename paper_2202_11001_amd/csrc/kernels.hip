// gfx950 kernels of the dual simplex-mesh objective evaluator.
//
// Work decomposition (Sec. 2.2: the affected tetrahedra of a partial change
// are re-evaluated; Sec. 2.3: every objective is a sum of per-cell terms):
//   one workgroup per (FOS element, chunk of its affected tetrahedra,
//   solution) in partial evaluation, or per (chunk of tetrahedra, solution) in
//   full evaluation.  Its work units are (version, direction, tetrahedron,
//   batch of 64 voxel rows); each of the 4 waves takes a contiguous range of
//   units.  A wave computes the exact x-span of 64 rows (one row per lane),
//   prefix-sums the span lengths, and then sweeps the voxels of those rows 64
//   at a time, adjacent lanes on adjacent voxels, so that both the streamed
//   own-image reads and the trilinear gathers from the other image are
//   coalesced.
//
// Exactness: coordinates are lattice integers (1/128 voxel, |u| <= 2^16), so
// every orientation value and every face function evaluated at a voxel centre
// is an integer below 2^53 and FP64 arithmetic on it is exact; the voxel set of
// a tetrahedron is therefore decided bit-exactly.  Sampling and the
// dissimilarity sum are FP32 (per-lane compensated sums, FP64 across lanes).
#include <hip/hip_runtime.h>

#include "dsm_internal.h"

namespace dsm {

namespace {

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Lattice value of one coordinate and its constraint bits.
__device__ __forceinline__ unsigned lattice_of(float x, int D, double& u) {
  if (!isfinite(x)) {
    u = 0.0;
    return DSM_FLAG_NONFINITE;
  }
  const double v = ((double)x + 0.5) * kLat;
  u = v;
  if (v != floor(v)) return DSM_FLAG_LATTICE;
  if (v < 0.0 || v > kLat * D) return DSM_FLAG_DOMAIN;
  return 0u;
}

// 6 x signed volume of (a, b, c, d); exact for lattice integers.
__device__ __forceinline__ double orient(const double a[3], const double b[3], const double c[3], const double d[3]) {
  const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
  const double cx = v[1] * w[2] - v[2] * w[1];
  const double cy = v[2] * w[0] - v[0] * w[2];
  const double cz = v[0] * w[1] - v[1] * w[0];
  return u[0] * cx + u[1] * cy + u[2] * cz;
}

// Face functions of a positively oriented tetrahedron: o_i(U) = G_i . U + K_i
// is the orientation with vertex i replaced by U (zero on the face opposite i,
// vol at vertex i).  U lies in the tetrahedron iff o_i(U) >= thr_i for all i,
// where thr_i = 0 if the first non-zero component of G_i (x, then y, then z) is
// positive and 1 otherwise: the top-left rule of Sec. 2.3.1 extended to 3-D by
// perturbing U by (+e, +e^2, +e^3).
struct Faces {
  double G[4][3];
  double K[4];
  int thr[4];
};

__device__ __forceinline__ void make_faces(const double L[4][3], Faces& f) {
  for (int i = 0; i < 4; ++i) {
    const int j = i == 0 ? 1 : 0;
    const int k = i <= 1 ? 2 : 1;
    const int l = i <= 2 ? 3 : 2;
    const double a[3] = {L[k][0] - L[j][0], L[k][1] - L[j][1], L[k][2] - L[j][2]};
    const double b[3] = {L[l][0] - L[j][0], L[l][1] - L[j][1], L[l][2] - L[j][2]};
    double g[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double d[3] = {L[i][0] - L[j][0], L[i][1] - L[j][1], L[i][2] - L[j][2]};
    if (dot3(g, d) < 0.0) {
      g[0] = -g[0];
      g[1] = -g[1];
      g[2] = -g[2];
    }
    for (int c = 0; c < 3; ++c) f.G[i][c] = g[c];
    f.K[i] = -dot3(g, L[j]);
    const bool pos = g[0] != 0.0 ? g[0] > 0.0 : (g[1] != 0.0 ? g[1] > 0.0 : g[2] > 0.0);
    f.thr[i] = pos ? 0 : 1;
  }
}

__device__ __forceinline__ bool inside(const Faces& f, const double U[3], double o[4]) {
  bool in = true;
  for (int i = 0; i < 4; ++i) {
    o[i] = dot3(f.G[i], U) + f.K[i];
    in = in && (o[i] >= (double)f.thr[i]);
  }
  return in;
}

// inclusive voxel index range of lattice interval [lo, hi] (voxel i centred at 128 i + 64)
__device__ __forceinline__ void vox_range(double lo, double hi, int D, int& a, int& b) {
  a = max(0, (int)ceil((lo - 64.0) / kLat));
  b = min(D - 1, (int)floor((hi - 64.0) / kLat));
}

// Blockid -> logical index so that each of the 8 XCDs (which receive
// workgroups round robin) processes one contiguous range of logical indices;
// consecutive logical indices share a FOS element and hence an image region.
__device__ __forceinline__ int xcd_logical(int bid, int n) {
  const int x = bid & 7, k = bid >> 3;
  const int q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// Element order of a single-problem partial launch: every eighth element,
// starting from 0, then from 1, and so on.  The logical workgroup space is
// element-major and each XCD takes a contiguous range of it, so in mesh order
// the XCDs holding the border layers (whose points have smaller stars) would
// finish early; interleaved, every XCD takes elements from the whole mesh.
// Returns the element at position gp of that order, for G elements.
__device__ __forceinline__ int interleaved_group(int gp, int G) {
  int r = 0, base = 0;
  for (; r < 7; ++r) {
    const int cnt = (G - r + 7) >> 3;  // elements g < G with g % 8 == r
    if (gp < base + cnt) break;
    base += cnt;
  }
  return ((gp - base) << 3) + r;
}

// Makes LDS writes of some lanes visible to the other lanes of the same wave
// (and keeps the compiler from moving LDS accesses across this point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the kFinishLanes lanes of a lane group, in a fixed butterfly order
// (every lane of the group ends with the same sum).
__device__ __forceinline__ double group_sum(double v) {
  for (int off = kFinishLanes / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kFinishLanes);
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wave, all lanes active: DPP
// shifts within rows of 16 lanes, then the row totals carried by the
// broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return v;
}

// Inclusive prefix sum within each row of 16 lanes (the lanes of a row active).
__device__ __forceinline__ int row16_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);  // row_shr:8
  return v;
}

// Parameters of one (tetrahedron, direction) for rasterising the own grid's
// voxels and mapping them into the other grid.  Lives in LDS.
constexpr int kMaxSlices = 64;  // slice-table capacity; taller tetrahedra enumerate bounding-box rows

struct RasterTet {
  double A[4], C0[4], CY[4], CZ[4], rA[4];  // o_i(x,y,z) = A x + C0 + CY y + CZ z at voxel (x,y,z)
  double J[3][3];  // own voxel coords -> other grid voxel coords: p' = P0 + J v
  double P0[3];
  int thr[4];
  int zlo, nz, ylo, ny;  // bounding box (slices, rows)
  int nrows;             // candidate rows
  int sliced;            // 1: candidate rows from the slice table, 0: every bounding-box row
  int pairs;             // slice table: 0 one row group per slice, 1 one per pair of slices
  unsigned short y0[kMaxSlices];      // first candidate row (its y) of each row group
  unsigned short rs[kMaxSlices + 1];  // exclusive prefix of candidate rows per row group (<= 64 * 512)
};

// Conservative row range [ya, yb] of the cross-section of the tetrahedron
// (own-grid lattice vertices L, integers below 2^17 and hence exact in FP32)
// with voxel slice z: the rows whose centres lie in the y-extent of the
// section polygon (every voxel of the closed tetrahedron in that slice does),
// whose vertices are the edge / plane intersections.  They are computed in
// FP32 with an approximate reciprocal, with an error of a few 1e-3 lattice
// units at most; the extent is widened by 1/2 lattice unit against it.  The
// exact spans decide the voxels.
__device__ __forceinline__ void slice_rows(const float L[4][3], int z, int Dy, int& ya, int& yb) {
  const float Uz = 128.f * z + 64.f;
  float lo = INFINITY, hi = -INFINITY;
  for (int a = 0; a < 4; ++a) {
    if (L[a][2] == Uz) {
      lo = fminf(lo, L[a][1]);
      hi = fmaxf(hi, L[a][1]);
    }
    for (int b = a + 1; b < 4; ++b) {
      const float za = L[a][2], zb = L[b][2];
      if ((za < Uz && zb > Uz) || (za > Uz && zb < Uz)) {
        const float y = fmaf((Uz - za) * __builtin_amdgcn_rcpf(zb - za), L[b][1] - L[a][1], L[a][1]);
        lo = fminf(lo, y);
        hi = fmaxf(hi, y);
      }
    }
  }
  if (lo > hi) {
    ya = 0;
    yb = -1;
    return;
  }
  ya = max(0, (int)ceilf((lo - 64.5f) * (1.f / 128.f)));
  yb = min(Dy - 1, (int)floorf((hi - 63.5f) * (1.f / 128.f)));
}

// Rasterisation parameters of the tetrahedron with own-grid vertices xo[4][3]
// and other-grid vertices xt[4][3] (voxel units, already validated on the
// lattice), in two parts so that no thread holds all of it in registers.
// setup_task(k) for k in [0, 14) fills the face functions (k < 4), the affine
// map's matrix (4 <= k < 13) and the bounding box (k = 13); the 14 tasks may
// run on any threads.  setup_slices then runs on one wave, after the tasks'
// writes are visible to it, and fills the slice table and the map's offset.
constexpr int kSetupTasks = 14;

__device__ void setup_task(const float* xo, const float* xt, const int D[3], int lane, RasterTet& rt) {
  if (lane < 4) {
    // face opposite vertex `lane`
    const int i = lane;
    const int j = i == 0 ? 1 : 0, k = i <= 1 ? 2 : 1, l = i <= 2 ? 3 : 2;
    double Lj[3], a[3], b[3], d[3];
    for (int c = 0; c < 3; ++c) {
      Lj[c] = ((double)xo[3 * j + c] + 0.5) * kLat;
      a[c] = ((double)xo[3 * k + c] + 0.5) * kLat - Lj[c];
      b[c] = ((double)xo[3 * l + c] + 0.5) * kLat - Lj[c];
      d[c] = ((double)xo[3 * i + c] + 0.5) * kLat - Lj[c];
    }
    double g[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    if (dot3(g, d) < 0.0) {
      g[0] = -g[0];
      g[1] = -g[1];
      g[2] = -g[2];
    }
    const double K = -dot3(g, Lj);
    rt.A[i] = kLat * g[0];
    rt.CY[i] = kLat * g[1];
    rt.CZ[i] = kLat * g[2];
    rt.C0[i] = 64.0 * (g[0] + g[1] + g[2]) + K;
    rt.rA[i] = g[0] != 0.0 ? 1.0 / (kLat * g[0]) : 0.0;
    const bool pos = g[0] != 0.0 ? g[0] > 0.0 : (g[1] != 0.0 ? g[1] > 0.0 : g[2] > 0.0);
    rt.thr[i] = pos ? 0 : 1;
  } else if (lane < 13) {
    // J[r][c] = sum_k Oedge[r][k] * 128 adj(M)[k][c] / vol, M = own edge matrix (lattice)
    const int r = (lane - 4) / 3, c = (lane - 4) % 3;
    double m[3][3];
    for (int rr = 0; rr < 3; ++rr)
      for (int cc = 0; cc < 3; ++cc) m[rr][cc] = ((double)xo[3 * (cc + 1) + rr] - (double)xo[rr]) * kLat;
    const double vol = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                       m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    // column c of adj(M): cofactors of row c of M
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    double adj[3];
    for (int k = 0; k < 3; ++k) {
      const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      adj[k] = m[c1][k1] * m[c2][k2] - m[c1][k2] * m[c2][k1];
    }
    double acc = 0.0;
    for (int k = 0; k < 3; ++k) acc += ((double)xt[3 * (k + 1) + r] - (double)xt[r]) * adj[k];
    rt.J[r][c] = vol > 0.0 ? acc * kLat / vol : 0.0;
  } else if (lane == 13) {
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
      lo[c] = hi[c] = xo[c];
      for (int q = 1; q < 4; ++q) {
        lo[c] = fmin(lo[c], (double)xo[3 * q + c]);
        hi[c] = fmax(hi[c], (double)xo[3 * q + c]);
      }
    }
    int za, zb, ya, yb;
    vox_range((lo[2] + 0.5) * kLat, (hi[2] + 0.5) * kLat, D[2], za, zb);
    vox_range((lo[1] + 0.5) * kLat, (hi[1] + 0.5) * kLat, D[1], ya, yb);
    rt.zlo = za;
    rt.nz = max(0, zb - za + 1);
    rt.ylo = ya;
    rt.ny = max(0, yb - ya + 1);
  }
}

// Candidate rows of the row group that starts at slice k: slice k alone
// (pairs = 0), or slices k and k + 1 for even k (pairs = 1), whose candidate
// rows alternate between the two slices over the union of their row ranges.
// [ya, yb] is slice k's row range; with pairs, lane ^ 1 holds slice k + 1's
// (called on both lanes).  Returns the group's first y in gya and its number of
// candidate rows in cnt (0 on lanes that start no group).
template <int kPairs>
__device__ __forceinline__ void group_rows(int ya, int yb, int k, int nz, int& gya, int& cnt) {
  int lo = ya, hi = yb, m = 1;
  if (kPairs) {
    const int oya = __shfl_xor(ya, 1, 64), oyb = __shfl_xor(yb, 1, 64);
    if (k + 1 < nz) {
      m = 2;
      if (oyb >= oya) {
        lo = yb >= ya ? min(ya, oya) : oya;
        hi = yb >= ya ? max(yb, oyb) : oyb;
      }
    }
  }
  gya = hi >= lo ? lo : 0;
  cnt = (k & kPairs) || k >= nz ? 0 : m * max(0, hi - lo + 1);
}

__device__ void setup_slices(const float* xo, const float* xt, const int D[3], int lane, RasterTet& rt) {
  const int nz = rt.nz;
  if (nz <= kMaxSlices) {
    // candidate rows of slice zlo + lane, prefix-summed over the slices
    int cnt = 0, ya = 0;
    if (lane < nz) {
      float L[4][3];
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 3; ++c) L[q][c] = (xo[3 * q + c] + 0.5f) * 128.f;
      int yb;
      slice_rows(L, rt.zlo + lane, D[1], ya, yb);
      cnt = max(0, yb - ya + 1);
    }
    const int incl = wave_incl_scan(cnt);
    if (lane < nz) {
      rt.rs[lane] = (unsigned short)(incl - cnt);
      rt.y0[lane] = (unsigned short)ya;
    }
    if (lane == 63) {
      rt.rs[min(nz, kMaxSlices)] = (unsigned short)incl;
      rt.nrows = incl;
      rt.sliced = 1;
      rt.pairs = 0;
    }
  } else if (lane == 0) {
    rt.nrows = nz * rt.ny;
    rt.sliced = 0;
    rt.pairs = 0;
  }
  if (lane < 3) {
    const int r = lane;
    rt.P0[r] = (double)xt[r] - (rt.J[r][0] * (double)xo[0] + rt.J[r][1] * (double)xo[1] + rt.J[r][2] * (double)xo[2]);
  }
  wave_sync();
}

// setup_slices on a group of 16 lanes (one DPP row, `sub` = lane within the
// group; all 16 lanes call it) for tetrahedra of few slices: slices in rounds of
// 16, the candidate-row prefix carried from round to round.  Returns the number
// of rows (on every lane of the group).  kPairs: row groups of slice pairs
// (group_rows).
template <int kPairs>
__device__ int setup_slices16(const float* xo, const float* xt, const int D[3], int lane, int sub, RasterTet& rt) {
  constexpr int pairs = kPairs;
  const int nz = rt.nz;
  int nrows;
  if (nz <= kMaxSlices) {
    float L[4][3];
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c) L[q][c] = (xo[3 * q + c] + 0.5f) * 128.f;
    int carry = 0;
    for (int base = 0; base < nz; base += 16) {
      const int k = base + sub;
      int ya = 0, yb = -1;
      if (k < nz) slice_rows(L, rt.zlo + k, D[1], ya, yb);
      int gya, cnt;
      group_rows<kPairs>(ya, yb, k, nz, gya, cnt);
      const int incl = row16_incl_scan(cnt);
      if (k < nz && !(k & pairs)) {
        rt.rs[k >> pairs] = (unsigned short)(carry + incl - cnt);
        rt.y0[k >> pairs] = (unsigned short)gya;
      }
      carry += __shfl(incl, lane | 15, 64);
    }
    nrows = carry;
    if (sub == 0) {
      rt.rs[(nz + pairs) >> pairs] = (unsigned short)carry;
      rt.nrows = carry;
      rt.sliced = 1;
      rt.pairs = pairs;
    }
  } else {
    nrows = nz * rt.ny;
    if (sub == 0) {
      rt.nrows = nrows;
      rt.sliced = 0;
      rt.pairs = 0;
    }
  }
  if (sub < 3) {
    const int r = sub;
    rt.P0[r] = (double)xt[r] - (rt.J[r][0] * (double)xo[0] + rt.J[r][1] * (double)xo[1] + rt.J[r][2] * (double)xo[2]);
  }
  return nrows;
}

// Both parts on one wave.
__device__ void setup_raster(const float* xo, const float* xt, const int D[3], int lane, RasterTet& rt) {
  if (lane < kSetupTasks) setup_task(xo, xt, D, lane, rt);
  wave_sync();
  setup_slices(xo, xt, D, lane, rt);
}

// Exact x-span [x0, x1] (inclusive; empty if x0 > x1) of voxel row (y, z).
__device__ __forceinline__ void row_span(const RasterTet& rt, int y, int z, int Dx, int& x0, int& x1) {
  int lo = 0, hi = Dx - 1;
  for (int i = 0; i < 4; ++i) {
    const double A = rt.A[i];
    // need A x + B >= thr  <=>  A x >= c
    const double c = (double)rt.thr[i] - (rt.C0[i] + rt.CY[i] * y + rt.CZ[i] * z);
    if (A > 0.0) {
      const double q = fmin(fmax(c * rt.rA[i], -2.0), (double)Dx + 1.0);
      int x = (int)ceil(q);
      if (A * (x - 1) >= c)
        x -= 1;
      else if (A * x < c)
        x += 1;
      lo = max(lo, x);
    } else if (A < 0.0) {
      const double q = fmin(fmax(c * rt.rA[i], -2.0), (double)Dx + 1.0);
      int x = (int)floor(q);
      if (A * (x + 1) >= c)
        x += 1;
      else if (A * x < c)
        x -= 1;
      hi = min(hi, x);
    } else if (c > 0.0) {
      lo = Dx;
      hi = -1;
    }
  }
  x0 = lo;
  x1 = hi;
}

// One compacted (non-empty) row: both fields are read from one LDS address.
struct RowRec {
  float4 rec;  // x: own-image linear index minus start (as int bits); yzw: mapped position of the span's first voxel
  int start;   // exclusive prefix of span lengths
  int pad[3];
};

struct WaveRows {
  RowRec row[64];
  int marker[128];  // per voxel slot of the current 128-voxel chunk pair: 1 where a row starts
};

// Computes the spans of rows [64 b, 64 b + 64) of rt, stores the non-empty
// ones compacted (in row order) in wr, and returns the number of voxels.  With
// a slice table, row r is y-major within its row group: y = y0 + (r - rs) of
// the group's slice, or, for a pair of slices, rows alternate between them,
// (y0, z), (y0, z + 1), (y0 + 1, z), ...; every bounding-box row otherwise,
// y = ylo + r % ny.  The linear index of a span's first voxel (x0, y, z) is
// lin = base + z sz + y sy + x0; wr stores lin minus the row's start, or with
// kOwnBytes the byte offset of its value in the bordered z-pair image minus 8
// times the start (the second row of a pair reads the second value of the
// element that holds the first row's voxel, so the two rows share the own
// image's cache lines).  The mapped position of the first voxel is
// P0 + J (x0, y, z) + shift.  *my_start receives the first voxel index of this
// lane's row, or a large negative value if it is empty.  kPairs must equal
// rt.pairs (a compile-time copy, so that the slice-by-slice order pays
// nothing for the other).
template <bool kOwnBytes, int kPairs>
__device__ __forceinline__ int build_rows(const RasterTet& rt, int b, int lane, const int D[3], int sy, int sz,
                                          int base, float shift, WaveRows& wr, int* my_start) {
  const int r0 = b * 64, r = r0 + lane;
  int len = 0, lin = 0;
  float bx = 0.f, by = 0.f, bz = 0.f;
  int y, z, h = 0;
  if (rt.sliced) {
    // lane k holds row group k's first candidate row and first y; row r lies
    // in the last group that starts at or before r: the group of the unit's
    // first row, advanced over the groups that start inside the unit (in order)
    const int nz = rt.nz, ng = (nz + kPairs) >> kPairs;
    const int rsk = lane < ng ? (int)rt.rs[lane] : 0x7fffffff;
    const int y0k = lane < ng ? (int)rt.y0[lane] : 0;
    // row r of group k (uniform), which starts at row s with y = ys
    auto place = [&](int k, int s, int ys) {
      const int rr = r - s;
      if (kPairs) {
        const int two = 2 * k + 1 < nz ? 1 : 0;  // the group is a pair of slices
        h = rr & two;
        y = ys + (rr >> two);
        z = rt.zlo + 2 * k + h;
      } else {
        y = ys + rr;
        z = rt.zlo + k;
      }
    };
    const int jb = __popcll(__ballot(rsk <= r0)) - 1;  // rs[0] = 0
    place(jb, __builtin_amdgcn_readlane(rsk, jb), __builtin_amdgcn_readlane(y0k, jb));
    unsigned long long inside = __ballot(rsk > r0 && rsk < r0 + 64);
    while (inside) {
      const int k = __builtin_ctzll(inside);
      inside &= inside - 1;
      const int s = __builtin_amdgcn_readlane(rsk, k);
      if (r >= s) place(k, s, __builtin_amdgcn_readlane(y0k, k));
    }
  } else {
    y = rt.ylo + r % rt.ny;
    z = rt.zlo + r / rt.ny;
  }
  if (r < rt.nrows) {
    int x0, x1;
    row_span(rt, y, z, D[0], x0, x1);
    if (x1 >= x0) {
      len = x1 - x0 + 1;
      lin = base + z * sz + y * sy + x0;
      if (kOwnBytes) lin = (lin - h * sz) * 8 + 4 * h;
      const double v[3] = {(double)x0, (double)y, (double)z};
      bx = (float)(rt.P0[0] + rt.J[0][0] * v[0] + rt.J[0][1] * v[1] + rt.J[0][2] * v[2] + shift);
      by = (float)(rt.P0[1] + rt.J[1][0] * v[0] + rt.J[1][1] * v[1] + rt.J[1][2] * v[2] + shift);
      bz = (float)(rt.P0[2] + rt.J[2][0] * v[0] + rt.J[2][1] * v[1] + rt.J[2][2] * v[2] + shift);
    }
  }
  const int incl = wave_incl_scan(len);
  const int start = incl - len;
  const unsigned long long ne = __ballot(len > 0);
  const int slot = __builtin_amdgcn_mbcnt_hi((unsigned)(ne >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)ne, 0u));
  wave_sync();
  if (len > 0) {
    wr.row[slot].start = start;
    wr.row[slot].rec = make_float4(__int_as_float(kOwnBytes ? lin - 8 * start : lin - start), bx, by, bz);
  }
  wave_sync();
  *my_start = len > 0 ? start : -(1 << 30);
  return __builtin_amdgcn_readlane(incl, 63);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const float* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, bytes, 0x00020000);
}

typedef float float4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4v load4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float4v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

__device__ __forceinline__ float load1(__amdgpu_buffer_rsrc_t r, int voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}

// Per-wave constants of the sampled (other) image.  Images use the bordered
// z-pair layout: element (x', y', z') holds the values at (x'-1, y'-1, z'-1)
// and (x'-1, y'-1, z'), border-replicated, so one 16-byte load at element
// (ix, iy, iz) returns the taps (x, z), (x, z+1), (x+1, z), (x+1, z+1) of the
// cell of shifted position q = p + 1 with ix = floor(q_x) etc.
struct SampleCtx {
  __amdgpu_buffer_rsrc_t own, oth;  // bordered image buffers
  int sx8, sxy8;                    // byte strides of y and z
  float tau;
};

// The 8 trilinear taps of the sampled image around shifted position
// (px, py, pz) = p + 1, p in [-0.5, D-0.5] up to rounding: truncation is floor,
// and the replicated border stands in for clamping p to [0, D-1].
struct Taps {
  float4v ty0, ty1;  // (x,z) (x,z+1) (x+1,z) (x+1,z+1) at y and at y+1
  float fx, fy, fz;
};

__device__ __forceinline__ Taps load_taps(const SampleCtx& c, float px, float py, float pz) {
  Taps t;
  const int ix = (int)px, iy = (int)py, iz = (int)pz;
  t.fx = __builtin_amdgcn_fractf(px);
  t.fy = __builtin_amdgcn_fractf(py);
  t.fz = __builtin_amdgcn_fractf(pz);
  const int voff = (int)(__umul24((unsigned)iy, (unsigned)c.sx8) + (__umul24((unsigned)iz, (unsigned)c.sxy8) + ((unsigned)ix << 3)));
  t.ty0 = load4(c.oth, voff, 0);
  t.ty1 = load4(c.oth, voff, c.sx8);
  return t;
}

// Sec. 2.3.1 contribution of a voxel pair: squared intensity difference, and
// the maximal difference 1 where an empty voxel meets a non-empty one; the
// empty indicator of the sampled position is interpolated like the intensity.
__device__ __forceinline__ float contrib_of(const SampleCtx& c, float a, const Taps& tp) {
  const float4v ty0 = tp.ty0, ty1 = tp.ty1;
  const float fx = tp.fx, fy = tp.fy, fz = tp.fz;
  struct {
    float x, y;
  } t00{ty0.x, ty0.z}, t10{ty1.x, ty1.z}, t01{ty0.y, ty0.w}, t11{ty1.y, ty1.w};
  const float tau = c.tau;
  const float i00 = fmaf(fx, t00.y - t00.x, t00.x), i10 = fmaf(fx, t10.y - t10.x, t10.x);
  const float i01 = fmaf(fx, t01.y - t01.x, t01.x), i11 = fmaf(fx, t11.y - t11.x, t11.x);
  const float i0 = fmaf(fy, i10 - i00, i00), i1 = fmaf(fy, i11 - i01, i01);
  const float b = fmaf(fz, i1 - i0, i0);
  // empty indicators of the 8 taps as wave masks (combined in scalar registers)
  constexpr int kOLE = 5;  // ordered less-or-equal
  const unsigned long long m000 = __builtin_amdgcn_fcmpf(t00.x, tau, kOLE), m100 = __builtin_amdgcn_fcmpf(t00.y, tau, kOLE);
  const unsigned long long m010 = __builtin_amdgcn_fcmpf(t10.x, tau, kOLE), m110 = __builtin_amdgcn_fcmpf(t10.y, tau, kOLE);
  const unsigned long long m001 = __builtin_amdgcn_fcmpf(t01.x, tau, kOLE), m101 = __builtin_amdgcn_fcmpf(t01.y, tau, kOLE);
  const unsigned long long m011 = __builtin_amdgcn_fcmpf(t11.x, tau, kOLE), m111 = __builtin_amdgcn_fcmpf(t11.y, tau, kOLE);
  const unsigned long long all = m000 & m100 & m010 & m110 & m001 & m101 & m011 & m111;
  const unsigned long long any = m000 | m100 | m010 | m110 | m001 | m101 | m011 | m111;
  const bool ea = a <= tau;
  const float d = a - b;
  // where the 8 taps of every lane agree, the interpolated indicator is the
  // first tap's: m is 0 or 1 and the contribution is d^2 or 1 (the values of
  // the general formula below)
  float res = ea != (t00.x <= tau) ? 1.f : d * d;
  if (any & ~all) {  // some lane has taps on both sides of tau: interpolate its indicator
    const float e000 = t00.x <= tau ? 1.f : 0.f, e100 = t00.y <= tau ? 1.f : 0.f;
    const float e010 = t10.x <= tau ? 1.f : 0.f, e110 = t10.y <= tau ? 1.f : 0.f;
    const float e001 = t01.x <= tau ? 1.f : 0.f, e101 = t01.y <= tau ? 1.f : 0.f;
    const float e011 = t11.x <= tau ? 1.f : 0.f, e111 = t11.y <= tau ? 1.f : 0.f;
    const float m00 = fmaf(fx, e100 - e000, e000), m10 = fmaf(fx, e110 - e010, e010);
    const float m01 = fmaf(fx, e101 - e001, e001), m11 = fmaf(fx, e111 - e011, e011);
    const float m0 = fmaf(fy, m10 - m00, m00), m1 = fmaf(fy, m11 - m01, m01);
    const float eb = fmaf(fz, m1 - m0, m0);
    const float m = fabsf((ea ? 1.f : 0.f) - eb);
    res = fmaf(1.f - m, d * d, m);
  }
  return res;
}

// Samples voxels q0 + lane (row r0) and q0 + 64 + lane (row r1) of the
// compacted rows and adds their contributions to the lane's compensated sum.
// Both samples' loads are issued before either is used.  With TAIL, slots
// past the last voxel repeat the last voxel (same row) and are weighted 0.
template <bool TAIL>
__device__ __forceinline__ void sweep_pair(const WaveRows& wr, const SampleCtx& sc, int q0, int nvox, int lane, int r0,
                                           int r1, float jx, float jy, float jz, float& sum, float& comp) {
  const int qa = q0 + lane, qb = qa + 64;
  const int ea = TAIL ? min(qa, nvox - 1) : qa, eb = TAIL ? min(qb, nvox - 1) : qb;
  const RowRec ra = wr.row[r0], rb = wr.row[r1];
  const float foa = (float)(ea - ra.start), fob = (float)(eb - rb.start);
  const float ava = load1(sc.own, __float_as_int(ra.rec.x) + (ea << 3));
  const Taps ta = load_taps(sc, fmaf(jx, foa, ra.rec.y), fmaf(jy, foa, ra.rec.z), fmaf(jz, foa, ra.rec.w));
  const float avb = load1(sc.own, __float_as_int(rb.rec.x) + (eb << 3));
  const Taps tb = load_taps(sc, fmaf(jx, fob, rb.rec.y), fmaf(jy, fob, rb.rec.z), fmaf(jz, fob, rb.rec.w));
  const float ca = contrib_of(sc, ava, ta);
  const float cb = contrib_of(sc, avb, tb);
  const float c = TAIL ? (qa < nvox ? ca : 0.f) + (qb < nvox ? cb : 0.f) : ca + cb;
  const float y = c - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// The last chunk of a row batch when at most 64 voxels are left: voxel
// q0 + lane only, slots past the last voxel repeat it and are weighted 0.
__device__ __forceinline__ void sweep_one(const WaveRows& wr, const SampleCtx& sc, int q0, int nvox, int lane, int r0,
                                          float jx, float jy, float jz, float& sum, float& comp) {
  const int qa = q0 + lane;
  const int ea = min(qa, nvox - 1);
  const RowRec ra = wr.row[r0];
  const float foa = (float)(ea - ra.start);
  const float ava = load1(sc.own, __float_as_int(ra.rec.x) + (ea << 3));
  const Taps ta = load_taps(sc, fmaf(jx, foa, ra.rec.y), fmaf(jy, foa, ra.rec.z), fmaf(jz, foa, ra.rec.w));
  const float ca = contrib_of(sc, ava, ta);
  const float c = qa < nvox ? ca : 0.f;
  const float y = c - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// Length in mm of b - a (voxel units, float or double components; float
// components are widened exactly).
template <class A, class B>
__device__ __forceinline__ double len_mm(const double sp[3], const A a[3], const B b[3]) {
  const double dx = ((double)a[0] - (double)b[0]) * sp[0], dy = ((double)a[1] - (double)b[1]) * sp[1],
               dz = ((double)a[2] - (double)b[2]) * sp[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

// Sec. 2.3.2: deformation term of one tetrahedron (edges weighted 1/k_e, plus
// the spoke from each vertex to the centroid of its opposite face); squared
// length differences in mm between the two grids.
__device__ double deformation_term(const DevProblem& pr, int t, const float S[4][3], const float Tg[4][3]) {
  const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {1, 2, 3, 2, 3, 3};
  double acc = 0.0;
  for (int e = 0; e < 6; ++e) {
    const double d = len_mm(pr.sp, S[pa[e]], S[pb[e]]) - len_mm(pr.sp, Tg[pa[e]], Tg[pb[e]]);
    acc += pr.tet_w[6 * t + e] * d * d;
  }
  for (int q = 0; q < 4; ++q) {
    double cs[3] = {0, 0, 0}, ct[3] = {0, 0, 0};
    for (int r = 0; r < 4; ++r)
      if (r != q)
        for (int c = 0; c < 3; ++c) {
          cs[c] += (double)S[r][c];
          ct[c] += (double)Tg[r][c];
        }
    for (int c = 0; c < 3; ++c) {
      cs[c] /= 3.0;
      ct[c] /= 3.0;
    }
    const double d = len_mm(pr.sp, S[q], cs) - len_mm(pr.sp, Tg[q], ct);
    acc += d * d;
  }
  return acc;
}

// Sec. 2.3.3: guidance points of image g inside tetrahedron (grid g) are mapped
// into the other image and contribute the squared mm distance to the nearest
// point of the same correspondence there.
__device__ double guidance_term(const DevProblem& pr, const float V[2][4][3]) {
  double acc = 0.0;
  for (int g = 0; g < 2; ++g) {
    if (pr.ng[g] == 0) continue;
    double L[4][3];  // lattice coordinates of grid g's vertices (exact)
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c) L[q][c] = ((double)V[g][q][c] + 0.5) * kLat;
    const double vol = orient(L[0], L[1], L[2], L[3]);
    if (!(vol > 0.0)) continue;
    Faces f;
    make_faces(L, f);
    for (int i = 0; i < pr.ng[g]; ++i) {
      const double U[3] = {pr.gpt[g][3 * i], pr.gpt[g][3 * i + 1], pr.gpt[g][3 * i + 2]};
      double o[4];
      if (!inside(f, U, o)) continue;
      double x[3] = {0, 0, 0};
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 3; ++c) x[c] += o[q] / vol * (double)V[1 - g][q][c];
      double best = INFINITY;
      const int corr = pr.gcorr[g][i];
      for (int j = 0; j < pr.ng[1 - g]; ++j) {
        if (pr.gcorr[1 - g][j] != corr) continue;
        double r[3];
        for (int c = 0; c < 3; ++c) r[c] = pr.gpt[1 - g][3 * j + c] / kLat - 0.5;
        best = fmin(best, len_mm(pr.sp, x, r));
      }
      if (best < INFINITY) acc += best * best;
    }
  }
  return acc;
}

// ------------------------------------------------------------ LDS layout

struct EvalLayout {
  size_t tet, xyz, units, part, waves, rts, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline EvalLayout eval_layout(int maxA, int nver) {
  EvalLayout L;
  size_t o = 0;
  L.tet = o;
  o = align16(o + sizeof(int) * maxA);
  L.xyz = o;  // [nver][maxA][2][4][3] float
  o = align16(o + sizeof(float) * 24 * (size_t)nver * maxA);
  L.units = o;  // [nver*2*maxA + 1] int (unit counts, then exclusive prefix)
  o = align16(o + sizeof(int) * (2 * (size_t)nver * maxA + 1));
  L.part = o;  // [nver*2*maxA][kWaves] double
  o = align16(o + sizeof(double) * kWaves * 2 * (size_t)nver * maxA);
  L.waves = o;  // [kWaves] WaveRows
  o = align16(o + sizeof(WaveRows) * kWaves);
  L.rts = o;  // [nver*2*maxA] RasterTet, one per (version, direction, tetrahedron)
  o = align16(o + sizeof(RasterTet) * 2 * (size_t)nver * maxA);
  L.total = o;
  return L;
}

// exclusive scan of n ints in LDS by wave 0 (n entries, writes n+1 with total)
__device__ void lds_exclusive_scan(int* v, int n, int tid) {
  if (tid < 64) {
    int carry = 0;
    for (int base = 0; base < n; base += 64) {
      const int x = base + tid < n ? v[base + tid] : 0;
      const int incl = wave_incl_scan(x);
      if (base + tid < n) v[base + tid] = carry + incl - x;
      carry += __builtin_amdgcn_readlane(incl, 63);
    }
    if (tid == 0) v[n] = carry;
  }
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniformf(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Source of vertex vid's coordinates in grid gr for version v (0 = candidate,
// 1 = current) of solution s, group g.
__device__ __forceinline__ const float* vertex_src(const EvalArgs& a, int s, int g, int v, int vid, int gr) {
  const float* src = a.X + (((size_t)s * 2 + gr) * a.pr.P + vid) * 3;
  if (v == 0 && a.partial) {
    const int pb = a.fos_off[g], pe = a.fos_off[g + 1], ncand = a.fos_off[a.G];
    for (int k = pb; k < pe; ++k)
      if (a.fos_pts[k] == vid) src = a.cand + (((size_t)s * ncand + k) * 2 + gr) * 3;
  }
  return src;
}

__device__ __forceinline__ int group_size(const EvalArgs& a, int g) {
  return a.partial ? a.aff_cnt[g] : min(kFullChunk, a.pr.T - g * kFullChunk);
}

__device__ __forceinline__ int group_tet(const EvalArgs& a, int g, int i) {
  return a.partial ? a.aff[(size_t)g * a.maxA + i] : g * kFullChunk + i;
}

// ------------------------------------------------------------ voxel sweep kernel

// Dissimilarity of every (version, tetrahedron) of one chunk of at most
// a.pchunk affected tetrahedra (partial evaluation) or of one group of
// kFullChunk tetrahedra (full evaluation) of one solution: writes
// simws[((s*G + g)*nver + v)*maxA + i].  Workgroups are numbered (group, chunk,
// solution) with the solution fastest, so the workgroups resident on an XCD
// sweep the same few tetrahedra of many solutions and share their image
// region in L2; with `interleave` the groups follow interleaved_group's order.
// Partial mode also writes the chunk's constraint flags and
// candidate voxel count to cflags / ccount [S][G][nchunk]; k_finish combines
// them.  ROWS: the row order, 0 slice by slice, 1 in slice pairs (both fixed
// at compile time), 2 a.row_pairs read at run time (a batch of problems with
// both orders).
template <int PARTIAL, int ROWS>
__device__ __forceinline__ void sweep_body(const EvalArgs& a, int logical, unsigned char* smem, bool interleave) {
  double* __restrict__ simws = a.simws;
  const DevProblem& pr = a.pr;
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
  const int nchunk = PARTIAL ? a.nchunk : 1;
  const int gl = logical / (a.S * nchunk), rem = logical - gl * (a.S * nchunk);
  // g and the counts below are the same on every lane; saying so keeps the
  // values derived from them (the direction of an entry, hence the image
  // buffer a load reads) in scalar registers
  const int g = uniform(PARTIAL && a.order ? a.order[gl] : (interleave ? interleaved_group(gl, a.G) : gl));
  const int c = rem / a.S, s = rem - c * a.S;
  const int nver = a.nver;
  const EvalLayout Lay = eval_layout(kMaxChunk, nver);
  int* s_tet = (int*)(smem + Lay.tet);
  float* s_xyz = (float*)(smem + Lay.xyz);
  int* s_units = (int*)(smem + Lay.units);
  double* s_part = (double*)(smem + Lay.part);
  WaveRows* s_rows = (WaveRows*)(smem + Lay.waves);
  RasterTet* s_rts = (RasterTet*)(smem + Lay.rts);
  __shared__ unsigned s_flags;
  __shared__ unsigned s_count[kWaves];

  // this chunk's tetrahedra: slots [i0, i0 + na) of the group
  const int na_all = uniform(PARTIAL ? a.aff_cnt[g] : min(kFullChunk, pr.T - g * kFullChunk));
  const int i0 = c * (PARTIAL ? a.pchunk : kFullChunk);
  if (na_all <= i0) return;  // malformed element (count -1) or no tetrahedra in this chunk: k_finish sets the flags
  if (PARTIAL && a.mask && a.mask[(size_t)s * a.G + g] == 0) return;  // not requested
  const int na = min(PARTIAL ? a.pchunk : kFullChunk, na_all - i0);
  if (tid == 0) s_flags = 0u;
  if (tid < kWaves) s_count[tid] = 0u;
  for (int i = tid; i < na; i += kWG) s_tet[i] = group_tet(a, g, i0 + i);
  __syncthreads();

  // vertex coordinates of every (version, tetrahedron, grid, vertex) and the
  // per-point constraint bits (lattice, box, border pins) of the candidate
  for (int e = tid; e < nver * na * 8; e += kWG) {
    const int v = e / (na * 8), r = e - v * na * 8;
    const int i = r >> 3, gr = (r >> 2) & 1, q = r & 3;
    const int vid = ((const int*)&pr.tets[s_tet[i]])[q];
    const float* src = vertex_src(a, s, g, v, vid, gr);
    float* dst = s_xyz + ((size_t)(v * na + i) * 8 + gr * 4 + q) * 3;
    unsigned fl = 0u;
    const int idx[3] = {vid % pr.n[0], (vid / pr.n[0]) % pr.n[1], vid / (pr.n[0] * pr.n[1])};
    for (int c = 0; c < 3; ++c) {
      const float x = src[c];
      dst[c] = x;
      double u;
      const unsigned fc = lattice_of(x, pr.D[c], u);
      fl |= fc;
      if (!fc && ((idx[c] == 0 && u != 0.0) || (idx[c] == pr.n[c] - 1 && u != kLat * pr.D[c]))) fl |= DSM_FLAG_BORDER;
    }
    if (v == 0 && PARTIAL && fl) atomicOr(&s_flags, fl);
  }
  __syncthreads();

  // set-up of every (version, direction, tetrahedron) entry: validity,
  // orientation flag, rasterisation parameters and the number of 64-row
  // units.  Direction 0 = target voxels mapped into the source (forward), 1 =
  // source voxels into the target.  Entry e's own-grid vertices are at
  // entry_xyz(e) + 12 own, the other grid's at + 12 (1 - own).
  const int nent = nver * 2 * na;
  auto entry_xyz = [&](int e, int& own) {
    const int v = e / (2 * na), r = e - v * 2 * na, dir = r / na, i = r - dir * na;
    own = 1 - dir;
    return s_xyz + (size_t)(v * na + i) * 24;
  };
  // validity, 32 threads per entry: the 24 coordinates on the lattice, then
  // the orientation of the own-grid tetrahedron; s_units[e] = 1 if it is set up
  for (int t = tid; t < nent * 32; t += kWG) {
    const int e = t >> 5, j = t & 31;
    int own;
    const float* xyz = entry_xyz(e, own);
    double dummy;
    const bool bad = j < 24 && lattice_of(xyz[j], pr.D[j % 3], dummy) != 0u;
    const unsigned long long bm = __ballot(bad) >> (lane & 32);  // this entry's half of the wave
    const bool bad_own = (bm >> (own * 12)) & 0xfffull, bad_oth = (bm >> ((1 - own) * 12)) & 0xfffull;
    int ok = 0;
    if (!bad_own) {
      double L[4][3];
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 3; ++c) L[q][c] = ((double)xyz[own * 12 + q * 3 + c] + 0.5) * kLat;
      const double vol = orient(L[0], L[1], L[2], L[3]);
      if (vol > 0.0 && !bad_oth)
        ok = 1;
      else if (!(vol > 0.0) && e < 2 * na && PARTIAL && j == 0)  // candidate version only
        atomicOr(&s_flags, own == 0 ? DSM_FLAG_INV_MOVING : DSM_FLAG_INV_FIXED);
    }
    if (j == 0) s_units[e] = ok;
  }
  __syncthreads();
  // face functions, affine map and bounding box: 16 threads per entry
  for (int t = tid; t < nent * 16; t += kWG) {
    const int e = t >> 4, k = t & 15;
    if (k < kSetupTasks && s_units[e]) {
      int own;
      const float* xyz = entry_xyz(e, own);
      setup_task(xyz + own * 12, xyz + (1 - own) * 12, pr.D, k, s_rts[e]);
    }
  }
  __syncthreads();
  // slice tables, 16 lanes per entry, and the units
  for (int e0 = wave * 4; e0 < nent; e0 += kWaves * 4) {
    const int e = e0 + (lane >> 4), sub = lane & 15;
    int nunits = 0;
    if (e < nent && s_units[e]) {
      int own;
      const float* xyz = entry_xyz(e, own);
      const float *xo = xyz + own * 12, *xt = xyz + (1 - own) * 12;
      const int nrows = ROWS == 2 ? (a.row_pairs ? setup_slices16<1>(xo, xt, pr.D, lane, sub, s_rts[e])
                                                 : setup_slices16<0>(xo, xt, pr.D, lane, sub, s_rts[e]))
                                  : setup_slices16<ROWS>(xo, xt, pr.D, lane, sub, s_rts[e]);
      nunits = (nrows + 63) >> 6;
    }
    wave_sync();
    if (e < nent && sub == 0) s_units[e] = nunits;
  }
  for (int e = tid; e < nent * kWaves; e += kWG) s_part[e] = 0.0;
  __syncthreads();
  lds_exclusive_scan(s_units, nent, tid);
  __syncthreads();
  const int total_units = uniform(s_units[nent]);

  // ---- voxel sweep
  SampleCtx sc;
  sc.sx8 = 8 * pr.ex;
  sc.sxy8 = 8 * pr.exy;
  sc.tau = pr.tau;
  const int own_base = pr.exy + pr.ex + 1;  // element of voxel (0, 0, 0)
  const __amdgpu_buffer_rsrc_t rs[2] = {image_rsrc(pr.img[0], pr.img_bytes), image_rsrc(pr.img[1], pr.img_bytes)};
  WaveRows& wr = s_rows[wave];
  const RasterTet* rtp = s_rts;
  int cur = -1;
  float jx = 0.f, jy = 0.f, jz = 0.f;
  unsigned counted = 0u;
  float sum = 0.f, comp = 0.f;  // compensated per-lane sum of the current (version, direction, tetrahedron)
  // each wave takes one contiguous range of units, so it sets up few tetrahedra
  const int u_begin = (wave * total_units) / kWaves, u_end = ((wave + 1) * total_units) / kWaves;
  for (int u = u_begin; u < u_end; ++u) {
    int e = cur < 0 ? 0 : cur;
    while (uniform(s_units[e + 1]) <= u) ++e;
    e = uniform(e);
    if (e != cur) {
      if (cur >= 0) {
        const double tot = wave_sum((double)sum - (double)comp);
        if (lane == 0) s_part[(size_t)cur * kWaves + wave] += tot;
        sum = comp = 0.f;
      }
      cur = e;
      const int r = e - (e / (2 * na)) * 2 * na, dir = r / na;
      const int own = 1 - dir;
      rtp = s_rts + e;
      jx = uniformf((float)rtp->J[0][0]);
      jy = uniformf((float)rtp->J[1][0]);
      jz = uniformf((float)rtp->J[2][0]);
      sc.own = own ? rs[1] : rs[0];
      sc.oth = own ? rs[0] : rs[1];
    }
    const int b = u - uniform(s_units[cur]);
    int my_start;
    const int nvox = uniform(ROWS == 2 ? (rtp->pairs ? build_rows<true, 1>(*rtp, b, lane, pr.D, pr.ex, pr.exy, own_base, 1.0f, wr, &my_start)
                                                     : build_rows<true, 0>(*rtp, b, lane, pr.D, pr.ex, pr.exy, own_base, 1.0f, wr, &my_start))
                                        : build_rows<true, ROWS>(*rtp, b, lane, pr.D, pr.ex, pr.exy, own_base, 1.0f, wr, &my_start));
    int carry = 0;  // non-empty rows that start before the current chunk
    for (int q0 = 0; q0 < nvox; q0 += 128) {
      // voxels q0 + lane and q0 + 64 + lane: rows starting in this pair of
      // chunks are marked, then counted below each slot with a ballot
      wr.marker[lane] = 0;
      wr.marker[64 + lane] = 0;
      wave_sync();
      const unsigned pos = (unsigned)(my_start - q0);
      if (pos < 128u) wr.marker[pos] = 1;
      wave_sync();
      const int mk0 = wr.marker[lane], mk1 = wr.marker[64 + lane];
      const unsigned long long M0 = __ballot(mk0 != 0), M1 = __ballot(mk1 != 0);
      const int r0 = carry + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(M0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)M0, 0u)) +
                     mk0 - 1;
      carry += __popcll(M0);
      const int r1 = carry + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(M1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)M1, 0u)) +
                     mk1 - 1;
      carry += __popcll(M1);
      if (q0 + 128 <= nvox)
        sweep_pair<false>(wr, sc, q0, nvox, lane, r0, r1, jx, jy, jz, sum, comp);
      else if (q0 + 64 >= nvox)
        sweep_one(wr, sc, q0, nvox, lane, r0, jx, jy, jz, sum, comp);
      else
        sweep_pair<true>(wr, sc, q0, nvox, lane, r0, r1, jx, jy, jz, sum, comp);
    }
    if (cur < 2 * na) counted += (unsigned)nvox;  // version 0 (candidate) voxels
  }
  if (cur >= 0) {
    const double tot = wave_sum((double)sum - (double)comp);
    if (lane == 0) s_part[(size_t)cur * kWaves + wave] += tot;
  }
  if (lane == 0) s_count[wave] = counted;
  __syncthreads();

  double* out = simws + ((size_t)s * a.G + g) * nver * a.maxA + i0;
  for (int e = tid; e < nver * na; e += kWG) {
    const int v = e / na, i = e - v * na;
    double sim = 0.0;
    for (int dir = 0; dir < 2; ++dir)
      for (int w = 0; w < kWaves; ++w) sim += s_part[((size_t)(v * 2 + dir) * na + i) * kWaves + w];
    out[(size_t)v * a.maxA + i] = sim;
  }
  if (PARTIAL && tid == 0) {
    const size_t ci = ((size_t)s * a.G + g) * nchunk + c;
    a.cflags[ci] = s_flags;
    unsigned tot = 0u;
    for (int w = 0; w < kWaves; ++w) tot += s_count[w];
    a.ccount[ci] = tot;
  }
}

template <int PARTIAL, int ROWS>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_sweep(EvalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  sweep_body<PARTIAL, ROWS>(a, xcd_logical(blockIdx.x, a.S * a.G * (PARTIAL ? a.nchunk : 1)), smem, PARTIAL != 0);
}

// Several problems in one launch.  Each job's workgroup range is split into 8
// equal contiguous parts, part x running on XCD x (hardware workgroup ids go
// round-robin over the XCDs): xcd_off[j] is the first per-XCD slot of job j,
// and a job with n workgroups takes ceil(n / 8) slots on every XCD, the
// surplus slots exiting at once.  So every XCD gets an eighth of every job
// (jobs of very different tetrahedron sizes would otherwise load the XCDs
// unevenly), and within a part the workgroups of one element's solutions stay
// together.  Elements follow interleaved_group's order within a job.
// Arguments read through the job table take more registers than kernel
// arguments; the 7-wave target (at most 72 VGPRs) ran small problems 5 %
// faster than 6 waves.  ROWS as for sweep_body.
template <int ROWS>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_sweep_batch(
    const EvalArgs* __restrict__ jobs, const int* __restrict__ xcd_off, int n_jobs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
  int j = 0;
  while (j + 1 < n_jobs && xcd_off[j + 1] <= k) ++j;
  j = uniform(j);
  const EvalArgs& a = jobs[j];
  const int n8 = uniform(xcd_off[j + 1] - xcd_off[j]);
  const int logical = x * n8 + (k - uniform(xcd_off[j]));
  if (logical >= a.S * a.G * a.nchunk) return;
  sweep_body<1, ROWS>(a, logical, smem, true);
}

// ------------------------------------------------------------ finishing kernel

// Adds the deformation and guidance terms (FP64, per tetrahedron) to the swept
// dissimilarity, writes per-tetrahedron terms, and in partial mode the
// normalised sums over each group in ascending tetrahedron order.  One group
// of kFinishLanes lanes per (group, solution) pair, one lane per affected
// tetrahedron (kFinishLanes at a time): a star averages 16 tetrahedra, so
// 8-lane groups keep the FP64 lanes busy over about two rounds (measured
// against 16 and 32 lanes per pair: 0.86, 1.07 and 1.7 ms per 512x512x100 step).
__device__ __forceinline__ void finish_body(const EvalArgs& a, int logical, int lane) {
  const double* __restrict__ simws = a.simws;
  const DevProblem& pr = a.pr;
  const int g = logical / a.S, s = logical - g * a.S;
  const int na = group_size(a, g);
  const size_t oi = (size_t)s * a.G + g;
  if (na < 0 || (a.partial && a.mask && a.mask[oi] == 0)) {
    if (lane < 3) {
      a.part_new[oi * 3 + lane] = 0.0;
      a.part_old[oi * 3 + lane] = 0.0;
    }
    if (a.partial && lane == 0) {
      a.flags[oi] = na < 0 ? DSM_FLAG_BAD_FOS : DSM_FLAG_SKIPPED;
      if (a.vcount) a.vcount[oi] = 0u;
    }
    return;
  }
  if (a.partial && lane == 0) {  // combine the chunks' flags and voxel counts in chunk order
    unsigned fl = 0u, cnt = 0u;
    for (int c = 0; c * a.pchunk < na; ++c) {
      fl |= a.cflags[oi * a.nchunk + c];
      cnt += a.ccount[oi * a.nchunk + c];
    }
    a.flags[oi] = fl;
    if (a.vcount) a.vcount[oi] = cnt;
  }
  // one lane per affected tetrahedron; the per-tetrahedron terms are summed
  // over the lane group in a fixed butterfly order
  const double* sims = simws + oi * a.nver * a.maxA;
  double accn[3] = {0, 0, 0}, acco[3] = {0, 0, 0};
  for (int base = 0; base < na; base += kFinishLanes) {
    const int i = base + lane;
    double tn[3] = {0, 0, 0}, to[3] = {0, 0, 0};
    for (int v = 0; v < a.nver; ++v) {
      double term[3] = {0, 0, 0};
      if (i < na) {
        const int t = group_tet(a, g, i);
        const int4 tv = pr.tets[t];
        const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
        float V[2][4][3];
        unsigned bad = 0u;
        for (int gr = 0; gr < 2; ++gr)
          for (int q = 0; q < 4; ++q) {
            const float* src = vertex_src(a, s, g, v, vid[q], gr);
            for (int c = 0; c < 3; ++c) {
              double u;
              V[gr][q][c] = src[c];
              bad |= lattice_of(src[c], pr.D[c], u);
            }
          }
        if (!bad) {
          term[0] = sims[(size_t)v * a.maxA + i];
          term[1] = deformation_term(pr, t, V[0], V[1]);
          term[2] = guidance_term(pr, V);
        }
        if (v == 0 && a.terms_out) {
          double* o = a.terms_out + ((size_t)s * pr.T + t) * 3;
          o[0] = term[0];
          o[1] = term[1];
          o[2] = term[2];
        }
      }
      for (int c = 0; c < 3; ++c) (v == 0 ? tn : to)[c] = term[c];
    }
    if (a.partial) {
      if (a.nver == 1 && i < na) {  // current terms from the cache
        const double* src = a.terms_in + ((size_t)s * pr.T + group_tet(a, g, i)) * 3;
        for (int c = 0; c < 3; ++c) to[c] = src[c];
      }
      for (int c = 0; c < 3; ++c) {
        accn[c] += group_sum(tn[c]);
        acco[c] += group_sum(to[c]);
      }
    }
  }
  if (a.partial && lane < 6) {
    const int c = lane % 3;
    if (lane < 3)
      a.part_new[oi * 3 + c] = accn[c] * pr.norm[c];
    else
      a.part_old[oi * 3 + c] = acco[c] * pr.norm[c];
  }
}

// FP64 geometry per lane: the 3-wave target (at most 168 VGPRs, with some
// registers spilled) ran the finish kernels 20 % faster than 2 waves without
// spills.
// Each 64-lane workgroup takes kFinishPairs consecutive pairs.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_finish(EvalArgs a, int n_pairs) {
  const int pair = blockIdx.x * kFinishPairs + (threadIdx.x / kFinishLanes);
  if (pair < n_pairs) finish_body(a, pair, threadIdx.x % kFinishLanes);
}

// Several problems: wg_off [n_jobs + 1] are the jobs' first workgroups, a job
// of n pairs taking ceil(n / kFinishPairs) of them.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_finish_batch(const EvalArgs* __restrict__ jobs, const int* __restrict__ wg_off,
                                                     int n_jobs) {
  int j = 0;
  while (j + 1 < n_jobs && wg_off[j + 1] <= (int)blockIdx.x) ++j;
  const EvalArgs& a = jobs[j];
  const int pair = ((int)blockIdx.x - wg_off[j]) * kFinishPairs + (int)(threadIdx.x / kFinishLanes);
  if (pair < a.S * a.G) finish_body(a, pair, threadIdx.x % kFinishLanes);
}

// ------------------------------------------------------------ small kernels

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Sec. 2.3.4 per point: lattice, box and border pins, both grids.
__global__ void k_fold_points(DevProblem pr, int S, const float* __restrict__ X, uint32_t* flags) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)S * pr.P) return;
  const int s = (int)(e / pr.P), p = (int)(e - (int64_t)s * pr.P);
  const int idx[3] = {p % pr.n[0], (p / pr.n[0]) % pr.n[1], p / (pr.n[0] * pr.n[1])};
  unsigned fl = 0u;
  for (int gr = 0; gr < 2; ++gr)
    for (int c = 0; c < 3; ++c) {
      double u;
      const unsigned fc = lattice_of(X[(((size_t)s * 2 + gr) * pr.P + p) * 3 + c], pr.D[c], u);
      fl |= fc;
      if (!fc && ((idx[c] == 0 && u != 0.0) || (idx[c] == pr.n[c] - 1 && u != kLat * pr.D[c]))) fl |= DSM_FLAG_BORDER;
    }
  if (fl) atomicOr(&flags[s], fl);
}

// Sec. 2.3.4 per tetrahedron: exact orientation in both grids.
__global__ void k_fold_tets(DevProblem pr, int S, const float* __restrict__ X, uint32_t* flags, int* first_bad) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)S * pr.T) return;
  const int s = (int)(e / pr.T), t = (int)(e - (int64_t)s * pr.T);
  const int4 tv = pr.tets[t];
  const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
  unsigned fl = 0u;
  for (int gr = 0; gr < 2; ++gr) {
    double L[4][3];
    unsigned bad = 0u;
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c) bad |= lattice_of(X[(((size_t)s * 2 + gr) * pr.P + vid[q]) * 3 + c], pr.D[c], L[q][c]);
    if (bad) continue;
    if (!(orient(L[0], L[1], L[2], L[3]) > 0.0)) fl |= gr == 0 ? DSM_FLAG_INV_MOVING : DSM_FLAG_INV_FIXED;
  }
  if (fl) {
    atomicOr(&flags[s], fl);
    if (first_bad) atomicMin(&first_bad[s], t);
  }
}

__global__ void k_first_bad_fix(int S, int* first_bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && first_bad[s] == 0x7fffffff) first_bad[s] = -1;
}

// Affected tetrahedra of element f with points fos_pts[b .. e): the sorted
// union of the points' stars, written to out (at most maxA); the count, or -1
// if it would exceed maxA.  One thread, insertion into the sorted prefix: the
// path for elements whose stars hold more than kAffCap entries.
__device__ int affected_serial(const DevProblem& pr, int b, int e, const int* __restrict__ fos_pts, int maxA,
                               int* out) {
  int n = 0;
  for (int k = b; k < e; ++k) {
    const int p = fos_pts[k];
    for (int j = pr.star_off[p]; j < pr.star_off[p + 1]; ++j) {
      const int t = pr.star[j];
      int pos = n;
      while (pos > 0 && out[pos - 1] > t) --pos;
      if (pos > 0 && out[pos - 1] == t) continue;
      if (n >= maxA) return -1;
      for (int m = n; m > pos; --m) out[m] = out[m - 1];
      out[pos] = t;
      ++n;
    }
  }
  return n;
}

constexpr int kAffCap = 1024;  // star entries of one element sorted in LDS

// Affected sets of the FOS elements (Sec. 2.2: the tetrahedra to re-evaluate
// when the element's points move): one wave per element gathers the stars of
// its points into LDS, sorts them (bitonic) and keeps the first of every run
// of equal ids, written in ascending order; aff_cnt[f] = their number, or -1
// for a malformed element or one whose set would exceed maxA.
__global__ __launch_bounds__(64) void k_affected(DevProblem pr, int F, const int* __restrict__ fos_off,
                                                 const int* __restrict__ fos_pts, int max_pts, int maxA, int* aff,
                                                 int* aff_cnt) {
  __shared__ int s_c[kAffCap];
  const int f = blockIdx.x, lane = threadIdx.x;
  const int b = fos_off[f], e = fos_off[f + 1];
  int* out = aff + (size_t)f * maxA;
  bool bad = b < 0 || e < b || e - b > max_pts;
  int total = 0;
  for (int k = b; !bad && k < e; ++k) {
    const int p = fos_pts[k];
    if (p < 0 || p >= pr.P)
      bad = true;
    else
      total += pr.star_off[p + 1] - pr.star_off[p];
  }
  if (bad) {
    if (lane == 0) aff_cnt[f] = -1;
    return;
  }
  if (total > kAffCap) {
    if (lane == 0) aff_cnt[f] = affected_serial(pr, b, e, fos_pts, maxA, out);
    return;
  }
  int base = 0;
  for (int k = b; k < e; ++k) {
    const int p = fos_pts[k], so = pr.star_off[p], n = pr.star_off[p + 1] - so;
    for (int i = lane; i < n; i += 64) s_c[base + i] = pr.star[so + i];
    base += n;
  }
  int n2 = 1;
  while (n2 < total) n2 <<= 1;
  for (int i = total + lane; i < n2; i += 64) s_c[i] = 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < n2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int a = s_c[i], c = s_c[ixj];
          if ((i & k) == 0 ? a > c : a < c) {
            s_c[i] = c;
            s_c[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  // lane l keeps the run starts among entries [l * chunk, (l + 1) * chunk)
  const int chunk = (total + 63) / 64;
  const int lo = min(lane * chunk, total), hi = min(lo + chunk, total);
  int cnt = 0;
  for (int i = lo; i < hi; ++i) cnt += i == 0 || s_c[i] != s_c[i - 1];
  const int incl = wave_incl_scan(cnt);
  const int n_unique = __builtin_amdgcn_readlane(incl, 63);
  if (n_unique > maxA) {
    if (lane == 0) aff_cnt[f] = -1;
    return;
  }
  int pos = incl - cnt;
  for (int i = lo; i < hi; ++i)
    if (i == 0 || s_c[i] != s_c[i - 1]) out[pos++] = s_c[i];
  if (lane == 0) aff_cnt[f] = n_unique;
}

// Full evaluation: fixed-order sum of the per-tetrahedron terms of each solution.
__global__ __launch_bounds__(kWG) void k_full_reduce(DevProblem pr, const double* __restrict__ terms, double* obj) {
  __shared__ double red[3][kWG];
  const int s = blockIdx.x, tid = threadIdx.x;
  double acc[3] = {0, 0, 0};
  for (int t = tid; t < pr.T; t += kWG)
    for (int c = 0; c < 3; ++c) acc[c] += terms[((size_t)s * pr.T + t) * 3 + c];
  for (int c = 0; c < 3; ++c) red[c][tid] = acc[c];
  __syncthreads();
  for (int w = kWG / 2; w >= 1; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + w];
    __syncthreads();
  }
  if (tid < 3) obj[(size_t)s * 3 + tid] = red[tid][0] * pr.norm[tid];
}

// Owner map of one grid (test hook): every voxel of every tetrahedron's exact
// voxel set claims its owner entry.
__global__ __launch_bounds__(kWG) void k_owner(DevProblem pr, const float* __restrict__ Xg, int* owner, int* overlap) {
  __shared__ WaveRows rows[kWaves];
  __shared__ RasterTet rts[kWaves];
  __shared__ float xo[12];
  const int t = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int4 tv = pr.tets[t];
  const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
  double L[4][3];
  unsigned bad = 0u;
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 3; ++c) bad |= lattice_of(Xg[(size_t)vid[q] * 3 + c], pr.D[c], L[q][c]);
  if (bad || !(orient(L[0], L[1], L[2], L[3]) > 0.0)) return;
  if (threadIdx.x < 12) xo[threadIdx.x] = Xg[(size_t)vid[threadIdx.x / 3] * 3 + threadIdx.x % 3];
  __syncthreads();
  RasterTet& rt = rts[wave];
  setup_raster(xo, xo, pr.D, lane, rt);
  const int nb = (rt.nrows + 63) >> 6;
  for (int b = wave; b < nb; b += kWaves) {
    WaveRows& wr = rows[wave];
    int my_start;
    const int nvox = build_rows<false, 0>(rt, b, lane, pr.D, pr.D[0], pr.DxDy, 0, 0.0f, wr, &my_start);
    int carry = 0;
    for (int q0 = 0; q0 < nvox; q0 += 64) {
      wr.marker[lane] = 0;
      wave_sync();
      const unsigned pos = (unsigned)(my_start - q0);
      if (pos < 64u) wr.marker[pos] = 1;
      wave_sync();
      const int mk = wr.marker[lane];
      const unsigned long long M = __ballot(mk != 0);
      const int r = carry + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(M >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)M, 0u)) +
                    mk - 1;
      carry += __popcll(M);
      const int q = q0 + lane;
      if (q < nvox) {
        const int idx = __float_as_int(wr.row[r].rec.x) + q;
        const int prev = atomicCAS(&owner[idx], -1, t);
        if (prev != -1) atomicAdd(overlap, 1);
      }
    }
  }
}

// Value of voxel (x, y, z) of a bordered z-pair image: the second half of
// element (x + 1, y + 1, z).
__device__ __forceinline__ double raw_voxel(const float* img, int ex, int exy, int x, int y, int z) {
  return (double)img[2 * ((size_t)(x + 1) + (size_t)ex * (y + 1) + (size_t)exy * z) + 1];
}

// FP64 trilinear sample of a bordered image at voxel-unit position x, clamped
// to [0, D-1] per axis (the resampling of the objectives, Sec. 2.3.1).
__device__ double trilinear64(const DevProblem& pr, const float* img, const double x[3]) {
  int i0[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    const double c = fmin(fmax(x[a], 0.0), (double)(pr.D[a] - 1));
    int i = (int)floor(c);
    if (i > pr.D[a] - 2) i = pr.D[a] - 2;
    i0[a] = i;
    f[a] = c - i;
  }
  double acc = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        acc += w * raw_voxel(img, pr.ex, pr.exy, i0[0] + dx, i0[1] + dy, i0[2] + dz);
      }
  return acc;
}

// The piecewise-affine map of one solution (Sec. 2.1) at every voxel of image
// `own`: each tetrahedron of grid `own` rasterises its exact voxel set (the
// same spans as the objectives) and maps every voxel centre with FP64
// barycentric coordinates from exact orientations onto the same tetrahedron of
// the other grid.  Writes the displacement (voxel units) and the other image
// sampled there.  One workgroup per tetrahedron.
__global__ __launch_bounds__(kWG) void k_transform(DevProblem pr, int own, const float* __restrict__ X2,
                                                   float* dvf, float* warped) {
  __shared__ WaveRows rows[kWaves];
  __shared__ RasterTet rts[kWaves];
  __shared__ float xs[2][12];
  const int t = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int4 tv = pr.tets[t];
  const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
  const float* Xo = X2 + (size_t)own * 3 * pr.P;
  const float* Xt = X2 + (size_t)(1 - own) * 3 * pr.P;
  double L[4][3], Lt[4][3], Xv[4][3];
  unsigned bad = 0u;
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 3; ++c) {
      bad |= lattice_of(Xo[(size_t)vid[q] * 3 + c], pr.D[c], L[q][c]);
      const float xt = Xt[(size_t)vid[q] * 3 + c];
      bad |= lattice_of(xt, pr.D[c], Lt[q][c]);
      Xv[q][c] = (double)xt;
    }
  const double vol = orient(L[0], L[1], L[2], L[3]);
  if (bad || !(vol > 0.0)) return;
  if (threadIdx.x < 24) {
    const int g = threadIdx.x / 12, e = threadIdx.x % 12;
    xs[g][e] = (g == 0 ? Xo : Xt)[(size_t)vid[e / 3] * 3 + e % 3];
  }
  __syncthreads();
  RasterTet& rt = rts[wave];
  setup_raster(xs[0], xs[1], pr.D, lane, rt);
  const float* other = pr.img[1 - own];
  const int nb = (rt.nrows + 63) >> 6;
  for (int b = wave; b < nb; b += kWaves) {
    WaveRows& wr = rows[wave];
    int my_start;
    const int nvox = build_rows<false, 0>(rt, b, lane, pr.D, pr.D[0], pr.DxDy, 0, 0.0f, wr, &my_start);
    int carry = 0;
    for (int q0 = 0; q0 < nvox; q0 += 64) {
      wr.marker[lane] = 0;
      wave_sync();
      const unsigned pos = (unsigned)(my_start - q0);
      if (pos < 64u) wr.marker[pos] = 1;
      wave_sync();
      const int mk = wr.marker[lane];
      const unsigned long long M = __ballot(mk != 0);
      const int r = carry + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(M >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)M, 0u)) +
                    mk - 1;
      carry += __popcll(M);
      const int q = q0 + lane;
      if (q < nvox) {
        const int idx = __float_as_int(wr.row[r].rec.x) + q;
        const int k = idx / pr.DxDy, rem = idx - k * pr.DxDy;
        const int j = rem / pr.D[0], i = rem - j * pr.D[0];
        const double U[3] = {kLat * i + 0.5 * kLat, kLat * j + 0.5 * kLat, kLat * k + 0.5 * kLat};
        double x[3] = {0.0, 0.0, 0.0};
        for (int v = 0; v < 4; ++v) {
          double W[4][3];
          for (int m = 0; m < 4; ++m)
            for (int c = 0; c < 3; ++c) W[m][c] = m == v ? U[c] : L[m][c];
          const double lam = orient(W[0], W[1], W[2], W[3]) / vol;
          for (int c = 0; c < 3; ++c) x[c] += lam * Xv[v][c];
        }
        if (dvf) {
          dvf[(size_t)idx * 3 + 0] = (float)(x[0] - i);
          dvf[(size_t)idx * 3 + 1] = (float)(x[1] - j);
          dvf[(size_t)idx * 3 + 2] = (float)(x[2] - k);
        }
        if (warped) warped[idx] = (float)trilinear64(pr, other, x);
      }
    }
  }
}

// Bordered z-pair layout from an image [Dz][Dy][Dx]: element (x', y', z')
// = (I[c(z'-1)][c(y'-1)][c(x'-1)], I[c(z')][c(y'-1)][c(x'-1)]); elements of a
// row past x' = Dx + 1 (pitch padding) repeat the last voxel.
__global__ void k_pack_bordered(const float* __restrict__ raw, float* __restrict__ out, int Dx, int Dy, int Dz,
                                BorderedLayout bl) {
  const int64_t n = bl.elements();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % bl.px);
    const int64_t r = e / bl.px;
    const int y = (int)(r % bl.py), z = (int)(r / bl.py);
    const int cx = min(max(x - 1, 0), Dx - 1), cy = min(max(y - 1, 0), Dy - 1);
    const int z0 = min(max(z - 1, 0), Dz - 1), z1 = min(z, Dz - 1);
    const size_t row = (size_t)cy * Dx + cx, plane = (size_t)Dx * Dy;
    float2 v;
    v.x = raw[(size_t)z0 * plane + row];
    v.y = raw[(size_t)z1 * plane + row];
    reinterpret_cast<float2*>(out)[e] = v;
  }
}

__global__ void k_fill_i32(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

// ------------------------------------------------------------ launchers

size_t eval_lds_bytes(int maxA, int nver) { return eval_layout(maxA, nver).total; }

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  k_fill_u32<<<blocks, 256, 0, stream>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fold(const DevProblem& pr, int S, const float* X, uint32_t* flags, int32_t* first_bad,
                       hipStream_t stream) {
  hipError_t e = launch_fill_u32(flags, S, 0u, stream);
  if (e != hipSuccess) return e;
  if (first_bad) {
    k_fill_i32<<<(S + 255) / 256, 256, 0, stream>>>(first_bad, S, 0x7fffffff);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t np = (int64_t)S * pr.P, nt = (int64_t)S * pr.T;
  k_fold_points<<<(unsigned)((np + 255) / 256), 256, 0, stream>>>(pr, S, X, flags);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_fold_tets<<<(unsigned)((nt + 255) / 256), 256, 0, stream>>>(pr, S, X, flags, first_bad);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (first_bad) {
    k_first_bad_fix<<<(S + 255) / 256, 256, 0, stream>>>(S, first_bad);
    e = hipGetLastError();
  }
  return e;
}

// Element order of a partial launch (G <= kOrderMax): the elements sorted by
// their number of affected tetrahedra, descending (ties by index), are dealt
// to the 8 XCDs in rounds of 8 in alternating direction (0..7, 7..0, ...); the
// order lists XCD 0's elements, then XCD 1's, and so on.  Each XCD's
// contiguous range of the element-major workgroup space then holds elements of
// similar total cost.  Bitonic sort of (cost, index) keys in LDS, one
// workgroup.
__global__ __launch_bounds__(1024) void k_order(int G, const int* __restrict__ aff_cnt, int* __restrict__ order) {
  __shared__ unsigned long long key[kOrderMax];
  const int t = threadIdx.x;
  int n = 1;
  while (n < G) n <<= 1;
  for (int i = t; i < n; i += 1024)
    key[i] = i < G ? ((unsigned long long)(0xffffffffu - (unsigned)max(aff_cnt[i], 0)) << 32) | (unsigned)i : ~0ull;
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < n; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned long long u = key[i], v = key[l];
          if ((u > v) == ((i & k) == 0)) {
            key[i] = v;
            key[l] = u;
          }
        }
      }
      __syncthreads();
    }
  const int nb = G >> 4, rem = G & 15;
  for (int i = t; i < G; i += 1024) {
    const int r = i & 15, x = r < 8 ? r : 15 - r;
    int start = 0;  // elements dealt to the XCDs before x
    for (int y = 0; y < x; ++y) start += 2 * nb + (y < rem ? 1 : 0) + (15 - y < rem ? 1 : 0);
    order[start + (i >> 4) * 2 + (r >= 8 ? 1 : 0)] = (int)(unsigned)(key[i] & 0xffffffffull);
  }
}

hipError_t launch_order(int G, const int* aff_cnt, int* order, hipStream_t stream) {
  if (G <= 0 || G > kOrderMax) return hipSuccess;
  k_order<<<1, 1024, 0, stream>>>(G, aff_cnt, order);
  return hipGetLastError();
}

hipError_t launch_affected(const DevProblem& pr, int F, const int* fos_off, const int* fos_pts, int max_pts,
                           int maxA, int* aff, int* aff_cnt, hipStream_t stream) {
  if (F <= 0) return hipSuccess;
  k_affected<<<F, 64, 0, stream>>>(pr, F, fos_off, fos_pts, max_pts, maxA, aff, aff_cnt);
  return hipGetLastError();
}

hipError_t launch_eval(const EvalArgs& a, hipEvent_t ev_begin, hipEvent_t ev_end, hipStream_t stream) {
  const int64_t nwg = (int64_t)a.S * a.G;
  if (nwg <= 0) return hipSuccess;
  const size_t lds = eval_lds_bytes(kMaxChunk, a.nver);
  if (ev_begin) (void)hipEventRecord(ev_begin, stream);
  if (a.partial && a.row_pairs)
    k_sweep<1, 1><<<(unsigned)(nwg * a.nchunk), kWG, lds, stream>>>(a);
  else if (a.partial)
    k_sweep<1, 0><<<(unsigned)(nwg * a.nchunk), kWG, lds, stream>>>(a);
  else if (a.row_pairs)
    k_sweep<0, 1><<<(unsigned)nwg, kWG, lds, stream>>>(a);
  else
    k_sweep<0, 0><<<(unsigned)nwg, kWG, lds, stream>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_end) (void)hipEventRecord(ev_end, stream);
  k_finish<<<(unsigned)((nwg + kFinishPairs - 1) / kFinishPairs), 64, 0, stream>>>(a, (int)nwg);
  return hipGetLastError();
}

hipError_t launch_eval_batch(const EvalArgs* jobs_dev, const int* wg_off_dev, int n_jobs, int per_xcd, int total_finish,
                             size_t lds, int rows, hipStream_t stream) {
  if (per_xcd <= 0) return hipSuccess;
  const unsigned nwg = (unsigned)(8 * per_xcd);
  if (rows == 0)
    k_sweep_batch<0><<<nwg, kWG, lds, stream>>>(jobs_dev, wg_off_dev, n_jobs);
  else if (rows == 1)
    k_sweep_batch<1><<<nwg, kWG, lds, stream>>>(jobs_dev, wg_off_dev, n_jobs);
  else
    k_sweep_batch<2><<<nwg, kWG, lds, stream>>>(jobs_dev, wg_off_dev, n_jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_finish_batch<<<(unsigned)total_finish, 64, 0, stream>>>(jobs_dev, wg_off_dev + (n_jobs + 1), n_jobs);
  return hipGetLastError();
}

hipError_t launch_full_reduce(const DevProblem& pr, int S, const double* terms, double* obj, hipStream_t stream) {
  k_full_reduce<<<S, kWG, 0, stream>>>(pr, terms, obj);
  return hipGetLastError();
}

hipError_t launch_pack_bordered(const float* raw, float* out, int Dx, int Dy, int Dz, BorderedLayout bl,
                                hipStream_t stream) {
  const int64_t n = bl.elements();
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  k_pack_bordered<<<blocks, 256, 0, stream>>>(raw, out, Dx, Dy, Dz, bl);
  return hipGetLastError();
}

hipError_t launch_transform(const DevProblem& pr, int own, const float* X2, float* dvf, float* warped,
                            hipStream_t stream) {
  const int64_t V = (int64_t)pr.DxDy * pr.D[2];
  const uint32_t nan_bits = 0x7fc00000u;
  hipError_t e = hipSuccess;
  if (dvf) {
    k_fill_u32<<<(unsigned)std::min<int64_t>((3 * V + 255) / 256, 4096), 256, 0, stream>>>((uint32_t*)dvf, 3 * V,
                                                                                          nan_bits);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (warped) {
    k_fill_u32<<<(unsigned)std::min<int64_t>((V + 255) / 256, 4096), 256, 0, stream>>>((uint32_t*)warped, V,
                                                                                      nan_bits);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!dvf && !warped) return hipSuccess;
  k_transform<<<pr.T, kWG, 0, stream>>>(pr, own, X2, dvf, warped);
  return hipGetLastError();
}

hipError_t launch_owner(const DevProblem& pr, const float* Xg, int* owner, int* overlap, hipStream_t stream) {
  const int64_t V = (int64_t)pr.DxDy * pr.D[2];
  k_fill_i32<<<(unsigned)std::min<int64_t>((V + 255) / 256, 4096), 256, 0, stream>>>(owner, V, -1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_fill_i32<<<1, 64, 0, stream>>>(overlap, 1, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_owner<<<pr.T, kWG, 0, stream>>>(pr, Xg, owner, overlap);
  return hipGetLastError();
}

}  // namespace dsm
