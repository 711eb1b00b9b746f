// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/dsm.h"

namespace dsm {

constexpr int kWG = 256;          // threads per workgroup of the evaluation kernels
constexpr int kWaves = kWG / 64;  // wave64 waves per workgroup
constexpr double kLat = 128.0;    // lattice steps per voxel
// Clustering in objective space: at most kClusterMax clusters over at most
// kClusterSelMax selected solutions, at most kClusterRounds k-means rounds.
constexpr int kClusterMax = 16, kClusterSelMax = 1024, kClusterRounds = 50;
constexpr int kFullChunk = 8;     // tetrahedra per workgroup in full evaluation
// Affected tetrahedra per workgroup in partial evaluation: a per-problem
// setting in [kMinPartChunk, kMaxPartChunk] (dsm_set_part_chunk), default
// kPartChunk; the LDS layout is sized for kMaxChunk.
constexpr int kPartChunk = 8, kMinPartChunk = 4, kMaxPartChunk = 8;
constexpr int kMaxChunk = kFullChunk > kMaxPartChunk ? kFullChunk : kMaxPartChunk;
// The finishing kernel gives each (group, solution) pair kFinishLanes lanes
// (one per affected tetrahedron at a time), kFinishPairs pairs per 64-lane wave.
constexpr int kFinishLanes = 8;
constexpr int kFinishPairs = 64 / kFinishLanes;

// Sampled images are stored z-pair interleaved with a replicated one-voxel
// border: element (x', y', z') of the (Dx+2) x (Dy+2) x (Dz+1) element grid
// holds (I[c(z'-1)][c(y'-1)][c(x'-1)], I[c(z')][c(y'-1)][c(x'-1)]) with c()
// clamping each index into the image.  A position p (voxel units) is sampled
// at p + 1: every tap of any p in [-0.5, D-0.5] then lies inside the element
// grid, and the taps that fall outside the image repeat the border value, so
// interpolating them gives exactly the value at the position clamped to
// [0, D-1] without a clamp instruction.
// The row pitch px (elements per stored row, >= Dx + 2) is a tuning
// parameter: the gathers of one wave touch a few rows at once, and some row
// strides make them collide in the memory pipeline.  The default is the
// smallest pitch >= Dx + 2 that is 8 mod 16 elements (row stride 64 mod 128
// bytes); dsm_autotune_pitch measures alternatives.
struct BorderedLayout {
  int px, py, pz;  // element grid dims
  __host__ __device__ int64_t elements() const { return (int64_t)px * py * pz; }
};
inline int default_pitch(int Dx) { return Dx + 2 + ((8 - (Dx + 2) % 16) + 16) % 16; }
inline BorderedLayout bordered_layout(int Dx, int Dy, int Dz, int pitch) {
  return {pitch > 0 ? pitch : default_pitch(Dx), Dy + 2, Dz + 1};
}
// Largest accepted pitch: the byte offsets of one image must fit a 32-bit buffer offset.
inline bool pitch_ok(int Dx, int Dy, int Dz, int pitch) {
  return pitch >= Dx + 2 && pitch <= 4 * (Dx + 2) + 64 &&
         (int64_t)pitch * (Dy + 2) * (Dz + 1) * 8 < ((int64_t)1 << 31);
}

// Everything a kernel needs to know about one problem (passed by value).
struct DevProblem {
  const float* img[2];   // [0] source (moving), [1] target (fixed); bordered z-pair layout (BorderedLayout)
  int img_bytes;         // bytes of one bordered image (buffer range)
  int ex, exy;           // element strides of y and z in the bordered layout
  int D[3];
  int DxDy;
  float tau;             // empty iff value <= tau
  double sp[3];          // voxel spacing in mm
  int n[3];              // points per axis
  int P, T;
  const int4* tets;      // [T] vertex ids, positively oriented on the undeformed grid
  const double* tet_w;   // [T][6] 1/k_e of the edges 01 02 03 12 13 23
  const int* star_off;   // [P+1]
  const int* star;       // [4T]
  int ng[2];             // guidance points per image
  const double* gpt[2];  // [ng][3] lattice units
  const int* gcorr[2];   // [ng] correspondence ids
  double norm[3];        // objective normalisers
};

struct EvalArgs {
  DevProblem pr;
  int S;                 // solutions
  int G;                 // groups: FOS elements (partial) or tetrahedron chunks (full)
  int partial;           // 1: partial evaluation, 0: full evaluation
  int row_pairs;         // 1: the sweep's rows alternate between the slices of a pair (dsm_set_row_order);
                         // placed in the padding before X, so the fields after it keep their offsets
  const float* X;        // [S][2][P][3]
  const int* fos_off;    // partial only
  const int* fos_pts;
  const float* cand;     // [S][fos_off[G]][2][3]
  const int* aff;        // [G][maxA] affected tetrahedra, ascending
  const int* aff_cnt;    // [G], -1 = malformed element
  const int* order;      // [G] order of the elements over the XCDs (partial), or null
  int maxA;
  int nver;              // 1: candidate only; 2: candidate and current recomputed
  const double* terms_in;  // [S][T][3] cache of current terms or null
  double* part_old;      // [S][G][3]
  double* part_new;
  uint32_t* flags;       // [S][G]
  double* terms_out;     // [S][T][3] or null
  uint32_t* vcount;      // [S][G] or null
  const uint8_t* mask;   // [S][G] or null: evaluate only where non-zero (partial)
  double* simws;         // swept dissimilarity workspace of the problem
  int pchunk;            // partial: affected tetrahedra per workgroup
  int nchunk;            // partial: workgroups (chunks of pchunk affected tetrahedra) per group
  uint32_t* cflags;      // partial: [S][G][nchunk] constraint flags per chunk
  uint32_t* ccount;      // partial: [S][G][nchunk] candidate voxel count per chunk
};

// Host-side topology (topology.cpp).
struct HostTopology {
  int P = 0, C = 0, T = 0, E = 0, max_star = 0;
  std::vector<int> tets;      // [T][4]
  std::vector<double> tet_w;  // [T][6]
  std::vector<int> star_off;  // [P+1]
  std::vector<int> star;      // [4T]
};
bool build_topology(const int mesh[3], HostTopology& out);
void identity_grid(const int mesh[3], const int dims[3], float* X);

// Kernel launchers (kernels.hip).  All enqueue on `stream` and return the
// launch status.
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_fold(const DevProblem& pr, int S, const float* X, uint32_t* flags, int32_t* first_bad,
                       hipStream_t stream);
hipError_t launch_affected(const DevProblem& pr, int F, const int* fos_off, const int* fos_pts, int max_pts,
                           int maxA, int* aff, int* aff_cnt, hipStream_t stream);
hipError_t launch_eval(const EvalArgs& a, hipEvent_t ev_begin, hipEvent_t ev_end, hipStream_t stream);
// Orders the G elements of a partial launch so that the XCDs' contiguous
// ranges carry similar work (costs from the affected counts).  Only for
// G <= kOrderMax; larger launches use a fixed interleaved order.
constexpr int kOrderMax = 4096;
hipError_t launch_order(int G, const int* aff_cnt, int* order, hipStream_t stream);
// wg_off_dev [2][n_jobs + 1]: the jobs' per-XCD slot offsets in the sweep (a
// job of n workgroups takes ceil(n / 8) slots on each XCD; per_xcd slots in
// all), then their workgroup offsets in the finishing kernel (a job of n
// pairs takes ceil(n / kFinishPairs) workgroups; total_finish in all).  rows:
// 0 every job's rows by slice, 1 every job's by slice pair, 2 both occur.
hipError_t launch_eval_batch(const EvalArgs* jobs_dev, const int* wg_off_dev, int n_jobs, int per_xcd, int total_finish,
                             size_t lds, int rows, hipStream_t stream);
hipError_t launch_full_reduce(const DevProblem& pr, int S, const double* terms, double* obj, hipStream_t stream);
hipError_t launch_owner(const DevProblem& pr, const float* Xg, int* owner, int* overlap, hipStream_t stream);
// Piecewise-affine map of one solution X2 [2][P][3] at every voxel of image own:
// displacement dvf [V][3] and the other image sampled there, warped [V] (either may be null).
hipError_t launch_transform(const DevProblem& pr, int own, const float* X2, float* dvf, float* warped,
                            hipStream_t stream);
hipError_t launch_pack_bordered(const float* raw, float* out, int Dx, int Dy, int Dz, BorderedLayout bl,
                                hipStream_t stream);
size_t eval_lds_bytes(int maxA, int nver);

// Error string of the calling thread, read by dsm_last_error (api.cpp).
dsm_status set_error(dsm_status st, const char* msg);
void clear_error();

}  // namespace dsm

// The problem object behind the opaque ABI handle.
struct dsm_problem {
  dsm::DevProblem dev{};
  dsm::HostTopology topo;
  int dims[3]{};
  int mesh[3]{};
  int64_t V = 0;
  int max_S = 0, max_F = 0, max_pts = 0, maxA = 0;
  int device = 0;
  // device buffers owned by the problem
  float* d_img = nullptr;       // [2][Dz+1][Dy+2][pitch][2] bordered z-pair layout
  size_t img_stride = 0;        // floats per bordered image
  float* d_raw = nullptr;       // [2][Dz][Dy][Dx] the images as given (source, target), for re-packing
  int pitch = 0;                // row pitch of d_img in elements
  int* d_tets = nullptr;
  double* d_tet_w = nullptr;
  int* d_star_off = nullptr;
  int* d_star = nullptr;
  double* d_gpt = nullptr;      // [n_m + n_f][3]
  int* d_gcorr = nullptr;
  int* d_aff = nullptr;         // [max_F][maxA]
  int* d_aff_cnt = nullptr;     // [max_F]
  int* d_order = nullptr;       // [max_F] element order of the last partial launch
  double* d_terms = nullptr;    // [max_S][T][3] workspace for full evaluation
  double* d_simws = nullptr;    // swept dissimilarity per (solution, group, version, tetrahedron)
  size_t simws_len = 0;
  uint32_t* d_cflags = nullptr; // [max_S][max_F][nchunk] per-chunk flags of a partial evaluation
  uint32_t* d_ccount = nullptr; // [max_S][max_F][nchunk] per-chunk voxel counts
  int part_chunk = dsm::kPartChunk;  // affected tetrahedra per workgroup in partial evaluation
  int nchunk = 1;               // ceil(maxA / part_chunk); the chunk arrays hold ceil(maxA / kMinPartChunk)
  int row_order = DSM_ROWS_BY_SLICE;  // or DSM_ROWS_BY_SLICE_PAIR (dsm_set_row_order)
  std::vector<float> identity;  // [P][3]
  float* d_ident = nullptr;     // device copy of the undeformed grid [P][3]
  std::vector<hipEvent_t> ev;   // timing event pairs (begin, end)
  int ev_used = 0;
};
