// Learned pre-screening of partial-evaluation candidates: a small MLP
// (192 -> 128 -> 128 -> 3, ReLU) that predicts the objective deltas of a
// single-point partial change from local features, trained on the exact deltas
// the evaluator produces.  Acceptance still rests on the exact evaluator:
// screening only chooses which candidate is evaluated and whether it is
// evaluated at all.
//
// All matrix products run on gfx950 matrix cores: v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation).  Weights are kept in FP32 (master copy,
// Adam state) and BF16 (operands).  Activations are rounded to BF16 where they
// feed the next product; everything else is FP32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dsm_internal.h"

namespace dsm {
namespace {

constexpr int kIn = 192, kHid = 128, kOut = 3, kOutPad = 16, kNumFeat = 188;
// parameter layout of the FP32 master copy
constexpr int kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid, kW3 = kB2 + kHid,
              kB3 = kW3 + kOutPad * kHid, kNParams = kB3 + kOutPad;
static_assert(kNParams == 43280, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16, round to nearest even
__device__ __forceinline__ unsigned short f2bf(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ f32x4 mfma(const u16x8& a, const u16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

__device__ __forceinline__ u16x8 load8(const unsigned short* p) { return *(const u16x8*)p; }

__device__ __forceinline__ u16x8 zero8() {
  u16x8 z;
  for (int e = 0; e < 8; ++e) z[e] = 0;
  return z;
}

struct MlpW {
  const unsigned short *w1, *w2, *w3;    // BF16 [128][192], [128][128], [16][128] (out, in)
  const unsigned short *w2t, *w3t;       // BF16 transposes [128][128], [128][16] (in, out)
  const float *b1, *b2, *b3;             // FP32 biases
};

// LDS tile of one wave: 16 rows x 128 columns of BF16 with a padded stride
constexpr int kLdsStride = 136;

// Y[16][16] (+bias) = A[16][K] x W^T, W [ncols][K] row-major BF16; A is either
// a global BF16 matrix (rows a_row0.., stride a_stride, rows >= nrows zero) or an
// LDS tile.  Applies ReLU and stores BF16 into `out` (LDS tile) when relu_out.
template <int K>
__device__ __forceinline__ f32x4 tile_product(const unsigned short* A, int a_stride, bool a_valid, const unsigned short* W,
                                              int col0, int lane) {
  const int i = lane & 15, kb = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < K / 32; ++kk) {
    const u16x8 a = a_valid ? load8(A + (size_t)i * a_stride + 32 * kk + 8 * kb) : zero8();
    const u16x8 b = load8(W + (size_t)(col0 + i) * K + 32 * kk + 8 * kb);
    acc = mfma(a, b, acc);
  }
  return acc;
}

// Forward pass of 16 rows held by one wave.  x: global BF16 rows (stride 192)
// of which `valid` exist.  Leaves H1 and H2 (BF16, post-ReLU) in LDS tiles and
// returns the outputs of row 4*kb + r, column i in y[r] (columns >= 3 are 0).
__device__ void forward16(const MlpW& w, const unsigned short* x, bool row_valid, unsigned short* h1,
                          unsigned short* h2, int lane, f32x4& y) {
  const int i = lane & 15, kb = lane >> 4;
  for (int ct = 0; ct < kHid / 16; ++ct) {
    const f32x4 acc = tile_product<kIn>(x, kIn, row_valid, w.w1, 16 * ct, lane);
    const float b = w.b1[16 * ct + i];
    for (int r = 0; r < 4; ++r) h1[(4 * kb + r) * kLdsStride + 16 * ct + i] = f2bf(fmaxf(acc[r] + b, 0.f));
  }
  __syncthreads();
  for (int ct = 0; ct < kHid / 16; ++ct) {
    const f32x4 acc = tile_product<kHid>(h1, kLdsStride, true, w.w2, 16 * ct, lane);
    const float b = w.b2[16 * ct + i];
    for (int r = 0; r < 4; ++r) h2[(4 * kb + r) * kLdsStride + 16 * ct + i] = f2bf(fmaxf(acc[r] + b, 0.f));
  }
  __syncthreads();
  const f32x4 acc = tile_product<kHid>(h2, kLdsStride, true, w.w3, 0, lane);
  const float b = w.b3[i];
  for (int r = 0; r < 4; ++r) y[r] = i < kOut ? acc[r] + b : 0.f;
}

// Screening forward pass: 64 rows per workgroup of 4 waves.  The rows are
// staged in LDS once; each wave computes a 32-column slice of a layer for all
// 64 rows, so every weight fragment read from memory serves 4 row blocks.
constexpr int kXs = kIn + 8;  // padded LDS strides (BF16 elements)
constexpr int kHs = kHid + 8;

__global__ __launch_bounds__(256) void k_mlp_forward64(MlpW w, const unsigned short* __restrict__ xb, int N,
                                                       float* __restrict__ out) {
  __shared__ __align__(16) unsigned short xs[64 * kXs];  // inputs, then H2
  __shared__ __align__(16) unsigned short h1[64 * kHs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, kb = lane >> 4;
  const int row0 = blockIdx.x * 64;
  for (int e = tid; e < 64 * kIn / 8; e += 256) {
    const int r = e / (kIn / 8), c = e % (kIn / 8);
    const u16x8 v = row0 + r < N ? load8(xb + (size_t)(row0 + r) * kIn + 8 * c) : zero8();
    *(u16x8*)(xs + r * kXs + 8 * c) = v;
  }
  __syncthreads();
  // layer 1: H1 = relu(X W1^T + b1), wave -> columns [32 wave, 32 wave + 32)
  {
    f32x4 acc[2][4];
    for (int t = 0; t < 2; ++t)
      for (int rb = 0; rb < 4; ++rb) acc[t][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kIn / 32; ++kk) {
      u16x8 b[2];
      for (int t = 0; t < 2; ++t) b[t] = load8(w.w1 + (size_t)(32 * wave + 16 * t + i) * kIn + 32 * kk + 8 * kb);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const u16x8 a = *(const u16x8*)(xs + (16 * rb + i) * kXs + 32 * kk + 8 * kb);
        for (int t = 0; t < 2; ++t) acc[t][rb] = mfma(a, b[t], acc[t][rb]);
      }
    }
    for (int t = 0; t < 2; ++t) {
      const int col = 32 * wave + 16 * t + i;
      const float bias = w.b1[col];
      for (int rb = 0; rb < 4; ++rb)
        for (int r = 0; r < 4; ++r) h1[(16 * rb + 4 * kb + r) * kHs + col] = f2bf(fmaxf(acc[t][rb][r] + bias, 0.f));
    }
  }
  __syncthreads();
  // layer 2: H2 = relu(H1 W2^T + b2) into the input buffer (no longer needed)
  unsigned short* h2 = xs;
  {
    f32x4 acc[2][4];
    for (int t = 0; t < 2; ++t)
      for (int rb = 0; rb < 4; ++rb) acc[t][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kHid / 32; ++kk) {
      u16x8 b[2];
      for (int t = 0; t < 2; ++t) b[t] = load8(w.w2 + (size_t)(32 * wave + 16 * t + i) * kHid + 32 * kk + 8 * kb);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const u16x8 a = *(const u16x8*)(h1 + (16 * rb + i) * kHs + 32 * kk + 8 * kb);
        for (int t = 0; t < 2; ++t) acc[t][rb] = mfma(a, b[t], acc[t][rb]);
      }
    }
    for (int t = 0; t < 2; ++t) {  // the barrier after layer 1 ordered every read of the inputs before this
      const int col = 32 * wave + 16 * t + i;
      const float bias = w.b2[col];
      for (int rb = 0; rb < 4; ++rb)
        for (int r = 0; r < 4; ++r) h2[(16 * rb + 4 * kb + r) * kHs + col] = f2bf(fmaxf(acc[t][rb][r] + bias, 0.f));
    }
  }
  __syncthreads();
  // layer 3: Y = H2 W3^T + b3, wave -> row block `wave`
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < kHid / 32; ++kk) {
    const u16x8 a = *(const u16x8*)(h2 + (16 * wave + i) * kHs + 32 * kk + 8 * kb);
    const u16x8 b = load8(w.w3 + (size_t)i * kHid + 32 * kk + 8 * kb);
    acc = mfma(a, b, acc);
  }
  if (i < kOut) {
    const float bias = w.b3[i];
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + 16 * wave + 4 * kb + r;
      if (row < N) out[(size_t)row * kOut + i] = acc[r] + bias;
    }
  }
}

// Training rows: forward and backward of 16 minibatch rows per wave.  Writes
// the transposed BF16 operands of the weight-gradient products (inputs X, H1,
// H2 and output gradients dY, dZ2, dZ1, all [features][batch]) and the per-row
// squared error.  Loss = (1/B) sum_rows sum_{3 outputs} (y - t)^2.
struct TrainWs {
  unsigned short *xt, *h1t, *h2t, *dyt, *dz2t, *dz1t;  // [192|128|128|16|128|128][ld]
  float* row_loss;                                      // [B]
  int ld;                                               // B rounded up to a multiple of 32; rows past B are zero
};

__global__ __launch_bounds__(64) void k_mlp_rows(MlpW w, const unsigned short* __restrict__ xb,
                                                 const float* __restrict__ targets, const int* __restrict__ idx, int B,
                                                 TrainWs ws) {
  __shared__ __align__(16) unsigned short h1[16 * kLdsStride], h2[16 * kLdsStride], dz[16 * kLdsStride];
  __shared__ __align__(16) unsigned short xr[16 * kIn];
  __shared__ __align__(16) unsigned short dy[16 * 32];
  __shared__ float sq[16][4];
  const int lane = threadIdx.x, i = lane & 15, kb = lane >> 4;
  const int b0 = blockIdx.x * 16;
  // gather the 16 input rows into LDS (rows past B are zero)
  for (int e = lane; e < 16 * kIn / 8; e += 64) {
    const int r = e / (kIn / 8), c = e % (kIn / 8);
    const u16x8 v = (b0 + r < B) ? load8(xb + (size_t)idx[b0 + r] * kIn + 8 * c) : zero8();
    *(u16x8*)(xr + r * kIn + 8 * c) = v;
  }
  __syncthreads();
  f32x4 y;
  forward16(w, xr, true, h1, h2, lane, y);
  // dY = 2 (y - t) / (3 B), rows past B contribute nothing
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * kb + r, brow = b0 + row;
    float g = 0.f, e2 = 0.f;
    if (i < kOut && brow < B) {
      const float d = y[r] - targets[(size_t)idx[brow] * kOut + i];
      e2 = d * d;
      g = 2.f * d / (3.f * (float)B);
    }
    dy[row * 32 + i] = f2bf(g);
    dy[row * 32 + 16 + i] = 0;
    if (i < 4) sq[row][i] = i < kOut ? e2 : 0.f;
  }
  __syncthreads();
  if (lane < 16 && b0 + lane < B) ws.row_loss[b0 + lane] = sq[lane][0] + sq[lane][1] + sq[lane][2];
  // transposed copies of X, H1, H2, dY
  for (int e = lane; e < 16 * kIn; e += 64) {
    const int r = e % 16, c = e / 16;
    if (b0 + r < ws.ld) ws.xt[(size_t)c * ws.ld + b0 + r] = xr[r * kIn + c];
  }
  for (int e = lane; e < 16 * kHid; e += 64) {
    const int r = e % 16, c = e / 16;
    if (b0 + r < ws.ld) {
      ws.h1t[(size_t)c * ws.ld + b0 + r] = h1[r * kLdsStride + c];
      ws.h2t[(size_t)c * ws.ld + b0 + r] = h2[r * kLdsStride + c];
    }
  }
  for (int e = lane; e < 16 * kOutPad; e += 64) {
    const int r = e % 16, c = e / 16;
    if (b0 + r < ws.ld) ws.dyt[(size_t)c * ws.ld + b0 + r] = dy[r * 32 + c];
  }
  // dZ2 = (dY W3) * [H2 > 0]: A = dY [16][32] (columns >= 16 zero), B[o][j] = W3t[j][o]
  for (int ct = 0; ct < kHid / 16; ++ct) {
    const u16x8 a = load8(dy + i * 32 + 8 * kb);
    const u16x8 bm = kb < 2 ? load8(w.w3t + (size_t)(16 * ct + i) * kOutPad + 8 * kb) : zero8();
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(a, bm, acc);
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * kb + r, col = 16 * ct + i;
      const float g = bf2f(h2[row * kLdsStride + col]) > 0.f ? acc[r] : 0.f;
      dz[row * kLdsStride + col] = f2bf(g);
    }
  }
  __syncthreads();
  for (int e = lane; e < 16 * kHid; e += 64) {
    const int r = e % 16, c = e / 16;
    if (b0 + r < ws.ld) ws.dz2t[(size_t)c * ws.ld + b0 + r] = dz[r * kLdsStride + c];
  }
  // dZ1 = (dZ2 W2) * [H1 > 0]: B[m][j] = W2t[j][m]
  f32x4 accs[kHid / 16];
  for (int ct = 0; ct < kHid / 16; ++ct) accs[ct] = tile_product<kHid>(dz, kLdsStride, true, w.w2t, 16 * ct, lane);
  __syncthreads();
  for (int ct = 0; ct < kHid / 16; ++ct)
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * kb + r, col = 16 * ct + i;
      const float g = bf2f(h1[row * kLdsStride + col]) > 0.f ? accs[ct][r] : 0.f;
      dz[row * kLdsStride + col] = f2bf(g);
    }
  __syncthreads();
  for (int e = lane; e < 16 * kHid; e += 64) {
    const int r = e % 16, c = e / 16;
    if (b0 + r < ws.ld) ws.dz1t[(size_t)c * ws.ld + b0 + r] = dz[r * kLdsStride + c];
  }
}

// Weight gradients dW[o][c] = sum_b dZt[o][b] At[c][b] for one 16x16 tile per
// wave; B is a multiple of 32 (callers pad with zero rows).
__global__ __launch_bounds__(64) void k_mlp_wgrad(const unsigned short* __restrict__ dzt, const unsigned short* __restrict__ at,
                                                  int B, int ncols, float* __restrict__ dw) {
  const int lane = threadIdx.x, i = lane & 15, kb = lane >> 4;
  const int ot = blockIdx.y, ctile = blockIdx.x;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < B; k0 += 32) {
    const u16x8 a = load8(dzt + (size_t)(16 * ot + i) * B + k0 + 8 * kb);
    const u16x8 b = load8(at + (size_t)(16 * ctile + i) * B + k0 + 8 * kb);
    acc = mfma(a, b, acc);
  }
  for (int r = 0; r < 4; ++r) dw[(size_t)(16 * ot + 4 * kb + r) * ncols + 16 * ctile + i] = acc[r];
}

// Bias gradients and the minibatch loss: one wave per sum, lanes over the
// batch in a fixed order, then a fixed shuffle tree (deterministic).
__global__ __launch_bounds__(64) void k_mlp_bias_loss(const unsigned short* __restrict__ dz1t,
                                                      const unsigned short* __restrict__ dz2t,
                                                      const unsigned short* __restrict__ dyt,
                                                      const float* __restrict__ row_loss, int B, int ld,
                                                      float* __restrict__ grad, float* __restrict__ loss_out) {
  const int t = blockIdx.x, lane = threadIdx.x;
  const unsigned short* src = nullptr;
  float* dst = nullptr;
  if (t < kHid) {
    src = dz1t + (size_t)t * ld;
    dst = grad + kB1 + t;
  } else if (t < 2 * kHid) {
    src = dz2t + (size_t)(t - kHid) * ld;
    dst = grad + kB2 + (t - kHid);
  } else if (t < 2 * kHid + kOutPad) {
    src = dyt + (size_t)(t - 2 * kHid) * ld;
    dst = grad + kB3 + (t - 2 * kHid);
  }
  float acc = 0.f;
  if (src) {
    for (int b = lane; b < B; b += 64) acc += bf2f(src[b]);
  } else {
    for (int b = lane; b < B; b += 64) acc += row_loss[b];
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    if (src)
      *dst = acc;
    else if (loss_out)
      *loss_out = acc / (3.f * (float)B);
  }
}

// Adam step on the FP32 master parameters, then refresh of the BF16 operand copies.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kNParams) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  p[t] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_refresh_bf16(const float* __restrict__ p, unsigned short* w1, unsigned short* w2, unsigned short* w3,
                               unsigned short* w2t, unsigned short* w3t) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kHid * kIn) w1[t] = f2bf(p[kW1 + t]);
  if (t < kHid * kHid) {
    const int o = t / kHid, c = t % kHid;
    w2[t] = f2bf(p[kW2 + t]);
    w2t[c * kHid + o] = f2bf(p[kW2 + t]);
  }
  if (t < kOutPad * kHid) {
    const int o = t / kHid, c = t % kHid;
    w3[t] = f2bf(p[kW3 + t]);
    w3t[c * kOutPad + o] = f2bf(p[kW3 + t]);
  }
}

// Counter-based minibatch indices (splitmix64 of (seed, step, slot)).
__global__ void k_batch_indices(unsigned long long seed, int step, int N, int B, int Bpad, int* idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bpad) return;
  if (b >= B) {
    idx[b] = 0;
    return;
  }
  unsigned long long z = seed + 0x9e3779b97f4a7c15ull * ((unsigned long long)step * 0x100000001ull + (unsigned long long)b + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  idx[b] = (int)(z % (unsigned long long)N);
}

__global__ void k_iota(int n, int* idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) idx[b] = b;
}

// ---------------------------------------------------------------- features

// trilinear sample of a bordered z-pair image at voxel position p clamped to [0, D-1]
__device__ float sample_packed(const DevProblem& pr, const float* img, float px, float py, float pz) {
  px = fminf(fmaxf(px, 0.f), (float)(pr.D[0] - 1)) + 1.f;
  py = fminf(fmaxf(py, 0.f), (float)(pr.D[1] - 1)) + 1.f;
  pz = fminf(fmaxf(pz, 0.f), (float)(pr.D[2] - 1)) + 1.f;
  const int ix = (int)px, iy = (int)py, iz = (int)pz;
  const float fx = px - ix, fy = py - iy, fz = pz - iz;
  const float* e = img + 2 * ((size_t)iz * pr.exy + (size_t)iy * pr.ex + ix);
  const float* f = e + 2 * pr.ex;
  // e: (x,y,z),(x,y,z+1),(x+1,y,z),(x+1,y,z+1); f: the same at y+1
  const float c00 = e[0] + fx * (e[2] - e[0]), c01 = e[1] + fx * (e[3] - e[1]);
  const float c10 = f[0] + fx * (f[2] - f[0]), c11 = f[1] + fx * (f[3] - f[1]);
  const float c0 = c00 + fy * (c10 - c00), c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

// Raw features of candidate k of single-point element f of solution s:
//   [0, 6)     candidate minus current position of the point, both grids;
//   [6, 162)   for each of the 26 grid neighbours o (dz, dy, dx in {-1,0,1},
//              dx fastest, centre skipped) and each grid: neighbour position
//              relative to the candidate minus the undeformed relative offset
//              (0 where the neighbour does not exist);
//   [162, 188) source image at (candidate + h o) minus target image at
//              (candidate + h o), h = half the undeformed cube extent per axis;
//   [188, 192) zero.
// Rows are numbered (s, f, k) with k fastest.  32 lanes share a row: lane
// j < 26 computes neighbour slot j (its 6 displacement features and its
// intensity difference), lane 26 the moved-point features, lane 27 the padding.
// With PACK the values are standardised with the stored input statistics and
// rounded to BF16 in the same kernel, bit for bit what k_pack makes of the
// FP32 rows (sums and products are written with explicit rounding, so that
// both instantiations compute identical FP32 values).
template <bool PACK>
__global__ __launch_bounds__(256) void k_features(DevProblem pr, const float* __restrict__ X, int S, int F,
                                                  const int* __restrict__ pts, int K, const float* __restrict__ cand,
                                                  const float* __restrict__ ident, const float* __restrict__ mean,
                                                  const float* __restrict__ rstd, float* __restrict__ out32,
                                                  unsigned short* __restrict__ out16) {
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 5;
  const int j = threadIdx.x & 31;
  if (row >= (int64_t)S * F * K || j >= 28) return;
  const int s = (int)(row / ((int64_t)F * K));
  const int f = (int)((row / K) % F);
  const int p = pts[f];
  const bool valid = p >= 0 && p < pr.P;
  const float* c = cand + row * 6;  // [2][3]
  const float* Xs = X + (size_t)s * 6 * pr.P;
  float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float vi = 0.f;
  int col;
  if (j < 26) {
    col = 6 + 6 * j;
    if (valid) {
      const int t = j < 13 ? j : j + 1;  // centre (13) skipped
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
      const int pi = p % pr.n[0], pj = (p / pr.n[0]) % pr.n[1], pk = p / (pr.n[0] * pr.n[1]);
      const int qi = pi + dx, qj = pj + dy, qk = pk + dz;
      if (qi >= 0 && qi < pr.n[0] && qj >= 0 && qj < pr.n[1] && qk >= 0 && qk < pr.n[2]) {
        const int q = qi + pr.n[0] * (qj + pr.n[1] * qk);
        for (int g = 0; g < 2; ++g)
          for (int a = 0; a < 3; ++a)
            v[3 * g + a] = __fsub_rn(__fsub_rn(Xs[((size_t)g * pr.P + q) * 3 + a], c[3 * g + a]),
                                     __fsub_rn(ident[3 * q + a], ident[3 * p + a]));
      }
      float off[3];
      const int d[3] = {dx, dy, dz};
      for (int a = 0; a < 3; ++a) off[a] = __fmul_rn(__fdiv_rn((float)pr.D[a], 2.f * (float)(pr.n[a] - 1)), (float)d[a]);
      const float im = sample_packed(pr, pr.img[0], __fadd_rn(c[0], off[0]), __fadd_rn(c[1], off[1]), __fadd_rn(c[2], off[2]));
      const float it = sample_packed(pr, pr.img[1], __fadd_rn(c[3], off[0]), __fadd_rn(c[4], off[1]), __fadd_rn(c[5], off[2]));
      vi = __fsub_rn(im, it);
    }
  } else if (j == 26) {
    col = 0;
    if (valid)
      for (int g = 0; g < 2; ++g)
        for (int a = 0; a < 3; ++a) v[3 * g + a] = __fsub_rn(c[3 * g + a], Xs[((size_t)g * pr.P + p) * 3 + a]);
  } else {
    col = kNumFeat;  // 4 zero columns
  }
  const int nv = j == 27 ? kIn - kNumFeat : 6;
  if (PACK) {
    unsigned* o = reinterpret_cast<unsigned*>(out16 + row * kIn + col);  // 4-byte aligned: col is even
    for (int e = 0; e < nv; e += 2) {
      const unsigned lo = f2bf(__fmul_rn(__fsub_rn(v[e], mean[col + e]), rstd[col + e]));
      const unsigned hi = f2bf(__fmul_rn(__fsub_rn(v[e + 1], mean[col + e + 1]), rstd[col + e + 1]));
      o[e >> 1] = lo | (hi << 16);
    }
    if (j < 26) out16[row * kIn + kNumFeat - 26 + j] = f2bf(__fmul_rn(__fsub_rn(vi, mean[162 + j]), rstd[162 + j]));
  } else {
    float2* o = reinterpret_cast<float2*>(out32 + row * kIn + col);  // 8-byte aligned: col is even
    for (int e = 0; e < nv; e += 2) o[e >> 1] = make_float2(v[e], v[e + 1]);
    if (j < 26) out32[row * kIn + kNumFeat - 26 + j] = vi;
  }
}

// Standardise FP32 rows and round to BF16 operands; optionally standardise targets.
__global__ void k_pack(int N, const float* __restrict__ feats, const float* __restrict__ mean, const float* __restrict__ rstd,
                       unsigned short* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * kIn) return;
  const int c = (int)(e % kIn);
  out[e] = f2bf(__fmul_rn(__fsub_rn(feats[e], mean[c]), rstd[c]));
}

// Column mean and 1/std of N rows of width `width` (fixed-order FP64 sums, one
// workgroup per column).
__global__ __launch_bounds__(256) void k_column_stats(int N, int width, const float* __restrict__ x, float* mean,
                                                      float* rstd) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int r = t; r < N; r += 256) {
    const double v = x[(size_t)r * width + c];
    a += v;
    b += v * v;
  }
  s1[t] = a;
  s2[t] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      s1[t] += s1[t + w];
      s2[t] += s2[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double m = N > 0 ? s1[0] / N : 0.0;
    const double var = N > 0 ? fmax(s2[0] / N - m * m, 0.0) : 0.0;
    mean[c] = (float)m;
    rstd[c] = var > 1e-30 ? (float)(1.0 / sqrt(var)) : 1.f;  // constant columns pass through centred
  }
}

// Raw objective deltas (part_new - part_old) of N rows, standardised.
__global__ void k_targets(int N, const double* __restrict__ old, const double* __restrict__ nw, const float* __restrict__ mean,
                          const float* __restrict__ rstd, float* __restrict__ out, float* __restrict__ raw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * kOut) return;
  const float d = (float)(nw[e] - old[e]);
  if (raw) raw[e] = d;
  if (out) out[e] = (d - mean[e % kOut]) * rstd[e % kOut];
}

// Screening: per (solution, element) choose one of K candidates by predicted
// Pareto rank among the K (ties: smallest sum of standardised predictions) and
// flag it for exact evaluation iff its predicted delta would be accepted: it
// improves one objective without worsening another, or it improves one
// objective and the predicted objective vector is not dominated by any archive
// member.
__global__ void k_select(int S, int F, int K, const float* __restrict__ pred_std, const float* __restrict__ out_mean,
                         const float* __restrict__ out_scale, const double* __restrict__ obj, int n_arch,
                         const double* __restrict__ arch, float* __restrict__ pred_raw, int* __restrict__ pick,
                         unsigned char* __restrict__ run_exact) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * F) return;
  const int s = e / F;
  const float* ps = pred_std + (size_t)e * K * kOut;
  int best = 0, best_rank = 1 << 30;
  float best_sum = INFINITY;
  for (int k = 0; k < K; ++k) {
    int rank = 0;
    for (int j = 0; j < K; ++j) {
      if (j == k) continue;
      bool le = true, lt = false;
      for (int o = 0; o < kOut; ++o) {
        le = le && ps[j * kOut + o] <= ps[k * kOut + o];
        lt = lt || ps[j * kOut + o] < ps[k * kOut + o];
      }
      rank += (le && lt) ? 1 : 0;
    }
    const float sum = ps[k * kOut] + ps[k * kOut + 1] + ps[k * kOut + 2];
    if (rank < best_rank || (rank == best_rank && sum < best_sum)) {
      best = k;
      best_rank = rank;
      best_sum = sum;
    }
  }
  double d[kOut];
  for (int k = 0; k < K; ++k)
    for (int o = 0; o < kOut; ++o) {
      const float r = ps[k * kOut + o] * out_scale[o] + out_mean[o];
      if (pred_raw) pred_raw[((size_t)e * K + k) * kOut + o] = r;
      if (k == best) d[o] = r;
    }
  bool le = true, lt = false;
  for (int o = 0; o < kOut; ++o) {
    le = le && d[o] <= 0.0;
    lt = lt || d[o] < 0.0;
  }
  bool accept = le && lt;
  bool improves = false;
  for (int o = 0; o < kOut; ++o) improves = improves || d[o] < 0.0;
  if (!accept && improves && obj && n_arch > 0) {
    double nv[kOut];
    for (int o = 0; o < kOut; ++o) nv[o] = obj[(size_t)s * kOut + o] + d[o];
    bool dominated = false;
    for (int a = 0; a < n_arch && !dominated; ++a) {
      if (arch[(size_t)a * kOut] == INFINITY) break;  // padding ends the archive
      bool ale = true, alt = false;
      for (int o = 0; o < kOut; ++o) {
        ale = ale && arch[(size_t)a * kOut + o] <= nv[o];
        alt = alt || arch[(size_t)a * kOut + o] < nv[o];
      }
      dominated = ale && alt;
    }
    accept = !dominated;
  }
  pick[e] = best;
  run_exact[e] = accept ? 1 : 0;
}

// Gathers the picked candidate of every (solution, element): [S][F][K][2][3] -> [S][F][2][3].
__global__ void k_gather_pick(int S, int F, int K, const float* __restrict__ cand, const int* __restrict__ pick,
                              float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * F * 6) return;
  const int sf = e / 6, c = e % 6;
  const int k = min(max(pick[sf], 0), K - 1);
  out[e] = cand[((size_t)sf * K + k) * 6 + c];
}

}  // namespace
}  // namespace dsm

using namespace dsm;

struct dsm_surrogate {
  dsm_surrogate_desc desc{};
  int device = 0;
  int64_t step = 0;  // Adam steps taken
  float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
  unsigned short *d_w1 = nullptr, *d_w2 = nullptr, *d_w3 = nullptr, *d_w2t = nullptr, *d_w3t = nullptr;
  float *d_in_mean = nullptr, *d_in_rstd = nullptr, *d_out_mean = nullptr, *d_out_rstd = nullptr, *d_out_scale = nullptr;
  // training workspace for max_batch rows (padded to a multiple of 32)
  int bpad = 0;
  unsigned short *d_xt = nullptr, *d_h1t = nullptr, *d_h2t = nullptr, *d_dyt = nullptr, *d_dz2t = nullptr,
                 *d_dz1t = nullptr;
  float* d_row_loss = nullptr;
  int* d_idx = nullptr;
  // screening workspace for max_rows rows
  unsigned short* d_featb = nullptr;  // [max_rows][192]
  float* d_pred = nullptr;            // [max_rows][3]
};

namespace {

thread_local std::string s_err;

dsm_status sfail(dsm_status st, const char* msg) {
  s_err = msg;
  return st;
}

MlpW weights(const dsm_surrogate* m) {
  MlpW w;
  w.w1 = m->d_w1;
  w.w2 = m->d_w2;
  w.w3 = m->d_w3;
  w.w2t = m->d_w2t;
  w.w3t = m->d_w3t;
  w.b1 = m->d_params + kB1;
  w.b2 = m->d_params + kB2;
  w.b3 = m->d_params + kB3;
  return w;
}

void free_sur(dsm_surrogate* m) {
  if (!m) return;
  void* bufs[] = {m->d_params, m->d_m,      m->d_v,        m->d_grad,     m->d_w1,      m->d_w2,   m->d_w3,
                  m->d_w2t,    m->d_w3t,    m->d_in_mean,  m->d_in_rstd,  m->d_out_mean, m->d_out_rstd,
                  m->d_out_scale, m->d_xt,  m->d_h1t,      m->d_h2t,      m->d_dyt,     m->d_dz2t, m->d_dz1t,
                  m->d_row_loss, m->d_idx,  m->d_featb,    m->d_pred};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete m;
}

hipError_t refresh(dsm_surrogate* m, hipStream_t st) {
  k_refresh_bf16<<<(kHid * kIn + 255) / 256, 256, 0, st>>>(m->d_params, m->d_w1, m->d_w2, m->d_w3, m->d_w2t, m->d_w3t);
  return hipGetLastError();
}

// forward + backward of B rows given by d_idx; writes the gradient into d_grad
hipError_t gradient_pass(dsm_surrogate* m, const unsigned short* feats, const float* targets, int B, float* loss,
                         hipStream_t st) {
  const int ld = (B + 31) / 32 * 32;
  TrainWs ws{m->d_xt, m->d_h1t, m->d_h2t, m->d_dyt, m->d_dz2t, m->d_dz1t, m->d_row_loss, ld};
  k_mlp_rows<<<ld / 16, 64, 0, st>>>(weights(m), feats, targets, m->d_idx, B, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_mlp_wgrad<<<dim3(kIn / 16, kHid / 16), 64, 0, st>>>(m->d_dz1t, m->d_xt, ld, kIn, m->d_grad + kW1);
  k_mlp_wgrad<<<dim3(kHid / 16, kHid / 16), 64, 0, st>>>(m->d_dz2t, m->d_h1t, ld, kHid, m->d_grad + kW2);
  k_mlp_wgrad<<<dim3(kHid / 16, kOutPad / 16), 64, 0, st>>>(m->d_dyt, m->d_h2t, ld, kHid, m->d_grad + kW3);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_mlp_bias_loss<<<2 * kHid + kOutPad + 1, 64, 0, st>>>(m->d_dz1t, m->d_dz2t, m->d_dyt, m->d_row_loss, B, ld,
                                                                    m->d_grad, loss);
  return hipGetLastError();
}

}  // namespace

extern "C" {

const char* dsm_surrogate_last_error(void) { return s_err.c_str(); }

dsm_status dsm_surrogate_create(const dsm_surrogate_desc* d, dsm_surrogate** out) {
  s_err.clear();
  if (!out || !d) return sfail(DSM_ERR_ARG, "null argument");
  *out = nullptr;
  if (d->max_rows < 1 || d->max_batch < 32 || d->max_batch % 32 != 0)
    return sfail(DSM_ERR_ARG, "max_rows >= 1 and max_batch a positive multiple of 32 required");
  if (!(d->lr > 0.f) || !(d->beta1 >= 0.f && d->beta1 < 1.f) || !(d->beta2 >= 0.f && d->beta2 < 1.f) || !(d->eps > 0.f))
    return sfail(DSM_ERR_ARG, "bad Adam hyper-parameters");
  auto* m = new dsm_surrogate();
  m->desc = *d;
  m->bpad = d->max_batch;
  hipError_t e = hipGetDevice(&m->device);
#define S_TRY(expr)                                   \
  if (e == hipSuccess) e = (expr);                    \
  if (e != hipSuccess) {                              \
    free_sur(m);                                      \
    return sfail(e == hipErrorOutOfMemory ? DSM_ERR_NOMEM : DSM_ERR_DEVICE, hipGetErrorString(e)); \
  }
  S_TRY(hipMalloc(&m->d_params, sizeof(float) * kNParams));
  S_TRY(hipMalloc(&m->d_m, sizeof(float) * kNParams));
  S_TRY(hipMalloc(&m->d_v, sizeof(float) * kNParams));
  S_TRY(hipMalloc(&m->d_grad, sizeof(float) * kNParams));
  S_TRY(hipMalloc(&m->d_w1, 2 * kHid * kIn));
  S_TRY(hipMalloc(&m->d_w2, 2 * kHid * kHid));
  S_TRY(hipMalloc(&m->d_w3, 2 * kOutPad * kHid));
  S_TRY(hipMalloc(&m->d_w2t, 2 * kHid * kHid));
  S_TRY(hipMalloc(&m->d_w3t, 2 * kOutPad * kHid));
  S_TRY(hipMalloc(&m->d_in_mean, sizeof(float) * kIn));
  S_TRY(hipMalloc(&m->d_in_rstd, sizeof(float) * kIn));
  S_TRY(hipMalloc(&m->d_out_mean, sizeof(float) * kOut));
  S_TRY(hipMalloc(&m->d_out_rstd, sizeof(float) * kOut));
  S_TRY(hipMalloc(&m->d_out_scale, sizeof(float) * kOut));
  const size_t B = m->bpad;
  S_TRY(hipMalloc(&m->d_xt, 2 * kIn * B));
  S_TRY(hipMalloc(&m->d_h1t, 2 * kHid * B));
  S_TRY(hipMalloc(&m->d_h2t, 2 * kHid * B));
  S_TRY(hipMalloc(&m->d_dyt, 2 * kOutPad * B));
  S_TRY(hipMalloc(&m->d_dz2t, 2 * kHid * B));
  S_TRY(hipMalloc(&m->d_dz1t, 2 * kHid * B));
  S_TRY(hipMalloc(&m->d_row_loss, sizeof(float) * B));
  S_TRY(hipMalloc(&m->d_idx, sizeof(int) * B));
  S_TRY(hipMalloc(&m->d_featb, 2 * kIn * (size_t)d->max_rows));
  S_TRY(hipMalloc(&m->d_pred, sizeof(float) * kOut * (size_t)d->max_rows));
  // He-uniform initial weights, zero biases (host, from the seed); identity scaling
  std::vector<float> p(kNParams, 0.f);
  unsigned long long z = d->seed;
  auto next = [&z]() {
    z += 0x9e3779b97f4a7c15ull;
    unsigned long long x = z;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    x ^= x >> 31;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int rows, int cols, int fan_in) {
    const double lim = sqrt(6.0 / fan_in);
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) p[off + r * cols + c] = (float)((2.0 * next() - 1.0) * lim);
  };
  fill(kW1, kHid, kIn, kIn);
  fill(kW2, kHid, kHid, kHid);
  fill(kW3, kOut, kHid, kHid);  // output rows 3..15 stay zero
  S_TRY(hipMemcpy(m->d_params, p.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
  S_TRY(hipMemset(m->d_m, 0, sizeof(float) * kNParams));
  S_TRY(hipMemset(m->d_v, 0, sizeof(float) * kNParams));
  S_TRY(hipMemset(m->d_grad, 0, sizeof(float) * kNParams));
  std::vector<float> zeros(kIn, 0.f), ones(kIn, 1.f);
  S_TRY(hipMemcpy(m->d_in_mean, zeros.data(), sizeof(float) * kIn, hipMemcpyHostToDevice));
  S_TRY(hipMemcpy(m->d_in_rstd, ones.data(), sizeof(float) * kIn, hipMemcpyHostToDevice));
  S_TRY(hipMemcpy(m->d_out_mean, zeros.data(), sizeof(float) * kOut, hipMemcpyHostToDevice));
  S_TRY(hipMemcpy(m->d_out_rstd, ones.data(), sizeof(float) * kOut, hipMemcpyHostToDevice));
  S_TRY(hipMemcpy(m->d_out_scale, ones.data(), sizeof(float) * kOut, hipMemcpyHostToDevice));
  S_TRY(refresh(m, nullptr));
  S_TRY(hipDeviceSynchronize());
#undef S_TRY
  *out = m;
  return DSM_OK;
}

dsm_status dsm_surrogate_destroy(dsm_surrogate* m) {
  s_err.clear();
  if (!m) return sfail(DSM_ERR_ARG, "null surrogate");
  free_sur(m);
  return DSM_OK;
}

dsm_status dsm_surrogate_params(dsm_surrogate* m, float* host, int32_t set) {
  s_err.clear();
  if (!m || !host) return sfail(DSM_ERR_ARG, "null argument");
  hipError_t e;
  if (set) {
    e = hipMemcpy(m->d_params, host, sizeof(float) * kNParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = refresh(m, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  } else {
    e = hipMemcpy(host, m->d_params, sizeof(float) * kNParams, hipMemcpyDeviceToHost);
  }
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_fit_scaling(dsm_surrogate* m, int32_t N, const float* feats, const float* deltas, void* stream) {
  s_err.clear();
  if (!m || !feats || !deltas || N < 1) return sfail(DSM_ERR_ARG, "null argument or N < 1");
  hipStream_t st = (hipStream_t)stream;
  k_column_stats<<<kIn, 256, 0, st>>>(N, kIn, feats, m->d_in_mean, m->d_in_rstd);
  k_column_stats<<<kOut, 256, 0, st>>>(N, kOut, deltas, m->d_out_mean, m->d_out_rstd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
  // output scale = 1 / rstd (so that raw = std_pred * scale + mean)
  std::vector<float> r(kOut);
  e = hipMemcpyAsync(r.data(), m->d_out_rstd, sizeof(float) * kOut, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (float& x : r) x = 1.f / x;
  if (e == hipSuccess) e = hipMemcpy(m->d_out_scale, r.data(), sizeof(float) * kOut, hipMemcpyHostToDevice);
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_get_scaling(dsm_surrogate* m, float* in_mean, float* in_rstd, float* out_mean, float* out_rstd) {
  s_err.clear();
  if (!m) return sfail(DSM_ERR_ARG, "null surrogate");
  hipError_t e = hipSuccess;
  if (in_mean) e = hipMemcpy(in_mean, m->d_in_mean, sizeof(float) * kIn, hipMemcpyDeviceToHost);
  if (e == hipSuccess && in_rstd) e = hipMemcpy(in_rstd, m->d_in_rstd, sizeof(float) * kIn, hipMemcpyDeviceToHost);
  if (e == hipSuccess && out_mean) e = hipMemcpy(out_mean, m->d_out_mean, sizeof(float) * kOut, hipMemcpyDeviceToHost);
  if (e == hipSuccess && out_rstd) e = hipMemcpy(out_rstd, m->d_out_rstd, sizeof(float) * kOut, hipMemcpyDeviceToHost);
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_set_scaling(dsm_surrogate* m, const float* in_mean, const float* in_rstd, const float* out_mean,
                                     const float* out_rstd) {
  s_err.clear();
  if (!m || !in_mean || !in_rstd || !out_mean || !out_rstd) return sfail(DSM_ERR_ARG, "null argument");
  hipError_t e = hipMemcpy(m->d_in_mean, in_mean, sizeof(float) * kIn, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_in_rstd, in_rstd, sizeof(float) * kIn, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_out_mean, out_mean, sizeof(float) * kOut, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_out_rstd, out_rstd, sizeof(float) * kOut, hipMemcpyHostToDevice);
  float sc[kOut];
  for (int o = 0; o < kOut; ++o) sc[o] = 1.f / out_rstd[o];
  if (e == hipSuccess) e = hipMemcpy(m->d_out_scale, sc, sizeof(float) * kOut, hipMemcpyHostToDevice);
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_features(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts, int32_t K,
                                  const float* cand, float* feats, void* stream) {
  s_err.clear();
  if (!p || S < 0 || F < 0 || K < 1) return sfail(DSM_ERR_ARG, "null problem or bad sizes");
  const int64_t n = (int64_t)S * F * K;
  if (n == 0) return DSM_OK;
  if (!X || !fos_pts || !cand || !feats) return sfail(DSM_ERR_ARG, "null argument");
  k_features<false><<<(unsigned)((n + 7) / 8), 256, 0, (hipStream_t)stream>>>(p->dev, X, S, F, fos_pts, K, cand, p->d_ident,
                                                                           nullptr, nullptr, feats, nullptr);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_features_packed(dsm_surrogate* m, dsm_problem* p, int32_t S, const float* X, int32_t F,
                                         const int32_t* fos_pts, int32_t K, const float* cand, uint16_t* feats_bf16,
                                         void* stream) {
  s_err.clear();
  if (!m || !p || S < 0 || F < 0 || K < 1) return sfail(DSM_ERR_ARG, "null argument or bad sizes");
  const int64_t n = (int64_t)S * F * K;
  if (n == 0) return DSM_OK;
  if (!X || !fos_pts || !cand || !feats_bf16) return sfail(DSM_ERR_ARG, "null argument");
  k_features<true><<<(unsigned)((n + 7) / 8), 256, 0, (hipStream_t)stream>>>(p->dev, X, S, F, fos_pts, K, cand, p->d_ident,
                                                                          m->d_in_mean, m->d_in_rstd, nullptr,
                                                                          (unsigned short*)feats_bf16);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_pack(dsm_surrogate* m, int32_t N, const float* feats, uint16_t* feats_bf16, const double* part_old,
                              const double* part_new, float* targets, float* raw_deltas, void* stream) {
  s_err.clear();
  if (!m || N < 0) return sfail(DSM_ERR_ARG, "null surrogate or N < 0");
  if (N == 0) return DSM_OK;
  hipStream_t st = (hipStream_t)stream;
  if (feats && feats_bf16)
    k_pack<<<(unsigned)(((int64_t)N * kIn + 255) / 256), 256, 0, st>>>(N, feats, m->d_in_mean, m->d_in_rstd, feats_bf16);
  if (part_old && part_new && (targets || raw_deltas))
    k_targets<<<(N * kOut + 255) / 256, 256, 0, st>>>(N, part_old, part_new, m->d_out_mean, m->d_out_rstd, targets,
                                                       raw_deltas);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_forward(dsm_surrogate* m, int32_t N, const uint16_t* feats_bf16, float* pred, void* stream) {
  s_err.clear();
  if (!m || !feats_bf16 || !pred || N < 0) return sfail(DSM_ERR_ARG, "null argument");
  if (N == 0) return DSM_OK;
  k_mlp_forward64<<<(N + 63) / 64, 256, 0, (hipStream_t)stream>>>(weights(m), (const unsigned short*)feats_bf16, N, pred);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_gradient(dsm_surrogate* m, int32_t N, const uint16_t* feats_bf16, const float* targets, float* grad,
                                  float* loss, void* stream) {
  s_err.clear();
  if (!m || !feats_bf16 || !targets || !grad) return sfail(DSM_ERR_ARG, "null argument");
  if (N < 1 || N > m->bpad) return sfail(DSM_ERR_CAPACITY, "N outside [1, max_batch]");
  hipStream_t st = (hipStream_t)stream;
  k_iota<<<(m->bpad + 255) / 256, 256, 0, st>>>(N, m->d_idx);
  hipError_t e = gradient_pass(m, (const unsigned short*)feats_bf16, targets, N, loss, st);
  if (e == hipSuccess) e = hipMemcpyAsync(grad, m->d_grad, sizeof(float) * kNParams, hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_train(dsm_surrogate* m, int32_t N, const uint16_t* feats_bf16, const float* targets, int32_t steps,
                               int32_t batch, float* loss, void* stream) {
  s_err.clear();
  if (!m || !feats_bf16 || !targets || N < 1 || steps < 0) return sfail(DSM_ERR_ARG, "null argument or bad sizes");
  if (batch < 1 || batch > m->bpad || batch % 32 != 0)
    return sfail(DSM_ERR_CAPACITY, "batch must be a multiple of 32 within max_batch");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int k = 0; k < steps && e == hipSuccess; ++k) {
    k_batch_indices<<<(batch + 255) / 256, 256, 0, st>>>(m->desc.seed, (int)m->step, N, batch, batch, m->d_idx);
    e = gradient_pass(m, (const unsigned short*)feats_bf16, targets, batch, loss ? loss + k : nullptr, st);
    if (e != hipSuccess) break;
    m->step++;
    const float c1 = 1.f - powf(m->desc.beta1, (float)m->step), c2 = 1.f - powf(m->desc.beta2, (float)m->step);
    k_adam<<<(kNParams + 255) / 256, 256, 0, st>>>(m->d_params, m->d_grad, m->d_m, m->d_v, m->desc.lr, m->desc.beta1,
                                                  m->desc.beta2, m->desc.eps, c1, c2);
    e = hipGetLastError();
    if (e == hipSuccess) e = refresh(m, st);
  }
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

dsm_status dsm_surrogate_screen(dsm_surrogate* m, dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_pts,
                                int32_t K, const float* cand, const double* obj, int32_t n_archive, const double* archive,
                                float* pred, int32_t* pick, uint8_t* run_exact, float* cand_pick, void* stream) {
  s_err.clear();
  if (!m || !p || !X || !fos_pts || !cand || !pick || !run_exact) return sfail(DSM_ERR_ARG, "null argument");
  if (S < 0 || F < 0 || K < 1 || n_archive < 0 || (n_archive > 0 && !archive)) return sfail(DSM_ERR_ARG, "bad sizes");
  const int64_t n = (int64_t)S * F * K;
  if (n > m->desc.max_rows) return sfail(DSM_ERR_CAPACITY, "S*F*K exceeds max_rows");
  if (n == 0) return DSM_OK;
  hipStream_t st = (hipStream_t)stream;
  k_features<true><<<(unsigned)((n + 7) / 8), 256, 0, st>>>(p->dev, X, S, F, fos_pts, K, cand, p->d_ident, m->d_in_mean,
                                                            m->d_in_rstd, nullptr, m->d_featb);
  k_mlp_forward64<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(weights(m), m->d_featb, (int)n, m->d_pred);
  k_select<<<(S * F + 255) / 256, 256, 0, st>>>(S, F, K, m->d_pred, m->d_out_mean, m->d_out_scale, obj, n_archive, archive,
                                                 pred, pick, run_exact);
  if (cand_pick) k_gather_pick<<<(S * F * 6 + 255) / 256, 256, 0, st>>>(S, F, K, cand, pick, cand_pick);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DSM_OK : sfail(DSM_ERR_DEVICE, hipGetErrorString(e));
}

}  // extern "C"
