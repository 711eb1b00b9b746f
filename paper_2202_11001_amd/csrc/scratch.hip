// Partial evaluation that allocates nothing: its workspace (affected sets,
// element order, swept dissimilarity per tetrahedron, per-chunk flags and
// voxel counts) lives in a fixed device array instead of the problem's
// create-time workspace.  The kernels are those of dsm_eval_partial.
#include <stdio.h>

#include <mutex>

#include "dsm_internal.h"

namespace dsm {
namespace {

constexpr size_t kScratchBytes = size_t(DSM_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  In host code the name is
// only a handle for hipGetSymbolAddress: kernels receive the device address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// Address of this device's `scratch`, looked up with the device current on
// the first call that runs on it.
hipError_t scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the workspace regions inside `scratch`.
struct ScratchLayout {
  size_t aff, aff_cnt, order, simws, cflags, ccount, total;
};

ScratchLayout scratch_layout(int S, int F, int maxA, int nver, int nchunk) {
  ScratchLayout L;
  size_t o = 0;
  L.aff = o;
  o = align256(o + sizeof(int) * (size_t)F * maxA);
  L.aff_cnt = o;
  o = align256(o + sizeof(int) * (size_t)F);
  L.order = o;
  o = align256(o + sizeof(int) * (size_t)F);
  L.simws = o;
  o = align256(o + sizeof(double) * (size_t)S * F * nver * maxA);
  L.cflags = o;
  o = align256(o + sizeof(uint32_t) * (size_t)S * F * nchunk);
  L.ccount = o;
  o = align256(o + sizeof(uint32_t) * (size_t)S * F * nchunk);
  L.total = o;
  return L;
}

}  // namespace
}  // namespace dsm

using namespace dsm;

extern "C" {

dsm_status dsm_eval_partial_noalloc(dsm_problem* p, int32_t S, const float* X, int32_t F, const int32_t* fos_off,
                                    const int32_t* fos_pts, const float* cand, const double* tet_terms_in,
                                    double* part_old, double* part_new, uint32_t* flags, double* tet_terms_new,
                                    uint32_t* voxel_count, void* stream) {
  clear_error();
  char msg[256];
  if (!p) return set_error(DSM_ERR_ARG, "null argument");
  if (S < 0 || F < 0) return set_error(DSM_ERR_ARG, "negative S or F");
  if (S == 0 || F == 0) return DSM_OK;  // empty buffers may be null
  if (!X || !fos_off || !fos_pts || !cand || !part_old || !part_new || !flags)
    return set_error(DSM_ERR_ARG, "null argument");
  int device = -1;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return set_error(DSM_ERR_DEVICE, hipGetErrorString(e));
  if (device != p->device) {
    snprintf(msg, sizeof msg, "the problem lives on device %d but device %d is current", p->device, device);
    return set_error(DSM_ERR_ARG, msg);
  }
  if (device < 0 || device >= kMaxDevices) return set_error(DSM_ERR_UNSUPPORTED, "device index above 63");
  const int nver = tet_terms_in ? 1 : 2;
  const int nchunk = p->nchunk;
  const ScratchLayout L = scratch_layout(S, F, p->maxA, nver, nchunk);
  if (L.total > kScratchBytes) {
    snprintf(msg, sizeof msg,
             "S = %d, F = %d needs %zu bytes of workspace; the fixed workspace holds %zu (split the population)", S, F,
             L.total, kScratchBytes);
    return set_error(DSM_ERR_CAPACITY, msg);
  }
  unsigned char* base = nullptr;
  if ((e = scratch_address(device, &base)) != hipSuccess) return set_error(DSM_ERR_DEVICE, hipGetErrorString(e));
  int* aff = (int*)(base + L.aff);
  int* aff_cnt = (int*)(base + L.aff_cnt);
  int* order = (int*)(base + L.order);
  hipStream_t st = (hipStream_t)stream;
  e = launch_affected(p->dev, F, fos_off, fos_pts, p->max_pts, p->maxA, aff, aff_cnt, st);
  if (e == hipSuccess && F <= kOrderMax) e = launch_order(F, aff_cnt, order, st);
  if (e != hipSuccess) return set_error(DSM_ERR_DEVICE, hipGetErrorString(e));
  EvalArgs a{};
  a.pr = p->dev;
  a.S = S;
  a.G = F;
  a.partial = 1;
  a.X = X;
  a.fos_off = fos_off;
  a.fos_pts = fos_pts;
  a.cand = cand;
  a.aff = aff;
  a.aff_cnt = aff_cnt;
  a.order = F <= kOrderMax ? order : nullptr;
  a.maxA = p->maxA;
  a.nver = nver;
  a.terms_in = tet_terms_in;
  a.part_old = part_old;
  a.part_new = part_new;
  a.flags = flags;
  a.terms_out = tet_terms_new;
  a.vcount = voxel_count;
  a.mask = nullptr;
  a.simws = (double*)(base + L.simws);
  a.pchunk = p->part_chunk;
  a.row_pairs = p->row_order;
  a.nchunk = nchunk;
  a.cflags = (uint32_t*)(base + L.cflags);
  a.ccount = (uint32_t*)(base + L.ccount);
  if ((e = launch_eval(a, nullptr, nullptr, st)) != hipSuccess) return set_error(DSM_ERR_DEVICE, hipGetErrorString(e));
  return DSM_OK;
}

}  // extern "C"
