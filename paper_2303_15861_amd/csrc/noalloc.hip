// Exponential action without any device allocation, for callers that cannot allocate
// (code under HIP graph capture, allocation-free serving loops): the FP64 mu-mode
// product out = in x_1 E_1 x_2 E_2 (x_3 E_3) (Sec. 1, Sec. 5.2) with caller-owned
// factors, its intermediates in a file-scope device array instead of operator scratch.
//
// The array is a static __device__ object: every GPU the library runs on holds its own
// copy, at its own address, until the process ends. Host code never uses the array's
// name as an address (on the host it only names the symbol); mm_ctx_create resolves the
// device address once per device with hipGetSymbolAddress, with that device current,
// and every kernel argument uses the resolved pointer.
#include <mutex>

#include "mm_internal.h"

namespace mm {

namespace {

constexpr int kMaxDevices = 64;

// two grid functions of up to kNoAllocMaxDof values (2 x 16 MiB)
__device__ __align__(256) double scratch[2 * (size_t)kNoAllocMaxDof];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// One FP64 mode pass of an action on a d-dimensional grid (layouts as in exp_action):
// out = in x_mu M, M row-major n_mu x n_mu.
hipError_t fp64_pass(int d, const int* n, int mu, const double* M, const double* in, double* out, int tile,
                     hipStream_t s) {
  const int64_t dof = (int64_t)n[0] * n[1] * (d == 3 ? n[2] : 1);
  GemmArgs g{};
  g.groups = 1;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.Cadd[0] = nullptr;
  g.C[0] = out;
  g.inner = 1;
  g.tile = tile;
  const int nm = n[mu];
  if (mu == 0) {
    g.A[0] = in;
    g.B[0] = M;
    g.M = (int)(dof / nm);
    g.N = g.K = nm;
    g.lda = g.ldb = g.ldc = nm;
    g.b_trans = 0;
  } else if (mu == d - 1) {
    const int P = (int)(dof / nm);
    g.A[0] = M;
    g.B[0] = in;
    g.M = g.K = nm;
    g.N = P;
    g.lda = nm;
    g.ldb = g.ldc = P;
    g.b_trans = 1;
  } else {   // x2 of a 3D grid: per x3 slab
    g.A[0] = M;
    g.B[0] = in;
    g.M = g.K = nm;
    g.N = n[0];
    g.lda = nm;
    g.ldb = g.ldc = n[0];
    g.inner = n[2];
    g.sA = 0;
    g.sB = g.sC = (int64_t)n[0] * n[1];
    g.b_trans = 1;
  }
  return launch_gemm(MM_FP64, g, s);
}

}  // namespace

hipError_t noalloc_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // device `device` is current
  if (e != hipSuccess) return e;
  g_scratch[device] = (double*)p;
  return hipSuccess;
}

}  // namespace mm

extern "C" mm_status mumode_expv_noalloc(mm_ctx* ctx, int d, const int* n, const double* const* E,
                                         const double* in, double* out, void* stream) {
  if (!ctx) return MM_EINVAL;
  if ((d != 2 && d != 3) || !n || !E || !in || !out) {
    ctx->last_error = "mumode_expv_noalloc: d must be 2 or 3 and n, E, in, out non-null";
    return MM_EINVAL;
  }
  int64_t dof = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1 || n[mu] > 4096 || !E[mu]) {
      ctx->last_error = "mumode_expv_noalloc: every n[mu] must be in 1..4096 with a factor E[mu]";
      return MM_EINVAL;
    }
    dof *= n[mu];
  }
  if (dof > mm::kNoAllocMaxDof) {
    ctx->last_error = "mumode_expv_noalloc: n1*n2*n3 = " + std::to_string(dof) + " exceeds the scratch limit of " +
                      std::to_string(mm::kNoAllocMaxDof) + " grid values";
    return MM_EINVAL;
  }
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(mm::g_mu);
    if (ctx->device >= 0 && ctx->device < mm::kMaxDevices) base = mm::g_scratch[ctx->device];
  }
  if (!base) {
    ctx->last_error = "mumode_expv_noalloc: the scratch address of this device was not resolved";
    return MM_EDEVICE;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ctx->last_error = "mumode_expv_noalloc: hipSetDevice failed";
    return MM_EDEVICE;
  }
  hipStream_t s = (hipStream_t)stream;
  double* s0 = base;
  double* s1 = base + mm::kNoAllocMaxDof;
  int nn[3] = {n[0], n[1], d == 3 ? n[2] : 1};
  const int tile = ctx->gemm_tile;
  hipError_t e;
  // 3D: in -> s0 -> s1 -> out; 2D: in -> s0 -> out (in and out may alias)
  e = mm::fp64_pass(d, nn, 0, E[0], in, s0, tile, s);
  if (e == hipSuccess && d == 3) e = mm::fp64_pass(d, nn, 1, E[1], s0, s1, tile, s);
  if (e == hipSuccess) e = mm::fp64_pass(d, nn, d - 1, E[d - 1], d == 3 ? s1 : s0, out, tile, s);
  if (e != hipSuccess) {
    ctx->last_error = std::string("mumode_expv_noalloc: launch failed: ") + hipGetErrorString(e);
    return MM_EDEVICE;
  }
  return MM_OK;
}
