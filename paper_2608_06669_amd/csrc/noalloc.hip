// cc_gemm_noalloc: the batched matrix-core product of cc_diag_gemm_batched
// with its scratch memory (split-K partial sums, operands rounded once to
// FP32/BF16) taken from a fixed device array instead of hipMalloc, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops).
//
// The array lives in this file as a __device__ global. Its address on a
// device is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept; kernels only ever receive that address. Every
// call on a device shares the device's array, so calls that overlap on one
// device race; nothing in it needs clearing between calls (every split-K
// partial sum and every rounded operand element a product reads is written
// by the same call first).

#include <algorithm>
#include <mutex>

#include "../../include/pnkcc.h"
#include "api_internal.hpp"
#include "gemm.hpp"

using namespace pnk;

// 32 MiB of split-K partial sums (4 Mi doubles, the cap cc_diag_gemm_batched
// uses too), then 32 MiB of rounded operand copies.
static constexpr size_t kSplitBytes = sizeof(double) * kDiagSplitElems;
static_assert(kSplitBytes == size_t(32) << 20, "split-K part of the array");
static constexpr size_t kCastBytes = size_t(32) << 20;
static constexpr size_t kScratchBytes = kSplitBytes + kCastBytes;

// Host code never uses this name as an address: only the per-device
// address from hipGetSymbolAddress below reaches kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
cc_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return CC_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CC_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return CC_OK;
}

}  // namespace

extern "C" cc_status cc_gemm_noalloc(int M, int N, int K, int nbatch, const double* A, int64_t a_m, int64_t a_k,
                                     int64_t a_b, const double* B, int64_t b_k, int64_t b_n, int64_t b_b, double* C,
                                     int64_t c_m, int64_t c_n, int64_t c_b, double alpha, double beta,
                                     cc_precision prec, int flags, void* stream) {
  if (M < 1 || N < 1 || K < 1 || nbatch < 1 || !A || !B || !C) return CC_ERR_ARG;
  if (prec != CC_FP64 && prec != CC_FP32 && prec != CC_BF16) return CC_ERR_ARG;
  if (flags & ~3) return CC_ERR_ARG;
  // the rounded operand copies must fit their part of the array
  const bool precast = (flags & 1) && prec != CC_FP64;
  if (precast && (size_t)diag_cast_bytes(nbatch, M, N, K, prec) > kCastBytes) return CC_ERR_OOM;
  void* base = nullptr;
  const cc_status st = scratch_ptr(&base);
  if (st != CC_OK) return st;
  try {
    GemmDesc d;
    d.M = M; d.N = N; d.K = K;
    d.nb0 = nbatch;
    d.a_m = a_m; d.a_k = a_k; d.a_b0 = a_b;
    d.b_k = b_k; d.b_n = b_n; d.b_b0 = b_b;
    d.c_m = c_m; d.c_n = c_n; d.c_b0 = c_b;
    d.alpha = alpha; d.beta = beta;
    if (flags & 2) {
      d.ws = (double*)base;
      d.ws_elems = diag_splitk_elems(nbatch, M, N);
    }
    if (precast) {
      d.cast_ws = (unsigned char*)base + kSplitBytes;
      d.cast_ws_bytes = diag_cast_bytes(nbatch, M, N, K, prec);
    }
    gemm(d, A, Prec::F64, B, Prec::F64, C, Prec::F64, (Prec)prec, (hipStream_t)stream);
  } catch (const ArgError&) {
    return CC_ERR_ARG;
  } catch (const std::exception&) {
    (void)hipGetLastError();
    return CC_ERR_HIP;
  }
  return CC_OK;
}
