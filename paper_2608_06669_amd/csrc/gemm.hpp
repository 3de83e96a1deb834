// Strided, batched matrix products on the CDNA4 matrix cores.
//
//   C[b] = alpha * A[b] * B[b] + beta * C[b]
//
// Every operand is addressed by explicit element strides, so transposes and
// index permutations of 4-index tensors need no copies whenever the merged
// row, column and contraction indices are each a single arithmetic
// progression. The batch index is two-dimensional (b = b1 * nb0 + b0) with
// separate strides, which covers products like X_ab[c][d] = sum_P
// L[P][a][c] L[P][b][d] where A depends on a only and B on b only.
#pragma once

#include "common.hpp"

namespace pnk {

struct GemmDesc {
  int M = 0, N = 0, K = 0;
  int nb0 = 1, nb1 = 1;
  // element strides (not bytes)
  int64_t a_m = 0, a_k = 0, a_b0 = 0, a_b1 = 0;
  int64_t b_k = 0, b_n = 0, b_b0 = 0, b_b1 = 0;
  int64_t c_m = 0, c_n = 0, c_b0 = 0, c_b1 = 0;
  double alpha = 1.0, beta = 0.0;
  // Optional scratch for split-K: products with too few output tiles to
  // fill the GPU split the contraction into S chunks whose partial sums go
  // here and are then added in a fixed order (deterministic). Needs S *
  // nb0 * nb1 * M * N doubles; S is reduced to fit ws_elems.
  double* ws = nullptr;
  int64_t ws_elems = 0;
  // Optional scratch for FP32/BF16 products with FP64 operands: large
  // products first round each FP64 operand once into this buffer (rows
  // contiguous along k) instead of converting it in every tile that reads
  // it. Products whose packed operands do not fit are converted on load.
  void* cast_ws = nullptr;
  int64_t cast_ws_bytes = 0;
  // B stored in the compute type along k, rows readable and zero from K up
  // to this length (0: not known): a product whose A is packed may then run
  // its contraction over whole panels
  int64_t b_kzero = 0;
};

// Pointers carry their storage precision; `compute` selects the matrix-core
// instruction (F64: 4x4x4 f64; F32: 16x16x4 f32; BF16: 16x16x32 bf16),
// with float accumulation for F32 and BF16. Operands stored in a wider type
// are rounded to the compute type while being staged into LDS.
void gemm(const GemmDesc& d, const void* A, Prec a_prec, const void* B, Prec b_prec,
          void* C, Prec c_prec, Prec compute, hipStream_t stream);

// C = alpha (A1 B1 + A2 B2) + beta C in one launch: both products share
// strides, storage precisions (ap for A1, A2; bp for B1, B2) and the
// contraction length, and accumulate into the same registers.
void gemm_sum(const GemmDesc& d, const void* A1, const void* B1, const void* A2, const void* B2, Prec ap, Prec bp,
              void* C, Prec cp, Prec compute, hipStream_t stream);

// Convenience for all-FP64 products.
inline void gemm64(const GemmDesc& d, const double* A, const double* B, double* C,
                   hipStream_t s) {
  gemm(d, A, Prec::F64, B, Prec::F64, C, Prec::F64, Prec::F64, s);
}

}  // namespace pnk
