// Bandwidth-bound tensor kernels: permutations, vector updates, reductions.
#pragma once

#include "common.hpp"

namespace pnk {

// out[perm(idx)] = alpha * in[idx] + beta * out[perm(idx)] for a row-major
// 4-index tensor `in` of shape d[0..3]; output axis k is input axis perm[k].
// Tiles through LDS whenever the two fastest axes differ, so both the reads
// and the writes are coalesced.
void permute4(const double* in, double* out, const int d[4], const int perm[4], double alpha,
              double beta, hipStream_t s);

// y = a * x + b * y (b == 0: y is not read)
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
void fill(int64_t n, double v, double* y, hipStream_t s);
// y = x (device to device, on the stream)
void copy(int64_t n, const double* x, double* y, hipStream_t s);
// y[i] = (float or bf16 bits) x[i]
void cast_f64_to_f32(int64_t n, const double* x, float* y, hipStream_t s);
void cast_f64_to_bf16(int64_t n, const double* x, uint16_t* y, hipStream_t s);
// x [rows][cols] to y [rows][ld] (ld >= cols, padding zeroed), so that rows
// start on 16-byte boundaries for the matrix-core products' vector loads
void cast_f64_to_f32_rows(int64_t rows, int64_t cols, int64_t ld, const double* x, float* y, hipStream_t s);
void cast_f64_to_bf16_rows(int64_t rows, int64_t cols, int64_t ld, const double* x, uint16_t* y, hipStream_t s);

// R[i][j][a][b] += alpha * (X[i][j][a][b] + X[j][i][b][a])
void pair_symmetrize_add(int o, int v, const double* X, double alpha, double* R, hipStream_t s);

// Deterministic reductions: the result is written to a device double and
// does not depend on the launch (fixed block count and fixed summation
// order). `partials` needs reduce_partials_size() doubles.
constexpr int kReduceBlocks = 512;
int64_t reduce_partials_size(int nvec);
void dot(int64_t n, const double* x, const double* y, double* out, double* partials, hipStream_t s);
void nrm2(int64_t n, const double* x, double* out, double* partials, hipStream_t s);
void nrm_inf(int64_t n, const double* x, double* out, double* partials, hipStream_t s);
// out[i] = <Q_i, w>, Q_i = Q + i * ldq, i < m
void multi_dot(int64_t n, int m, const double* Q, int64_t ldq, const double* w, double* out,
               double* partials, hipStream_t s);
// w -= sum_i h[i] * Q_i   (h on the device)
void multi_axpy(int64_t n, int m, const double* Q, int64_t ldq, const double* h, double* w, hipStream_t s);
// x += sum_i y[i] * Q_i  (y on the device), scaled by sign
void combine(int64_t n, int m, const double* Q, int64_t ldq, const double* y, double sign, double* x,
             hipStream_t s);

// 64-bit content hash of n doubles (bit patterns), deterministic.
void hash64(int64_t n, const double* x, uint64_t* out, uint64_t* partials, hipStream_t s);

}  // namespace pnk
