// Matrix-core building blocks shared by the GEMM and the fused operator
// kernels: instruction shapes, operand conversion into LDS and the panel
// loader that stages a ROWS x BK block of an operand through registers.
//
// Matrix-core instructions and operand layouts (64 lanes, lane l):
//   f64  4x4x4 (4 blocks), used as one 4 x 16 x 4 product:
//        A[i][k] at i = l%4, k = l/16 (the same for the 4 blocks);
//        B[k][j] at j = l%16, k = l/16;  D[i][j] at i = l/16, j = l%16.
//   f32  16x16x4:  A[i][k] at i = l%16, k = l/16;  B[k][j] at j = l%16;
//        D[i][j] at j = l%16, i = 4*(l/16) + r, r = 0..3
//   bf16 16x16x32: A[i][k..k+7] at i = l%16, k = 8*(l/16); B likewise;
//        D as f32
#pragma once

#include "common.hpp"

namespace pnk {
namespace tiles {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Convert one stored element to the LDS (compute) representation.
template <typename S, typename L> __device__ inline L to_lds(S x);
template <> __device__ inline double to_lds<double, double>(double x) { return x; }
template <> __device__ inline float to_lds<double, float>(double x) { return (float)x; }
template <> __device__ inline float to_lds<float, float>(float x) { return x; }
template <> __device__ inline uint16_t to_lds<double, uint16_t>(double x) { return f32_to_bf16((float)x); }
template <> __device__ inline uint16_t to_lds<float, uint16_t>(float x) { return f32_to_bf16(x); }
template <> __device__ inline uint16_t to_lds<uint16_t, uint16_t>(uint16_t x) { return x; }

template <typename C> __device__ inline C from_acc(double x);
template <> __device__ inline double from_acc<double>(double x) { return x; }
template <> __device__ inline float from_acc<float>(double x) { return (float)x; }
template <typename C> __device__ inline double load_c(const C* p) { return (double)*p; }

// TM x TN: output tile of one instruction; NACC: accumulator values per lane
struct MmaF64 {
  using L = double;   // LDS element
  using Acc = double;
  static constexpr int KSTEP = 4, TM = 4, TN = 16, NACC = 1;
  static constexpr bool KCONTIG_LDS = false;  // LDS laid out [k][m]
};
struct MmaF32 {
  using L = float;
  using Acc = f4;
  static constexpr int KSTEP = 4, TM = 16, TN = 16, NACC = 4;
  static constexpr bool KCONTIG_LDS = false;
};
struct MmaBF16 {
  using L = uint16_t;
  using Acc = f4;
  static constexpr int KSTEP = 32, TM = 16, TN = 16, NACC = 4;
  static constexpr bool KCONTIG_LDS = true;  // LDS laid out [m][k]
};
template <class Acc> __device__ inline double acc_get(const Acc& a, int r) { return (double)a[r]; }
template <> __device__ inline double acc_get<double>(const double& a, int) { return a; }

constexpr int kPad = 1;   // [k][rows + pad], default pad
constexpr int kPadK = 8;  // [rows][k + kPadK]

template <class Mma, int ROWS, int BK, int PAD = kPad>
constexpr int lds_elems() {
  return Mma::KCONTIG_LDS ? ROWS * (BK + kPadK) : BK * (ROWS + PAD);
}

// Loads a ROWS x BK panel (ROWS = BM for A, BN for B) into registers and
// writes it to one LDS buffer. KC: the operand is contiguous along k. PAD:
// row padding of the [k][rows + PAD] layout.
template <class Mma, typename T, int ROWS, int BK, bool KC, int PAD = kPad>
struct Panel {
  using L = typename Mma::L;
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int NVEC = ROWS * BK / V;
  static constexpr int PER = (NVEC + 255) / 256;
  static_assert(ROWS % V == 0 && BK % V == 0, "panel must split into vectors");
  T r[PER * V];

  __device__ inline void coords(int q, int* row, int* kk) const {
    if (KC) { *row = q / (BK / V); *kk = (q % (BK / V)) * V; }
    else { *kk = q / (ROWS / V); *row = (q % (ROWS / V)) * V; }
  }

  __device__ inline void load(const T* __restrict__ g, int64_t s_row, int64_t s_k, int row0, int rows, int k0,
                              int kend, bool vec_ok, int tid) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * 256;
      if (q >= NVEC) break;
      int row, kk;
      coords(q, &row, &kk);
      const int gr = row0 + row, gk = k0 + kk;
      bool full;
      if (KC) full = vec_ok && gr < rows && gk + V <= kend;
      else full = vec_ok && gr + V <= rows && gk < kend;
      if (full) {
        const T* p = g + (int64_t)gr * s_row + (int64_t)gk * s_k;
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        *reinterpret_cast<uint4*>(&r[e * V]) = v;
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int rr = KC ? gr : gr + u;
          const int kx = KC ? gk + u : gk;
          r[e * V + u] = (rr < rows && kx < kend) ? g[(int64_t)rr * s_row + (int64_t)kx * s_k] : T(0);
        }
      }
    }
  }

  // As load, of (g1 - a g2) sc elementwise (g1, g2 with the same layout).
  __device__ inline void load_diff(const T* __restrict__ g1, const T* __restrict__ g2, T a, T sc, int64_t s_row,
                                   int64_t s_k, int row0, int rows, int k0, int kend, bool vec_ok, int tid) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * 256;
      if (q >= NVEC) break;
      int row, kk;
      coords(q, &row, &kk);
      const int gr = row0 + row, gk = k0 + kk;
      bool full;
      if (KC) full = vec_ok && gr < rows && gk + V <= kend;
      else full = vec_ok && gr + V <= rows && gk < kend;
      if (full) {
        const int64_t off = (int64_t)gr * s_row + (int64_t)gk * s_k;
        T t1[V], t2[V];
        const uint4 u1 = *reinterpret_cast<const uint4*>(g1 + off);
        const uint4 u2 = *reinterpret_cast<const uint4*>(g2 + off);
        __builtin_memcpy(t1, &u1, sizeof(u1));
        __builtin_memcpy(t2, &u2, sizeof(u2));
#pragma unroll
        for (int u = 0; u < V; ++u) r[e * V + u] = (t1[u] - a * t2[u]) * sc;
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int rr = KC ? gr : gr + u;
          const int kx = KC ? gk + u : gk;
          const int64_t off = (int64_t)rr * s_row + (int64_t)kx * s_k;
          r[e * V + u] = (rr < rows && kx < kend) ? (g1[off] - a * g2[off]) * sc : T(0);
        }
      }
    }
  }

  __device__ inline void store(L* __restrict__ lds, int tid) const {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * 256;
      if (q >= NVEC) break;
      int row, kk;
      coords(q, &row, &kk);
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int rr = KC ? row : row + u;
        const int kx = KC ? kk + u : kk;
        const L x = to_lds<T, L>(r[e * V + u]);
        if constexpr (Mma::KCONTIG_LDS) lds[rr * (BK + kPadK) + kx] = x;
        else lds[kx * (ROWS + PAD) + rr] = x;
      }
    }
  }
};

}  // namespace tiles
}  // namespace pnk
