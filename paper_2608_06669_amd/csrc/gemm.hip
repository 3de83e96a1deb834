// Matrix-core GEMM for gfx950 (CDNA4), FP64 / FP32 / BF16 compute.
//
// One workgroup = 4 wavefronts of 64 lanes computes a BM x BN tile of C.
// The waves form a WGM x WGN grid; each wave owns (BM/WGM) x (BN/WGN)
// outputs as a grid of 16 x 16 matrix-core tiles kept in registers for the
// whole K loop. A and B tiles of depth BK are staged through LDS: the next
// tile's global loads are issued before the current tile's MFMAs so their
// latency hides behind the matrix-core work. Operands are converted to the
// compute type as they are written to LDS, so FP64 tensors can feed the
// FP32 and BF16 products without a separate cast pass.
//
// Matrix-core operand layouts (64 lanes, lane l):
//   f64 / f32 16x16x4:  A[i][k] at i = l%16, k = l/16;  B[k][j] at j = l%16
//   bf16 16x16x32:      A[i][k..k+7] at i = l%16, k = 8*(l/16); B likewise
//   D f32 / bf16:       D[i][j] at j = l%16, i = 4*(l/16) + r, r = 0..3
//   D f64:              D[i][j] at j = l%16, i = l/16 + 4*r,   r = 0..3
//
// Workgroup order: tiles of one output column block (same B panel) are
// consecutive and are placed on the same XCD (hardware dispatches block ids
// round-robin over the 8 XCDs), so the B panel is fetched from HBM once and
// re-read by its neighbours from that XCD's L2.

#include "gemm.hpp"

#include <algorithm>

namespace pnk {
namespace {

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
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

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

struct MmaF64 {
  using L = double;   // LDS element
  using Acc = d4;
  static constexpr int KSTEP = 4;
  static constexpr bool KCONTIG_LDS = false;  // LDS laid out [k][m]
};
struct MmaF32 {
  using L = float;
  using Acc = f4;
  static constexpr int KSTEP = 4;
  static constexpr bool KCONTIG_LDS = false;
};
struct MmaBF16 {
  using L = uint16_t;
  using Acc = f4;
  static constexpr int KSTEP = 32;
  static constexpr bool KCONTIG_LDS = true;  // LDS laid out [m][k]
};

template <class Mma, int BM, int BN, int BK, int WGM>
struct Tile {
  static constexpr int WGN = 4 / WGM;
  static constexpr int WTM = BM / WGM;  // rows per wave
  static constexpr int WTN = BN / WGN;
  static constexpr int TMI = WTM / 16;
  static constexpr int TNI = WTN / 16;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be 16-aligned");
  static_assert(BK % Mma::KSTEP == 0, "BK must be a multiple of the MFMA depth");
  // LDS geometry: [BK][BM+PAD] or [BM][BK+PADK]
  static constexpr int PAD = 1;
  static constexpr int PADK = 8;
  static constexpr int A_LDS = Mma::KCONTIG_LDS ? BM * (BK + PADK) : BK * (BM + PAD);
  static constexpr int B_LDS = Mma::KCONTIG_LDS ? BN * (BK + PADK) : BK * (BN + PAD);
  static constexpr int EA = BM * BK / 256;  // A elements loaded per thread
  static constexpr int EB = BK * BN / 256;
  static_assert((BM * BK) % 256 == 0 && (BK * BN) % 256 == 0, "tile load split");
};

struct KArgs {
  int M, N, K, nb0;
  int splits, kchunk;  // split-K: blockIdx.z = zb * splits + split
  double* ws;          // partial sums [split][batch][M][N] when splits > 1
  int nbtot;
  int tiles_m, tiles_n;
  const void* A;
  int64_t a_m, a_k, a_b0, a_b1;
  const void* B;
  int64_t b_k, b_n, b_b0, b_b1;
  void* C;
  int64_t c_m, c_n, c_b0, c_b1;
  double alpha, beta;
};

template <class Mma, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM, bool A_KC, bool B_KC>
__global__ __launch_bounds__(256) void gemm_kernel(KArgs p) {
  using T = Tile<Mma, BM, BN, BK, WGM>;
  using L = typename Mma::L;
  using Acc = typename Mma::Acc;
  __shared__ __attribute__((aligned(16))) L As[T::A_LDS];
  __shared__ __attribute__((aligned(16))) L Bs[T::B_LDS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WGN;
  const int wn = wave % T::WGN;

  // XCD-aware tile order (see header comment)
  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int tm = bid % p.tiles_m;
  const int tn = bid / p.tiles_m;
  const int m0 = tm * BM;
  const int n0 = tn * BN;

  const int split = blockIdx.z % p.splits;
  const int zb = blockIdx.z / p.splits;
  const int b0 = blockIdx.y % p.nb0;
  const int b1 = blockIdx.y / p.nb0 + zb * (gridDim.y / p.nb0);
  const int kbeg = split * p.kchunk;
  const int kend = min(p.K, kbeg + p.kchunk);
  const TA* __restrict__ Ag = (const TA*)p.A + b0 * p.a_b0 + b1 * p.a_b1;
  const TB* __restrict__ Bg = (const TB*)p.B + b0 * p.b_b0 + b1 * p.b_b1;
  TC* __restrict__ Cg = (TC*)p.C + b0 * p.c_b0 + b1 * p.c_b1;

  Acc acc[T::TMI][T::TNI];
#pragma unroll
  for (int i = 0; i < T::TMI; ++i)
#pragma unroll
    for (int j = 0; j < T::TNI; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  TA ra[T::EA];
  TB rb[T::EB];

  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const int idx = tid + e * 256;
      const int m = A_KC ? idx / BK : idx % BM;
      const int k = A_KC ? idx % BK : idx / BM;
      const int gm = m0 + m, gk = k0 + k;
      ra[e] = (gm < p.M && gk < kend) ? Ag[gm * p.a_m + gk * p.a_k] : TA(0);
    }
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = tid + e * 256;
      const int n = B_KC ? idx / BK : idx % BN;
      const int k = B_KC ? idx % BK : idx / BN;
      const int gn = n0 + n, gk = k0 + k;
      rb[e] = (gn < p.N && gk < kend) ? Bg[gk * p.b_k + gn * p.b_n] : TB(0);
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const int idx = tid + e * 256;
      const int m = A_KC ? idx / BK : idx % BM;
      const int k = A_KC ? idx % BK : idx / BM;
      const L x = to_lds<TA, L>(ra[e]);
      if constexpr (Mma::KCONTIG_LDS) As[m * (BK + T::PADK) + k] = x;
      else As[k * (BM + T::PAD) + m] = x;
    }
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = tid + e * 256;
      const int n = B_KC ? idx / BK : idx % BN;
      const int k = B_KC ? idx % BK : idx / BN;
      const L x = to_lds<TB, L>(rb[e]);
      if constexpr (Mma::KCONTIG_LDS) Bs[n * (BK + T::PADK) + k] = x;
      else Bs[k * (BN + T::PAD) + n] = x;
    }
  };

  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    load_tiles(kbeg);
    store_tiles();
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load_tiles(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += Mma::KSTEP) {
      if constexpr (Mma::KCONTIG_LDS) {
        const int kk = ks + 8 * (lane >> 4);
        bf8 af[T::TMI], bfr[T::TNI];
#pragma unroll
        for (int i = 0; i < T::TMI; ++i) {
          const int m = wm * T::WTM + i * 16 + (lane & 15);
          u16x8 v = *reinterpret_cast<const u16x8*>(&As[m * (BK + T::PADK) + kk]);
          af[i] = __builtin_bit_cast(bf8, v);
        }
#pragma unroll
        for (int j = 0; j < T::TNI; ++j) {
          const int n = wn * T::WTN + j * 16 + (lane & 15);
          u16x8 v = *reinterpret_cast<const u16x8*>(&Bs[n * (BK + T::PADK) + kk]);
          bfr[j] = __builtin_bit_cast(bf8, v);
        }
#pragma unroll
        for (int i = 0; i < T::TMI; ++i)
#pragma unroll
          for (int j = 0; j < T::TNI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      } else {
        const int kk = ks + (lane >> 4);
        L af[T::TMI], bfr[T::TNI];
#pragma unroll
        for (int i = 0; i < T::TMI; ++i) af[i] = As[kk * (BM + T::PAD) + wm * T::WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < T::TNI; ++j) bfr[j] = Bs[kk * (BN + T::PAD) + wn * T::WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < T::TMI; ++i)
#pragma unroll
          for (int j = 0; j < T::TNI; ++j) {
            if constexpr (sizeof(L) == 8)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bfr[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    if (kt + 1 < nk) {
      __syncthreads();
      store_tiles();
      __syncthreads();
    }
  }

  // epilogue: C = alpha * acc + beta * C
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < T::TMI; ++i)
#pragma unroll
    for (int j = 0; j < T::TNI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (sizeof(typename Mma::L) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int gm = m0 + wm * T::WTM + i * 16 + row;
        const int gn = n0 + wn * T::WTN + j * 16 + (lane & 15);
        if (p.splits > 1) {
          if (gm < p.M && gn < p.N) {
            const int64_t b = (int64_t)b1 * p.nb0 + b0;
            p.ws[(((int64_t)split * p.nbtot + b) * p.M + gm) * p.N + gn] = (double)acc[i][j][r];
          }
        } else if (gm < p.M && gn < p.N) {
          TC* c = Cg + gm * p.c_m + gn * p.c_n;
          double v = alpha * (double)acc[i][j][r];
          if (beta != 0.0) v += beta * load_c<TC>(c);
          *c = from_acc<TC>(v);
        }
      }
}

// C[b][m][n] = alpha * sum_s ws[s][b][m][n] + beta * C[b][m][n] (fixed order)
template <typename TC>
__global__ __launch_bounds__(256) void splitk_reduce(KArgs p) {
  const int64_t MN = (int64_t)p.M * p.N;
  const int64_t total = MN * p.nbtot;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int s = 0; s < p.splits; ++s) acc += p.ws[(int64_t)s * total + e];
    const int64_t b = e / MN;
    const int m = (int)((e % MN) / p.N), n = (int)(e % p.N);
    const int b0 = (int)(b % p.nb0), b1 = (int)(b / p.nb0);
    TC* c = (TC*)p.C + b0 * p.c_b0 + b1 * p.c_b1 + m * p.c_m + n * p.c_n;
    double v = p.alpha * acc;
    if (p.beta != 0.0) v += p.beta * load_c<TC>(c);
    *c = from_acc<TC>(v);
  }
}

template <class Mma, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM>
void launch_cfg(const GemmDesc& d, const void* A, const void* B, void* C, hipStream_t s) {
  KArgs p;
  p.M = d.M; p.N = d.N; p.K = d.K; p.nb0 = d.nb0;
  p.tiles_m = (int)ceil_div(d.M, BM);
  p.tiles_n = (int)ceil_div(d.N, BN);
  p.A = A; p.a_m = d.a_m; p.a_k = d.a_k; p.a_b0 = d.a_b0; p.a_b1 = d.a_b1;
  p.B = B; p.b_k = d.b_k; p.b_n = d.b_n; p.b_b0 = d.b_b0; p.b_b1 = d.b_b1;
  p.C = C; p.c_m = d.c_m; p.c_n = d.c_n; p.c_b0 = d.c_b0; p.c_b1 = d.c_b1;
  p.alpha = d.alpha; p.beta = d.beta;
  const int64_t nb = (int64_t)d.nb0 * d.nb1;
  p.nbtot = (int)nb;
  // split-K when the output tiles cannot fill the GPU
  int splits = 1;
  const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n * nb;
  if (d.ws && tiles < 256 && d.K >= 4 * BK) {
    int64_t want = ceil_div(512, tiles);
    want = std::min<int64_t>(want, d.K / (2 * BK));
    want = std::min<int64_t>(want, d.ws_elems / std::max<int64_t>(1, nb * d.M * d.N));
    want = std::min<int64_t>(want, 256);
    if (want >= 2) splits = (int)want;
  }
  p.splits = splits;
  p.kchunk = splits > 1 ? (int)(ceil_div(ceil_div(d.K, splits), BK) * BK) : d.K;
  if (splits > 1) splits = (int)ceil_div(d.K, p.kchunk);  // no empty chunk
  p.splits = splits;
  p.ws = d.ws;
  // gridDim.y * gridDim.z covers the batch; y is a multiple of nb0
  int64_t gy = d.nb0, gz = d.nb1;
  while (gy * 2 <= 65535 && gz % 2 == 0) { gy *= 2; gz /= 2; }
  PNK_REQUIRE(gy <= 65535 && gz <= 65535, "gemm: batch too large");
  (void)nb;
  PNK_REQUIRE(gz * splits <= 65535, "gemm: split-K grid too large");
  dim3 grid((unsigned)(p.tiles_m * p.tiles_n), (unsigned)gy, (unsigned)(gz * splits));
  const bool akc = d.a_k == 1 && d.a_m != 1;
  const bool bkc = d.b_k == 1 && d.b_n != 1;
  if (akc && bkc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, true, true><<<grid, 256, 0, s>>>(p);
  else if (akc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, true, false><<<grid, 256, 0, s>>>(p);
  else if (bkc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, false, true><<<grid, 256, 0, s>>>(p);
  else gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, false, false><<<grid, 256, 0, s>>>(p);
  PNK_CHECK_LAUNCH();
  if (splits > 1) {
    const int64_t total = nb * d.M * d.N;
    splitk_reduce<TC><<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 4096), 256, 0, s>>>(p);
    PNK_CHECK_LAUNCH();
  }
}

// Tile choice: large tiles when the product has enough work to fill the
// 256 CUs several times over, small tiles otherwise.
template <class Mma, typename TA, typename TB, typename TC, int BK>
void launch_sized(const GemmDesc& d, const void* A, const void* B, void* C, hipStream_t s) {
  const int64_t nb = (int64_t)d.nb0 * d.nb1;
  const int64_t big = ceil_div(d.M, 128) * ceil_div(d.N, 128) * nb;
  if (d.M >= 96 && d.N >= 96 && big >= 512)
    launch_cfg<Mma, TA, TB, TC, 128, 128, BK, 2>(d, A, B, C, s);
  else
    launch_cfg<Mma, TA, TB, TC, 64, 64, BK, 2>(d, A, B, C, s);
}

}  // namespace

void gemm(const GemmDesc& d, const void* A, Prec ap, const void* B, Prec bp, void* C, Prec cp, Prec compute,
          hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.nb0 <= 0 || d.nb1 <= 0) return;
  PNK_REQUIRE(cp == Prec::F64 || cp == Prec::F32, "gemm: C must be f64 or f32");
  if (d.K <= 0) {
    // C = beta * C: express as a K=1 product with alpha = 0 would read A/B;
    // callers never request this shape.
    PNK_REQUIRE(false, "gemm: K must be positive");
  }
#define PNK_GEMM_CASE(MMA, TA, TB, TC, BK) \
  return launch_sized<MMA, TA, TB, TC, BK>(d, A, B, C, s)
  if (compute == Prec::F64) {
    PNK_REQUIRE(ap == Prec::F64 && bp == Prec::F64, "gemm: f64 compute needs f64 operands");
    if (cp == Prec::F64) PNK_GEMM_CASE(MmaF64, double, double, double, 16);
    PNK_GEMM_CASE(MmaF64, double, double, float, 16);
  }
  if (compute == Prec::F32) {
    PNK_REQUIRE(ap != Prec::BF16 && bp != Prec::BF16, "gemm: f32 compute needs f32/f64 operands");
    if (cp == Prec::F64) {
      if (ap == Prec::F64 && bp == Prec::F64) PNK_GEMM_CASE(MmaF32, double, double, double, 16);
      if (ap == Prec::F64 && bp == Prec::F32) PNK_GEMM_CASE(MmaF32, double, float, double, 16);
      if (ap == Prec::F32 && bp == Prec::F64) PNK_GEMM_CASE(MmaF32, float, double, double, 16);
      PNK_GEMM_CASE(MmaF32, float, float, double, 16);
    }
    if (ap == Prec::F64 && bp == Prec::F64) PNK_GEMM_CASE(MmaF32, double, double, float, 16);
    PNK_GEMM_CASE(MmaF32, float, float, float, 16);
  }
  // BF16 compute, FP32 accumulation
  if (cp == Prec::F64) {
    if (ap == Prec::F64 && bp == Prec::F64) PNK_GEMM_CASE(MmaBF16, double, double, double, 32);
    if (ap == Prec::F64 && bp == Prec::BF16) PNK_GEMM_CASE(MmaBF16, double, uint16_t, double, 32);
    if (ap == Prec::BF16 && bp == Prec::F64) PNK_GEMM_CASE(MmaBF16, uint16_t, double, double, 32);
    if (ap == Prec::BF16 && bp == Prec::BF16) PNK_GEMM_CASE(MmaBF16, uint16_t, uint16_t, double, 32);
  }
  PNK_REQUIRE(false, "gemm: unsupported precision combination");
#undef PNK_GEMM_CASE
}

}  // namespace pnk
