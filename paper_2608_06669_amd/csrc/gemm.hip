// Matrix-core GEMM for gfx950 (CDNA4), FP64 / FP32 / BF16 compute.
//
// One workgroup = 4 wavefronts of 64 lanes computes a BM x BN tile of C.
// The waves form a WGM x WGN grid; each wave owns (BM/WGM) x (BN/WGN)
// outputs as a grid of matrix-core instruction tiles held in registers for
// the whole K loop. A and B panels of depth BK are staged through two LDS
// buffers: while the matrix cores work on one buffer, the next panel's
// global loads are in flight and are then written to the other buffer, so
// each K step costs one barrier. Global loads are 16-byte vectors along the
// operand's contiguous index whenever strides and alignment allow. Operands
// are converted to the compute type as they are written to LDS, so FP64
// tensors feed the FP32 and BF16 products without a separate cast pass.
//
// Matrix-core instructions and operand layouts (64 lanes, lane l):
//   f64  4x4x4 (4 blocks), used as one 4 x 16 x 4 product:
//        A[i][k] at i = l%4, k = l/16 (the same for the 4 blocks);
//        B[k][j] at j = l%16, k = l/16;  D[i][j] at i = l/16, j = l%16.
//        On gfx950 this instruction runs at the full FP64 matrix rate,
//        while the 16x16x4 f64 instruction reaches about two thirds of it.
//   f32  16x16x4:  A[i][k] at i = l%16, k = l/16;  B[k][j] at j = l%16;
//        D[i][j] at j = l%16, i = 4*(l/16) + r, r = 0..3
//   bf16 16x16x32: A[i][k..k+7] at i = l%16, k = 8*(l/16); B likewise;
//        D as f32
//
// Workgroup order: each XCD takes a contiguous range of tiles (hardware
// dispatches block ids round-robin over the 8 XCDs), ordered in groups of 8
// row tiles with the row tile fastest, so the workgroups resident on one
// XCD share their A and B panels in that XCD's L2 (85 % L2 hits on a BF16
// 3600^3 product against 72 % in plain order).
//
// Products with too few output tiles to fill the GPU split the contraction
// (split-K); partial sums are added afterwards in a fixed order, so results
// never depend on timing.

#include "gemm.hpp"
#include "mfma_tiles.hpp"

#include <algorithm>
#include <type_traits>

namespace pnk {
namespace {

using namespace tiles;

struct KArgs {
  int M, N, K, nb0;
  int splits, kchunk;  // split-K: blockIdx.z = zb * splits + split
  double* ws;          // partial sums [split][batch][M][N] when splits > 1
  int nbtot;
  int tiles_m, tiles_n;
  int a_vec, b_vec;    // 16-byte vector loads allowed
  const void* A;
  int64_t a_m, a_k, a_b0, a_b1;
  const void* B;
  int64_t b_k, b_n, b_b0, b_b1;
  const void* A2;  // optional second product A2 B2 (same strides as A, B)
  const void* B2;
  void* C;
  int64_t c_m, c_n, c_b0, c_b1;
  double alpha, beta;
};

// LDS row padding of an FP64 panel stored [k][rows + pad]. The 4x4x4 f64
// reads take, per k, 4 consecutive values of A or 16 of B; half a wave (two
// k rows) is served per LDS cycle, so the two rows must fall on disjoint
// banks (64 banks of 4 bytes): a row stride of 9 modulo 32 doubles offsets
// them by 18 banks, 16 modulo 32 by 32 banks (the 16-value B reads need
// that). A panel loaded along k (KC) is written one value per lane at a
// stride of two rows, which a 16-modulo-32 stride turns into an 8-way
// conflict, so those panels take 9. Other compute types keep kPad.
template <class Mma, int ROWS, bool KC, bool IS_B>
constexpr int lds_pad() {
  if constexpr (sizeof(typename Mma::L) != 8) return kPad;
  const int want = (IS_B && !KC) ? 16 : 9;
  return ((want - ROWS) % 32 + 32) % 32;
}

template <class Mma, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM, bool A_KC, bool B_KC>
__global__ __launch_bounds__(256) void gemm_kernel(KArgs p) {
  using L = typename Mma::L;
  using Acc = typename Mma::Acc;
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TMI = WTM / Mma::TM, TNI = WTN / Mma::TN;
  static_assert(WTM % Mma::TM == 0 && WTN % Mma::TN == 0, "wave tile must split into instruction tiles");
  static_assert(BK % Mma::KSTEP == 0, "BK must be a multiple of the MFMA depth");
  constexpr int PA = lds_pad<Mma, BM, A_KC, false>();
  constexpr int PB = lds_pad<Mma, BN, B_KC, true>();
  constexpr int ALDS = lds_elems<Mma, BM, BK, PA>();
  constexpr int BLDS = lds_elems<Mma, BN, BK, PB>();
  __shared__ __attribute__((aligned(16))) L As[2][ALDS];
  __shared__ __attribute__((aligned(16))) L Bs[2][BLDS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN;
  const int wn = wave % WGN;

  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x;
  {
    // XCD x receives block ids x, x + 8, ...: give it the contiguous range
    // of q + (x < r) tiles that starts at x q + min(x, r)
    const int q = ntiles >> 3, r = ntiles & 7, x = bid & 7;
    bid = x * q + min(x, r) + (bid >> 3);
  }
  // tiles in groups of (up to) 8 row tiles: within a group the row tile
  // runs fastest, so the workgroups resident on one XCD share both their A
  // and their B panels in L2 (with the row tile fastest over all rows, each
  // XCD streamed every A panel once per column block)
  constexpr int kGroupM = 8;
  const int gsize = kGroupM * p.tiles_n;
  const int grp = bid / gsize;
  const int first_m = grp * kGroupM;
  const int gm = min(p.tiles_m - first_m, kGroupM);
  const int rem = bid - grp * gsize;
  const int tm = first_m + rem % gm;
  const int tn = rem / gm;
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
  const bool dual = p.A2 != nullptr;
  const TA* __restrict__ Ag2 = dual ? (const TA*)p.A2 + b0 * p.a_b0 + b1 * p.a_b1 : Ag;
  const TB* __restrict__ Bg2 = dual ? (const TB*)p.B2 + b0 * p.b_b0 + b1 * p.b_b1 : Bg;
  TC* __restrict__ Cg = (TC*)p.C + b0 * p.c_b0 + b1 * p.c_b1;

  Acc acc[TMI][TNI];
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j) acc[i][j] = Acc{};

  Panel<Mma, TA, BM, BK, A_KC, PA> pa;
  Panel<Mma, TB, BN, BK, B_KC, PB> pb;
  const bool avec = p.a_vec != 0, bvec = p.b_vec != 0;
  const int64_t a_row = p.a_m, a_kk = p.a_k, b_row = p.b_n, b_kk = p.b_k;

  // panels 0 .. nk1-1 read A, B; with a second product, panels nk1 ..
  // 2 nk1-1 read A2, B2 over the same k range into the same accumulators
  const int nk1 = (kend - kbeg + BK - 1) / BK;
  const int nk = dual ? 2 * nk1 : nk1;
  auto load = [&](int t) {
    const bool second = t >= nk1;
    const int k0 = kbeg + (second ? t - nk1 : t) * BK;
    pa.load(second ? Ag2 : Ag, a_row, a_kk, m0, p.M, k0, kend, avec, tid);
    pb.load(second ? Bg2 : Bg, b_row, b_kk, n0, p.N, k0, kend, bvec, tid);
  };
  if (nk > 0) {
    load(0);
    pa.store(As[0], tid);
    pb.store(Bs[0], tid);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    const L* Ac = As[cur];
    const L* Bc = Bs[cur];
#pragma unroll
    for (int ks = 0; ks < BK; ks += Mma::KSTEP) {
      if constexpr (Mma::KCONTIG_LDS) {
        const int kk = ks + 8 * (lane >> 4);
        bf8 af[TMI], bfr[TNI];
#pragma unroll
        for (int i = 0; i < TMI; ++i) {
          const int m = wm * WTM + i * 16 + (lane & 15);
          af[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Ac[m * (BK + kPadK) + kk]));
        }
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          const int n = wn * WTN + j * 16 + (lane & 15);
          bfr[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Bc[n * (BK + kPadK) + kk]));
        }
#pragma unroll
        for (int i = 0; i < TMI; ++i)
#pragma unroll
          for (int j = 0; j < TNI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      } else if constexpr (sizeof(L) == 8) {
        const int kk = ks + (lane >> 4);
        double af[TMI], bfr[TNI];
#pragma unroll
        for (int i = 0; i < TMI; ++i) af[i] = Ac[kk * (BM + PA) + wm * WTM + i * 4 + (lane & 3)];
#pragma unroll
        for (int j = 0; j < TNI; ++j) bfr[j] = Bc[kk * (BN + PB) + wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TMI; ++i)
#pragma unroll
          for (int j = 0; j < TNI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[i], bfr[j], acc[i][j], 0, 0, 0);
      } else {
        const int kk = ks + (lane >> 4);
        L af[TMI], bfr[TNI];
#pragma unroll
        for (int i = 0; i < TMI; ++i) af[i] = Ac[kk * (BM + PA) + wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TNI; ++j) bfr[j] = Bc[kk * (BN + PB) + wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TMI; ++i)
#pragma unroll
          for (int j = 0; j < TNI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) {
      // the other buffer was last read before the previous barrier
      pa.store(As[cur ^ 1], tid);
      pb.store(Bs[cur ^ 1], tid);
    }
    __syncthreads();
  }

  // epilogue: C = alpha * acc + beta * C, or raw partial sums for split-K
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int r = 0; r < Mma::NACC; ++r) {
        const int row = (Mma::NACC == 1) ? (lane >> 4) : 4 * (lane >> 4) + r;
        const int gm = m0 + wm * WTM + i * Mma::TM + row;
        const int gn = n0 + wn * WTN + j * Mma::TN + (lane & 15);
        if (gm >= p.M || gn >= p.N) continue;
        if (p.splits > 1) {
          const int64_t b = (int64_t)b1 * p.nb0 + b0;
          p.ws[(((int64_t)split * p.nbtot + b) * p.M + gm) * p.N + gn] = acc_get(acc[i][j], r);
        } else {
          TC* c = Cg + gm * p.c_m + gn * p.c_n;
          double v = alpha * acc_get(acc[i][j], r);
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
  // one row-major output: its address is the element index
  const bool flat = p.nbtot == 1 && p.c_n == 1 && p.c_m == p.N;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    // four chunks' loads in flight before they are added, in chunk order
    int s = 0;
    for (; s + 4 <= p.splits; s += 4) {
      const double x0 = p.ws[(int64_t)s * total + e], x1 = p.ws[(int64_t)(s + 1) * total + e];
      const double x2 = p.ws[(int64_t)(s + 2) * total + e], x3 = p.ws[(int64_t)(s + 3) * total + e];
      acc += x0;
      acc += x1;
      acc += x2;
      acc += x3;
    }
    for (; s < p.splits; ++s) acc += p.ws[(int64_t)s * total + e];
    TC* c;
    if (flat) {
      c = (TC*)p.C + e;
    } else {
      const int64_t b = e / MN;
      const int m = (int)((e % MN) / p.N), n = (int)(e % p.N);
      const int b0 = (int)(b % p.nb0), b1 = (int)(b / p.nb0);
      c = (TC*)p.C + b0 * p.c_b0 + b1 * p.c_b1 + m * p.c_m + n * p.c_n;
    }
    double v = p.alpha * acc;
    if (p.beta != 0.0) v += p.beta * load_c<TC>(c);
    *c = from_acc<TC>(v);
  }
}

// The same sum for many splits and few outputs: 16 lanes per output, each
// adding every 16th split in increasing order, then the 16 lane sums in
// order (deterministic, and no lane walks all splits).
template <typename TC>
__global__ __launch_bounds__(256) void splitk_reduce_wide(KArgs p) {
  __shared__ double sm[16][17];
  const int64_t MN = (int64_t)p.M * p.N;
  const int64_t total = MN * p.nbtot;
  const int eo = threadIdx.x & 15, sg = threadIdx.x >> 4;
  for (int64_t e0 = blockIdx.x * (int64_t)16; e0 < total; e0 += (int64_t)gridDim.x * 16) {
    const int64_t e = e0 + eo;
    double acc = 0.0;
    if (e < total)
      for (int s = sg; s < p.splits; s += 16) acc += p.ws[(int64_t)s * total + e];
    sm[sg][eo] = acc;
    __syncthreads();
    if (sg == 0 && e < total) {
      double sum = 0.0;
      for (int g = 0; g < 16; ++g) sum += sm[g][eo];
      const int64_t b = e / MN;
      const int m = (int)((e % MN) / p.N), n = (int)(e % p.N);
      const int b0 = (int)(b % p.nb0), b1 = (int)(b / p.nb0);
      TC* c = (TC*)p.C + b0 * p.c_b0 + b1 * p.c_b1 + m * p.c_m + n * p.c_n;
      double v = p.alpha * sum;
      if (p.beta != 0.0) v += p.beta * load_c<TC>(c);
      *c = from_acc<TC>(v);
    }
    __syncthreads();
  }
}

// BF16 product of two k-contiguous BF16 operands (rows 16-byte aligned, the
// contraction a multiple of 64, zero-padded), BM x 128 tiles, 64-deep
// panels in a ring of three LDS stages filled straight from global memory
// (16 bytes per lane, no register staging), so two panels' loads are in
// flight while the matrix cores work on the third. A stage holds A then B,
// [row][64] each; the eight 16-byte chunks of a row are stored at slot
// chunk ^ ((row / 2) % 8), which spreads the fragment reads of 16
// consecutive rows over all 64 banks (each wave's load writes 1 KB
// contiguously: its lanes fetch the chunks in slot order). Each wave forms
// a 64 x 64 block of the tile: BM = 128 with 4 waves (96 KB of LDS), or BM
// = 256 with 8 waves (144 KB: one workgroup per CU, two waves per SIMD; on
// MI355X 1.1-1.4x faster than 128 x 128 on the 3600 x 3600 x 7232, 210 x
// 16290 x 16290 and 400 x 3600 x 32400 products and 1.4x at 8192^3). Same
// tile order, split-K and epilogue as gemm_kernel.
template <int N>
__device__ inline void wait_vm_lgkm0() {  // vmcnt(N), lgkmcnt(0)
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}

template <int BM, int NW>
__global__ __launch_bounds__(64 * NW) void gemm_bf16_pipe(KArgs p) {
  constexpr int BN = 128, BK = 64, STAGES = 3, NT = 64 * NW;
  static_assert(BM == 64 * (NW / 2), "one 64 x 64 block per wave, two waves across the tile");
  constexpr int SE = (BM + BN) * BK;                             // elements per stage
  constexpr int CA = BM * BK / 8 / NT, CB = BN * BK / 8 / NT;  // 16-byte chunks per thread and stage
  __shared__ __attribute__((aligned(1024))) uint16_t st0[SE], st1[SE], st2[SE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x;
  {
    const int q = ntiles >> 3, r = ntiles & 7, x = bid & 7;
    bid = x * q + min(x, r) + (bid >> 3);
  }
  constexpr int kGroupM = 8;
  const int gsize = kGroupM * p.tiles_n;
  const int grp = bid / gsize;
  const int first_m = grp * kGroupM;
  const int gm = min(p.tiles_m - first_m, kGroupM);
  const int rem = bid - grp * gsize;
  const int m0 = (first_m + rem % gm) * BM;
  const int n0 = (rem / gm) * BN;

  const int split = blockIdx.z % p.splits;
  const int zb = blockIdx.z / p.splits;
  const int b0 = blockIdx.y % p.nb0;
  const int b1 = blockIdx.y / p.nb0 + zb * (gridDim.y / p.nb0);
  const int kbeg = split * p.kchunk;
  const int nk = (min(p.K, kbeg + p.kchunk) - kbeg) / BK;  // >= 1
  const uint16_t* __restrict__ Ag = (const uint16_t*)p.A + b0 * p.a_b0 + b1 * p.a_b1 + kbeg;
  const uint16_t* __restrict__ Bg = (const uint16_t*)p.B + b0 * p.b_b0 + b1 * p.b_b1 + kbeg;
  double* __restrict__ Cg = (double*)p.C + b0 * p.c_b0 + b1 * p.c_b1;

  // this thread's chunks c = j NT + tid (row c / 8, slot c % 8) of A (j <
  // CA) and of B (j < CB) (rows past the matrix read its last row; those
  // outputs are not written)
  const uint16_t* ga[CA];
  const uint16_t* gb[CB];
#pragma unroll
  for (int j = 0; j < CA; ++j) {
    const int c = j * NT + tid, r = c >> 3, slot = c & 7, g = slot ^ ((r >> 1) & 7);
    ga[j] = Ag + (int64_t)min(m0 + r, p.M - 1) * p.a_m + 8 * g;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int c = j * NT + tid, r = c >> 3, slot = c & 7, g = slot ^ ((r >> 1) & 7);
    gb[j] = Bg + (int64_t)min(n0 + r, p.N - 1) * p.b_n + 8 * g;
  }
  // panel t into stage st (past the last panel: the last one again, never
  // read). (The global address goes in as void*: converted implicitly, the
  // host pass drops the template's launch stub.)
  auto issue = [&](uint16_t* st, int t) {
    const int k0 = min(t, nk - 1) * BK;
#pragma unroll
    for (int j = 0; j < CA; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(ga[j] + k0),
                                       (__attribute__((address_space(3))) void*)(st + (j * NT + wave * 64) * 8), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < CB; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(gb[j] + k0),
                                       (__attribute__((address_space(3))) void*)(st + BM * BK + (j * NT + wave * 64) * 8),
                                       16, 0, 0);
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](const uint16_t* st) {
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      const int q = 4 * ks + (lane >> 4);  // this lane's 8-element chunk of the 32-deep step
      bf8 af[4], bfr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 64 + i * 16 + (lane & 15);
        af[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(st + row * BK + 8 * (q ^ ((row >> 1) & 7))));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wn * 64 + j * 16 + (lane & 15);
        bfr[j] = __builtin_bit_cast(
            bf8, *reinterpret_cast<const u16x8*>(st + BM * BK + row * BK + 8 * (q ^ ((row >> 1) & 7))));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
  };
  issue(st0, 0);
  issue(st1, 1);
  // step t: wait for panel t (CA + CB loads per panel per thread; the next
  // panel's may still be in flight) and for this wave's earlier LDS reads,
  // then a barrier (every wave's share of panel t has landed and every wave
  // is done with the stage about to be refilled), refill that stage with
  // panel t + 2, and compute panel t. (A plain barrier: the workgroup fence
  // of __syncthreads would wait for all loads in flight.)
  auto step = [&](int t, const uint16_t* cur, uint16_t* nxt) {
    wait_vm_lgkm0<(CA + CB) * (STAGES - 2)>();
    __builtin_amdgcn_s_barrier();
    issue(nxt, t + STAGES - 1);
    compute(cur);
  };
  // panel t sits in stage t % 3. Whole rounds of three in the loop, the
  // rest after it: with steps under a condition inside the loop the compiler
  // no longer tells the stages apart and waits for every load in flight
  // before each LDS read
  int t = 0;
  for (; t + 3 <= nk; t += 3) {
    step(t, st0, st2);
    step(t + 1, st1, st0);
    step(t + 2, st2, st1);
  }
  if (t < nk) step(t, st0, st2);
  if (t + 1 < nk) step(t + 1, st1, st0);
  wait_vm_lgkm0<0>();  // no load still writing LDS when the workgroup ends

  // epilogue (three uniform cases, each straight-line so the compiler can
  // count its memory operations): split-K partial sums; C = alpha acc; C =
  // alpha acc + beta C with the 16 reads of C of a row of tiles issued
  // together before its writes
  const double alpha = p.alpha, beta = p.beta;
  auto row_of = [&](int i, int r) { return m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r; };
  auto col_of = [&](int j) { return n0 + wn * 64 + j * 16 + (lane & 15); };
  if (p.splits > 1) {
    double* __restrict__ W = p.ws + ((int64_t)split * p.nbtot + (int64_t)b1 * p.nb0 + b0) * p.M * p.N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row_of(i, r) < p.M && col_of(j) < p.N) W[(int64_t)row_of(i, r) * p.N + col_of(j)] = (double)acc[i][j][r];
  } else if (beta == 0.0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row_of(i, r) < p.M && col_of(j) < p.N)
            Cg[row_of(i, r) * p.c_m + col_of(j) * p.c_n] = alpha * (double)acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double cv[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          cv[j][r] = Cg[min(row_of(i, r), p.M - 1) * p.c_m + min(col_of(j), p.N - 1) * p.c_n];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row_of(i, r) < p.M && col_of(j) < p.N)
            Cg[row_of(i, r) * p.c_m + col_of(j) * p.c_n] = alpha * (double)acc[i][j][r] + beta * cv[j][r];
    }
  }
}

// FP64 product, A k-contiguous, B k-contiguous (B_KC) or n-contiguous, the
// contraction a multiple of 16: 64 x 64 tiles, 16-deep panels loaded
// straight into LDS (16 bytes = two doubles per lane) in a ring of three
// stages, as in gemm_bf16_pipe. A k-contiguous operand is stored [row][16]
// with the eight 16-byte chunks of a row at slot chunk ^ (row % 8); B
// n-contiguous is stored [k][64] with its 32 chunks at slot chunk ^ (8 (k %
// 4)): the 4 x 4 x 4 operand reads (4 rows x 4 k of A, 16 columns x 4 k of
// B per instruction) then fall on distinct banks. A second product (A2,
// B2) continues the same k loop into the same accumulators.
template <bool B_KC>
__global__ __launch_bounds__(256, 2) void gemm_f64_pipe(KArgs p) {
  constexpr int BM = 64, BN = 64, BK = 16, STAGES = 3, AE = BM * BK, SE = AE + BN * BK;
  __shared__ __attribute__((aligned(1024))) double st0[SE], st1[SE], st2[SE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int ntiles = p.tiles_m * p.tiles_n;
  int bid = blockIdx.x;
  {
    const int q = ntiles >> 3, r = ntiles & 7, x = bid & 7;
    bid = x * q + min(x, r) + (bid >> 3);
  }
  constexpr int kGroupM = 8;
  const int gsize = kGroupM * p.tiles_n;
  const int grp = bid / gsize;
  const int first_m = grp * kGroupM;
  const int gm = min(p.tiles_m - first_m, kGroupM);
  const int rem = bid - grp * gsize;
  const int m0 = (first_m + rem % gm) * BM;
  const int n0 = (rem / gm) * BN;

  const int split = blockIdx.z % p.splits;
  const int zb = blockIdx.z / p.splits;
  const int b0 = blockIdx.y % p.nb0;
  const int b1 = blockIdx.y / p.nb0 + zb * (gridDim.y / p.nb0);
  const int kbeg = split * p.kchunk;
  const int nk1 = (min(p.K, kbeg + p.kchunk) - kbeg) / BK;  // >= 1
  const bool dual = p.A2 != nullptr;
  const int nk = dual ? 2 * nk1 : nk1;
  const int64_t lda = p.a_m, ldb = B_KC ? p.b_n : p.b_k;
  const int64_t aoff = b0 * p.a_b0 + b1 * p.a_b1 + kbeg;
  const int64_t boff = b0 * p.b_b0 + b1 * p.b_b1 + (B_KC ? kbeg : (int64_t)kbeg * ldb);
  double* __restrict__ Cg = (double*)p.C + b0 * p.c_b0 + b1 * p.c_b1;

  // this thread's chunks c = j 256 + tid, j = 0, 1, of A and of B (offsets
  // within an operand; rows and columns past the matrix read its last ones,
  // whose outputs are not written)
  int64_t oa[2], ob[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int c = j * 256 + tid;
    {
      const int r = c >> 3, g = (c & 7) ^ (r & 7);
      oa[j] = (int64_t)min(m0 + r, p.M - 1) * lda + 2 * g;
    }
    if constexpr (B_KC) {
      const int r = c >> 3, g = (c & 7) ^ (r & 7);
      ob[j] = (int64_t)min(n0 + r, p.N - 1) * ldb + 2 * g;
    } else {
      const int k = c >> 5, g = (c & 31) ^ (8 * (k & 3));
      ob[j] = (int64_t)k * ldb + min(n0 + 2 * g, p.N - 2);
    }
  }
  const double* A1 = (const double*)p.A + aoff;
  const double* B1 = (const double*)p.B + boff;
  const double* A2 = dual ? (const double*)p.A2 + aoff : A1;
  const double* B2 = dual ? (const double*)p.B2 + boff : B1;
  // panel t into stage st (past the last panel: the last one again, never read)
  auto issue = [&](double* st, int t) {
    t = min(t, nk - 1);
    const bool second = t >= nk1;
    const int k0 = (second ? t - nk1 : t) * BK;
    const double* Ab = (second ? A2 : A1) + k0;
    const double* Bb = (second ? B2 : B1) + (B_KC ? (int64_t)k0 : (int64_t)k0 * ldb);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      __builtin_amdgcn_global_load_lds(Ab + oa[j], (__attribute__((address_space(3))) void*)(st + (j * 256 + wave * 64) * 2),
                                       16, 0, 0);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      __builtin_amdgcn_global_load_lds(Bb + ob[j],
                                       (__attribute__((address_space(3))) void*)(st + AE + (j * 256 + wave * 64) * 2),
                                       16, 0, 0);
  };
  double acc[8][2];
#pragma unroll
  for (int a = 0; a < 8; ++a) acc[a][0] = acc[a][1] = 0.0;
  auto compute = [&](const double* st) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int k = ks + (lane >> 4);
      double af[8], bf[2];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int m = wm * 32 + a * 4 + (lane & 3);
        af[a] = st[m * BK + 2 * ((k >> 1) ^ (m & 7)) + (k & 1)];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int n = wn * 32 + b * 16 + (lane & 15);
        if constexpr (B_KC) bf[b] = st[AE + n * BK + 2 * ((k >> 1) ^ (n & 7)) + (k & 1)];
        else bf[b] = st[AE + k * BN + 2 * ((n >> 1) ^ (8 * (k & 3))) + (n & 1)];
      }
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };
  issue(st0, 0);
  issue(st1, 1);
  // step t: panel t's 4 loads per thread landed (the next panel's 4 may be
  // in flight) and this wave's earlier LDS reads done, then a plain barrier,
  // the refill of the stage read at step t - 1, and panel t
  auto step = [&](int t, const double* cur, double* nxt) {
    wait_vm_lgkm0<4 * (STAGES - 2)>();
    __builtin_amdgcn_s_barrier();
    issue(nxt, t + STAGES - 1);
    compute(cur);
  };
  int t = 0;
  for (; t + 3 <= nk; t += 3) {
    step(t, st0, st2);
    step(t + 1, st1, st0);
    step(t + 2, st2, st1);
  }
  if (t < nk) step(t, st0, st2);
  if (t + 1 < nk) step(t + 1, st1, st0);
  wait_vm_lgkm0<0>();

  const double alpha = p.alpha, beta = p.beta;
  auto row_of = [&](int a) { return m0 + wm * 32 + a * 4 + (lane >> 4); };
  auto col_of = [&](int b) { return n0 + wn * 32 + b * 16 + (lane & 15); };
  if (p.splits > 1) {
    double* __restrict__ W = p.ws + ((int64_t)split * p.nbtot + (int64_t)b1 * p.nb0 + b0) * p.M * p.N;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        if (row_of(a) < p.M && col_of(b) < p.N) W[(int64_t)row_of(a) * p.N + col_of(b)] = acc[a][b];
  } else if (beta == 0.0) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        if (row_of(a) < p.M && col_of(b) < p.N) Cg[row_of(a) * p.c_m + col_of(b) * p.c_n] = alpha * acc[a][b];
  } else {
    double cv[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) cv[a][b] = Cg[min(row_of(a), p.M - 1) * p.c_m + min(col_of(b), p.N - 1) * p.c_n];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        if (row_of(a) < p.M && col_of(b) < p.N)
          Cg[row_of(a) * p.c_m + col_of(b) * p.c_n] = alpha * acc[a][b] + beta * cv[a][b];
  }
}

// Products with a short contraction (K <= kSmallK) and a short output side
// (<= kSmallSide): a matrix-core tile would be mostly padding and the cost
// is one pass over the long operand. Each lane owns one index of the long
// output side, holds its K operand values in registers and produces every
// output along the short side; the short operand is staged in LDS and read
// as broadcasts. LONG_N: the long side is N.
constexpr int kSmallK = 32, kSmallSide = 32;

template <bool LONG_N>
__global__ __launch_bounds__(256) void gemm_smallk(KArgs p) {
  __shared__ double sh[kSmallSide * kSmallK];  // the short operand, [s][k]
  const int b0 = blockIdx.y % p.nb0;
  const int b1 = blockIdx.y / p.nb0 + blockIdx.z * (gridDim.y / p.nb0);
  const double* __restrict__ A = (const double*)p.A + b0 * p.a_b0 + b1 * p.a_b1;
  const double* __restrict__ B = (const double*)p.B + b0 * p.b_b0 + b1 * p.b_b1;
  double* __restrict__ C = (double*)p.C + b0 * p.c_b0 + b1 * p.c_b1;
  const int L = LONG_N ? p.N : p.M;
  const int S = LONG_N ? p.M : p.N;
  // the short side is split over p.splits groups of workgroups. With at
  // least 8 blocks of 256 along the long side, the groups of one block share
  // an XCD (block ids go round-robin over the 8 XCDs), so its operand is
  // read from HBM once; fewer blocks (batched products) map in order
  const int sgn = p.splits;
  const int nlb = (L + 255) / 256;
  int lblock, sg;
  if (nlb >= 8) {
    const int xcd = (int)(blockIdx.x % 8), q8 = (int)(blockIdx.x / 8);
    lblock = xcd + 8 * (q8 / sgn);
    sg = q8 % sgn;
  } else {
    lblock = (int)blockIdx.x / sgn;
    sg = (int)blockIdx.x % sgn;
  }
  const int sper = (S + sgn - 1) / sgn;
  const int s0 = sg * sper, s1 = min(S, s0 + sper);
  for (int q = threadIdx.x; q < S * p.K; q += 256) {
    const int s = q / p.K, k = q % p.K;
    sh[s * kSmallK + k] = LONG_N ? A[s * p.a_m + k * p.a_k] : B[k * p.b_k + s * p.b_n];
  }
  __syncthreads();
  const int l = lblock * 256 + threadIdx.x;
  if (l >= L || s0 >= s1) return;
  double r[kSmallK];
#pragma unroll
  for (int k = 0; k < kSmallK; ++k)
    r[k] = k < p.K ? (LONG_N ? B[k * p.b_k + l * p.b_n] : A[l * p.a_m + k * p.a_k]) : 0.0;
  for (int s = s0; s < s1; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kSmallK; ++k)
      if (k < p.K) acc += sh[s * kSmallK + k] * r[k];
    double* c = LONG_N ? C + s * p.c_m + l * p.c_n : C + l * p.c_m + s * p.c_n;
    double v = p.alpha * acc;
    if (p.beta != 0.0) v += p.beta * *c;
    *c = v;
  }
}

void launch_smallk(const GemmDesc& d, const void* A, const void* B, void* C, hipStream_t s) {
  KArgs p{};
  p.M = d.M; p.N = d.N; p.K = d.K; p.nb0 = d.nb0; p.splits = 1;
  p.A = A; p.a_m = d.a_m; p.a_k = d.a_k; p.a_b0 = d.a_b0; p.a_b1 = d.a_b1;
  p.B = B; p.b_k = d.b_k; p.b_n = d.b_n; p.b_b0 = d.b_b0; p.b_b1 = d.b_b1;
  p.C = C; p.c_m = d.c_m; p.c_n = d.c_n; p.c_b0 = d.c_b0; p.c_b1 = d.c_b1;
  p.alpha = d.alpha; p.beta = d.beta;
  // the long side is the one with more elements; ties go to N (usually the
  // contiguous index of C)
  const bool long_n = d.N >= d.M;
  const int L = long_n ? d.N : d.M;
  const int S = long_n ? d.M : d.N;
  int64_t gy = d.nb0, gz = d.nb1;
  while (gy * 2 <= 65535 && gz % 2 == 0) { gy *= 2; gz /= 2; }
  PNK_REQUIRE(gy <= 65535 && gz <= 65535, "gemm: batch too large");
  // one lane per index of the long side leaves a few waves per SIMD when
  // the long side is short of a million: split the short side into groups
  // (at most four) until about 4096 waves run
  const int64_t nlb = ceil_div(L, 256);
  const int64_t waves = nlb * 4 * (int64_t)d.nb0 * d.nb1;
  p.splits = (int)std::max<int64_t>(1, std::min<int64_t>({4, S, ceil_div(4096, std::max<int64_t>(waves, 1))}));
  dim3 grid((unsigned)((nlb >= 8 ? 8 * ceil_div(nlb, 8) : nlb) * p.splits), (unsigned)gy, (unsigned)gz);
  if (long_n) gemm_smallk<true><<<grid, 256, 0, s>>>(p);
  else gemm_smallk<false><<<grid, 256, 0, s>>>(p);
  PNK_CHECK_LAUNCH();
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
bool vec_ok(const void* base, int64_t s_row, int64_t s_k, int64_t s_b0, int64_t s_b1, bool kc) {
  const int64_t V = 16 / (int64_t)sizeof(T);
  if (!aligned16(base) || s_b0 % V != 0 || s_b1 % V != 0) return false;
  if (kc) return s_k == 1 && s_row % V == 0;
  return s_row == 1 && s_k % V == 0;
}

template <class Mma, typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM>
void launch_cfg(const GemmDesc& d, const void* A, const void* B, const void* A2, const void* B2, void* C,
                hipStream_t s) {
  KArgs p;
  p.A2 = A2;
  p.B2 = A2 ? B2 : nullptr;
  p.M = d.M; p.N = d.N; p.K = d.K; p.nb0 = d.nb0;
  p.tiles_m = (int)ceil_div(d.M, BM);
  p.tiles_n = (int)ceil_div(d.N, BN);
  p.A = A; p.a_m = d.a_m; p.a_k = d.a_k; p.a_b0 = d.a_b0; p.a_b1 = d.a_b1;
  p.B = B; p.b_k = d.b_k; p.b_n = d.b_n; p.b_b0 = d.b_b0; p.b_b1 = d.b_b1;
  p.C = C; p.c_m = d.c_m; p.c_n = d.c_n; p.c_b0 = d.c_b0; p.c_b1 = d.c_b1;
  p.alpha = d.alpha; p.beta = d.beta;
  const int64_t nb = (int64_t)d.nb0 * d.nb1;
  p.nbtot = (int)nb;
  const bool akc = d.a_k == 1 && d.a_m != 1;
  const bool bkc = d.b_k == 1 && d.b_n != 1;
  p.a_vec = vec_ok<TA>(A, d.a_m, d.a_k, d.a_b0, d.a_b1, akc) && (!A2 || vec_ok<TA>(A2, d.a_m, d.a_k, d.a_b0, d.a_b1, akc));
  p.b_vec = vec_ok<TB>(B, d.b_n, d.b_k, d.b_b0, d.b_b1, bkc) && (!A2 || vec_ok<TB>(B2, d.b_n, d.b_k, d.b_b0, d.b_b1, bkc));
  // split-K when the output tiles cannot fill the GPU
  int splits = 1;
  const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n * nb;
  // (short contractions are not split: the extra pass over the partial sums
  // would cost more than the product). About 900 workgroups in all (3.5 per
  // CU): for the o v x o v products of the rotated 10/90 workload that is 4
  // chunks, 10 % faster than 3 (a sweep over 3..12); thin products with a
  // long contraction stay near 512 (8 chunks for the ladder, its best).
  // Long contractions with fewer than 512 tiles (one or two workgroups per
  // CU, each walking thousands of k steps) are split too: the T1 part of
  // the ladder at o=20/v=180 (400 x 3600 x 32400, 399 tiles) ran at 22
  // TFLOP/s unsplit.
  // gridDim.y * gridDim.z covers the batch; y is a multiple of nb0, and z
  // also carries the chunks
  int64_t gy = d.nb0, gz = d.nb1;
  while (gy * 2 <= 65535 && gz % 2 == 0) { gy *= 2; gz /= 2; }
  const bool thin = d.M <= 64 && d.K >= 1024;
  const int64_t ws_fit =
      d.ws ? std::min<int64_t>(d.ws_elems / std::max<int64_t>(1, nb * d.M * d.N), 65535 / gz) : 0;
  constexpr bool f64 = sizeof(typename Mma::L) == 8;
  if (f64 && d.ws && ((d.K >= 8192 && tiles < 2048) || (d.K >= 2048 && tiles >= 256 && tiles < 1024))) {
    // Long FP64 contractions: split so that the work items (tiles x
    // chunks) reach about 2048 of 64 x 64 tiles' worth (8 per CU, enough
    // resident workgroups to hide latency) and fill the 256 CUs in whole
    // rounds; up to 8 chunks for a few hundred tiles or more, up to 1024 for
    // a handful (thin products streaming a long operand). Contractions of
    // 2048 or more with a few hundred tiles (2 or 3 per CU, unevenly) are
    // split the same way (the 600 x 3600 x 3600 DF product at o = 20, v =
    // 180: 570 tiles). At o = 20, v = 180
    // this took the antisymmetric ladder (756 tiles) from 3.0 to 2.5 ms with
    // 3 chunks and the symmetric one (384 tiles of 72 x 128) to 2.7 ms with
    // 4 (3 chunks, 4.5 rounds: 3.15).
    const double target = 2048.0 * 4096.0 / (BM * BN);
    const int64_t cap = tiles >= 256 ? 8 : 1024;
    double best = -1.0;
    for (int64_t sp = 1; sp <= cap && sp <= d.K / (2 * BK) && sp <= ws_fit; ++sp) {
      const int64_t items = tiles * sp;
      const double fill = std::min(1.0, (double)items / target);
      const double rounds = (double)items / (double)(ceil_div(items, 256) * 256);
      if (fill * rounds > best + 1e-9) {
        best = fill * rounds;
        splits = (int)sp;
      }
    }
  } else if (d.ws && d.K >= 256 && (tiles < 256 || (tiles < 512 && d.K >= 8192))) {
    int64_t want = ceil_div(thin ? 512 : 900, tiles);
    want = std::min<int64_t>(want, d.K / (2 * BK));
    want = std::min<int64_t>(want, ws_fit);
    want = std::min<int64_t>(want, 256);
    if (want >= 2) splits = (int)want;
  }
  p.kchunk = splits > 1 ? (int)(ceil_div(ceil_div(d.K, splits), BK) * BK) : d.K;
  if (splits > 1) splits = (int)ceil_div(d.K, p.kchunk);  // no empty chunk
  p.splits = splits;
  p.ws = d.ws;
  PNK_REQUIRE(gy <= 65535 && gz * splits <= 65535, "gemm: batch too large");
  dim3 grid((unsigned)(p.tiles_m * p.tiles_n), (unsigned)gy, (unsigned)(gz * splits));
  // BF16 operands both k-contiguous with whole 64-deep panels (the packed
  // copies): the pipelined kernel
  constexpr bool pipe_cfg = std::is_same<Mma, MmaBF16>::value && std::is_same<TA, uint16_t>::value &&
                            std::is_same<TB, uint16_t>::value && std::is_same<TC, double>::value && BM == 128 &&
                            BN == 128 && BK == 64;
  // FP64, A k-contiguous, B k- or n-contiguous (an even number of columns),
  // whole 16-deep panels, 16-byte rows: the pipelined FP64 kernel
  constexpr bool f64_cfg = std::is_same<Mma, MmaF64>::value && std::is_same<TA, double>::value &&
                           std::is_same<TB, double>::value && std::is_same<TC, double>::value && BM == 64 && BN == 64 &&
                           BK == 16;
  const bool bnc = d.b_n == 1 && d.b_k != 1;
  auto reduce = [&](const KArgs& q) {
    if (q.splits <= 1) return;
    const int64_t total = nb * d.M * d.N;
    if (q.splits >= 32)
      splitk_reduce_wide<TC><<<(unsigned)std::min<int64_t>(ceil_div(total, 16), 8192), 256, 0, s>>>(q);
    else
      splitk_reduce<TC><<<(unsigned)std::min<int64_t>(ceil_div(total, 256), 4096), 256, 0, s>>>(q);
    PNK_CHECK_LAUNCH();
  };
  if (pipe_cfg && akc && bkc && !A2 && d.K % 64 == 0 && p.a_vec && p.b_vec && d.M > 128) {
    // more than 128 rows: 256 x 128 tiles with 8 waves, one workgroup per
    // CU. Tiles that cannot fill the GPU take split-K in whole rounds of
    // 256 workgroups where possible (at most 8 chunks of 8 or more panels):
    // the ladder at o = 20, v = 180 (128 tiles) runs in 2 chunks, the T1
    // part (58 tiles) in 4
    KArgs q = p;
    q.tiles_m = (int)ceil_div(d.M, 256);
    const int64_t t2 = (int64_t)q.tiles_m * q.tiles_n * nb;
    int sp = 1;
    if (d.ws && t2 < 256) {
      double best = (double)t2 / 256.0;
      for (int64_t c = 2; c <= 8 && c <= d.K / (64 * 8) && c <= ws_fit; ++c) {
        const int64_t items = t2 * c;
        const double eff = (double)items / (double)(ceil_div(items, 256) * 256);
        if (eff > best + 1e-9) {
          best = eff;
          sp = (int)c;
        }
      }
    }
    q.kchunk = sp > 1 ? (int)(ceil_div(ceil_div(d.K, sp), 64) * 64) : d.K;
    if (sp > 1) sp = (int)ceil_div(d.K, q.kchunk);
    q.splits = sp;
    PNK_REQUIRE(gz * sp <= 65535, "gemm: batch too large");
    dim3 g2((unsigned)(q.tiles_m * q.tiles_n), (unsigned)gy, (unsigned)(gz * sp));
    gemm_bf16_pipe<256, 8><<<g2, 512, 0, s>>>(q);
    PNK_CHECK_LAUNCH();
    reduce(q);
    return;
  }
  if (pipe_cfg && akc && bkc && !A2 && d.K % 64 == 0 && p.a_vec && p.b_vec) {
    gemm_bf16_pipe<128, 4><<<grid, 256, 0, s>>>(p);
  } else if (f64_cfg && akc && d.K % 16 == 0 && p.a_vec && p.b_vec && d.M >= 2 && (bkc || (bnc && d.N % 2 == 0))) {
    if (bkc) gemm_f64_pipe<true><<<grid, 256, 0, s>>>(p);
    else gemm_f64_pipe<false><<<grid, 256, 0, s>>>(p);
  } else if (akc && bkc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, true, true><<<grid, 256, 0, s>>>(p);
  else if (akc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, true, false><<<grid, 256, 0, s>>>(p);
  else if (bkc) gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, false, true><<<grid, 256, 0, s>>>(p);
  else gemm_kernel<Mma, TA, TB, TC, BM, BN, BK, WGM, false, false><<<grid, 256, 0, s>>>(p);
  PNK_CHECK_LAUNCH();
  reduce(p);
}


// Tile choice. FP64: 64 x 64 with 16-deep panels (a sweep over 32/64/96/128
// x 64 tiles and 16/32-deep panels on MI355X put it at or within 3 % of the
// best for square products from 900 to 3600); row counts that 72-row tiles
// fit much better take 72 x 128; thin products (at most 64 rows) with a
// long contraction stream their wide operand from HBM and take 32-deep
// panels (about 20 % faster there).
// FP32/BF16: 128 x 128. Small products: 64 x 64 (split-K fills the GPU).
template <class Mma, typename TA, typename TB, typename TC, int BK>
void launch_sized(const GemmDesc& d, const void* A, const void* B, const void* A2, const void* B2, void* C,
                  hipStream_t s) {
  const int64_t nb = (int64_t)d.nb0 * d.nb1;
  if constexpr (sizeof(typename Mma::L) == 8) {
    // long contractions of more than 64 rows that the pipelined FP64 kernel
    // takes (A k-contiguous with 16-byte rows, B k-contiguous or
    // n-contiguous with an even column count): its 64 x 64 tiles before the
    // 72/80-row rules below (thin products keep their 32-deep tiles); a
    // contraction that is not a whole number of 16-deep panels runs its
    // last K % 16 columns as a second product added into C (the ladders at
    // o = 20, v = 180: K = 16290 and 16110)
    const bool akc = d.a_k == 1 && d.a_m != 1, bkc = d.b_k == 1 && d.b_n != 1, bnc = d.b_n == 1 && d.b_k != 1;
    const bool pipe_ok =
        akc && d.M > 64 && d.K >= 1024 && (bkc || (bnc && d.N % 2 == 0)) &&
        vec_ok<double>(A, d.a_m, d.a_k, d.a_b0, d.a_b1, true) &&
        (!A2 || vec_ok<double>(A2, d.a_m, d.a_k, d.a_b0, d.a_b1, true)) &&
        vec_ok<double>(B, d.b_n, d.b_k, d.b_b0, d.b_b1, bkc) && (!A2 || vec_ok<double>(B2, d.b_n, d.b_k, d.b_b0, d.b_b1, bkc));
    if (pipe_ok) {
      const int r = d.K % 16;
      GemmDesc dm = d;
      dm.K = d.K - r;
      launch_cfg<Mma, TA, TB, TC, 64, 64, 16, 2>(dm, A, B, A2, B2, C, s);
      if (r) {
        GemmDesc dt = d;
        dt.K = r;
        dt.beta = 1.0;
        const int64_t ka = (int64_t)(d.K - r) * d.a_k, kb = (int64_t)(d.K - r) * d.b_k;
        launch_cfg<Mma, TA, TB, TC, 64, 64, 16, 2>(dt, (const double*)A + ka, (const double*)B + kb,
                                                   A2 ? (const double*)A2 + ka : nullptr,
                                                   A2 ? (const double*)B2 + kb : nullptr, C, s);
      }
      return;
    }
    // otherwise, row counts that 72- or 80-row tiles cover with at least 10 %
    // less padding than 64-row ones (such as the ladder's 210 pair rows, 216
    // against 256, and the 400 rows of its T1 part, 400 against 448, when
    // their operands do not suit the pipelined kernel), with a long
    // contraction: 72 x 128 or 80 x 128 with 8-deep panels (9 % and 16 %
    // faster than the register-staged 64 x 64 tiles there)
    const int64_t r64 = ceil_div(d.M, 64) * 64, r72 = ceil_div(d.M, 72) * 72, r80 = ceil_div(d.M, 80) * 80;
    // (at least 128 such tiles: fewer go to 64 x 64 tiles and many chunks)
    const int64_t n128 = ceil_div(d.N, 128) * nb;
    if (d.K >= 1024 && r80 < r72 && 10 * r80 <= 9 * r64 && (r80 / 80) * n128 >= 128)
      launch_cfg<Mma, TA, TB, TC, 80, 128, 8, 2>(d, A, B, A2, B2, C, s);
    else if (d.K >= 1024 && 10 * r72 <= 9 * r64 && (r72 / 72) * n128 >= 128)
      launch_cfg<Mma, TA, TB, TC, 72, 128, 8, 2>(d, A, B, A2, B2, C, s);
    // a few 64-row tiles with a long contraction (the antisymmetric ladder's
    // 190 pair rows at o = 20): 64 x 128 with 8-deep panels, 5 % faster
    else if (d.M > 64 && d.M <= 256 && d.K >= 8192 && (r64 / 64) * n128 >= 128)
      launch_cfg<Mma, TA, TB, TC, 64, 128, 8, 2>(d, A, B, A2, B2, C, s);
    else if (d.M <= 64 && d.K >= 1024) launch_cfg<Mma, TA, TB, TC, 64, 64, 32, 2>(d, A, B, A2, B2, C, s);
    else launch_cfg<Mma, TA, TB, TC, 64, 64, BK, 2>(d, A, B, A2, B2, C, s);
  } else {
    const int64_t big = ceil_div(d.M, 128) * ceil_div(d.N, 128) * nb;
    // BF16 128 x 128 tiles take two matrix-core steps per panel (64-deep):
    // 25-45 % faster than one on the ring, ladder and T1-ladder products
    constexpr bool bf16 = std::is_same<Mma, MmaBF16>::value;
    constexpr int BK128 = bf16 ? 64 : BK;
    // (BF16 with a long contraction takes them from 64 tiles on, split-K
    // filling the GPU: 1.2-2.3x faster than 64 x 64 on the T1 part of the
    // ladder and the antisymmetric ladder at o = 20, v = 180)
    // (BF16 products the pipelined kernel takes, two packed operands with
    // whole panels: from 32 tiles on, split-K filling the GPU)
    const bool pipe_ok = bf16 && std::is_same<TA, uint16_t>::value && std::is_same<TB, uint16_t>::value &&
                         d.a_k == 1 && d.b_k == 1 && d.K % 64 == 0 && !A2;
    const bool wide = big >= 256 || (bf16 && d.K >= 8192 && big >= 64) || (pipe_ok && big >= 32);
    if (d.M >= 64 && d.N >= 96 && wide) launch_cfg<Mma, TA, TB, TC, 128, 128, BK128, 2>(d, A, B, A2, B2, C, s);
    else launch_cfg<Mma, TA, TB, TC, 64, 64, BK, 2>(d, A, B, A2, B2, C, s);
  }
}

}  // namespace

namespace {

// Rounds one FP64 operand of a (batched) product to the compute type and
// writes it as rows contiguous along k: out[b][r][koff + k] (row length
// ld) = in[b0 * s_b0 + b1 * s_b1 + r * s_r + k * s_k], b = b1 * nb0 + b0.
// 32 x 32 tiles through LDS, so reads are coalesced along whichever index
// is contiguous in the input and writes along k.
struct PackArgs {
  const double* in;
  int64_t s_r, s_k, s_b0, s_b1;
  int rows, K, kz, nb0, ld, koff;  // columns koff .. koff + kz - 1 written, zeros past K
  void* out;
  int vst;  // rows of out 16-byte aligned at every multiple of 8 columns (16-byte stores)
};

template <typename T>
__global__ __launch_bounds__(256) void pack_operand(PackArgs p) {
  // 32 rows x 64 k per workgroup: read coalesced along whichever index is
  // contiguous in the input, then 8 lanes per row write 8 consecutive k
  // each (one 16-byte store of BF16, two of FP32, where aligned)
  __shared__ double tile[64][33];  // [k - k0][r - r0]
  const int tiles_k = (p.kz + 63) / 64;
  const int r0 = (blockIdx.x / tiles_k) * 32, k0 = (blockIdx.x % tiles_k) * 64;
  const int b = blockIdx.y;
  const int b0 = b % p.nb0, b1 = b / p.nb0;
  const double* in = p.in + b0 * p.s_b0 + b1 * p.s_b1;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  if (p.s_r == 1 && p.s_k != 1) {
    // consecutive lanes walk r
    for (int j = ty; j < 64; j += 8) {
      const int r = r0 + tx, k = k0 + j;
      tile[j][tx] = r < p.rows && k < p.K ? in[(int64_t)r + (int64_t)k * p.s_k] : 0.0;
    }
  } else {
    // consecutive lanes walk k
    for (int j = ty; j < 32; j += 8)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + j, k = k0 + 32 * h + tx;
        tile[32 * h + tx][j] = r < p.rows && k < p.K ? in[(int64_t)r * p.s_r + (int64_t)k * p.s_k] : 0.0;
      }
  }
  __syncthreads();
  const int rr = threadIdx.x >> 3, kc = (threadIdx.x & 7) * 8;
  const int r = r0 + rr;
  if (r >= p.rows) return;
  T y[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) y[e] = to_lds<double, T>(tile[kc + e][rr]);
  T* dst = (T*)p.out + (int64_t)b * p.rows * p.ld + (int64_t)r * p.ld + p.koff + k0 + kc;
  if (p.vst && k0 + kc + 8 <= p.kz) {
    uint4* d4 = reinterpret_cast<uint4*>(dst);
#pragma unroll
    for (int q = 0; q < (int)sizeof(y) / 16; ++q) {
      uint4 w;
      __builtin_memcpy(&w, reinterpret_cast<const char*>(y) + 16 * q, 16);
      d4[q] = w;
    }
  } else {
    for (int e = 0; e < 8 && k0 + kc + e < p.kz; ++e) dst[e] = y[e];
  }
}

// The same rounding for an input already contiguous along k (s_k = 1),
// with 16-byte aligned rows and segments: no transpose, so each lane reads
// 16 / sizeof(T) consecutive doubles of a row and writes them as one
// 16-byte store. Lanes walk the row's chunks, rows follow each other in the
// grid-stride. (Measured on MI355X against a form with one 16-byte load and
// one pair store per lane, fully coalesced: about 5 % faster on the 3600 x
// 3600 operands of the ring products.)
template <typename T>
__global__ __launch_bounds__(256) void pack_operand_kc(PackArgs p) {
  constexpr int VE = 16 / (int)sizeof(T);  // elements per 16-byte store
  const int b = blockIdx.y;
  const int b0 = b % p.nb0, b1 = b / p.nb0;
  const double* __restrict__ in = p.in + b0 * p.s_b0 + b1 * p.s_b1;
  T* __restrict__ out = (T*)p.out + (int64_t)b * p.rows * p.ld + p.koff;
  const int cpr = (p.kz + VE - 1) / VE;  // chunks per row
  const int64_t total = (int64_t)p.rows * cpr;
  for (int64_t c = blockIdx.x * (int64_t)256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    const int r = (int)(c / cpr), k0 = (int)(c % cpr) * VE;
    const double* src = in + (int64_t)r * p.s_r + k0;
    double x[VE];
    if (k0 + VE <= p.K) {
#pragma unroll
      for (int e = 0; e < VE; e += 2) {
        const double2 t = *reinterpret_cast<const double2*>(src + e);
        x[e] = t.x;
        x[e + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) x[e] = k0 + e < p.K ? src[e] : 0.0;
    }
    T y[VE];
#pragma unroll
    for (int e = 0; e < VE; ++e) y[e] = to_lds<double, T>(x[e]);
    T* dst = out + (int64_t)r * p.ld + k0;
    if (k0 + VE <= p.kz) {
      uint4 w;
      __builtin_memcpy(&w, y, 16);
      *reinterpret_cast<uint4*>(dst) = w;
    } else {
      for (int e = 0; k0 + e < p.kz; ++e) dst[e] = y[e];
    }
  }
}

template <typename T>
void pack(const double* in, int64_t s_r, int64_t s_k, int64_t s_b0, int64_t s_b1, int rows, int K, int kz, int nb0,
          int nb1, int ld, int koff, void* out, hipStream_t s) {
  const int vst = ((uintptr_t)out & 15u) == 0 && ld % 8 == 0 && koff % 8 == 0;
  PackArgs p{in, s_r, s_k, s_b0, s_b1, rows, K, kz, nb0, ld, koff, out, vst};
  // k-contiguous input with 16-byte aligned chunks in and out
  constexpr int VE = 16 / (int)sizeof(T);
  const bool kc = s_k == 1 && rows > 0 && ((uintptr_t)in & 15u) == 0 && s_r % 2 == 0 && s_b0 % 2 == 0 &&
                  s_b1 % 2 == 0 && ((uintptr_t)out & 15u) == 0 && ld % VE == 0 && koff % VE == 0;
  if (kc) {
    const int64_t total = (int64_t)rows * ceil_div(kz, VE);
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(total, 256), 4096), (unsigned)(nb0 * nb1));
    pack_operand_kc<T><<<grid, 256, 0, s>>>(p);
  } else {
    dim3 grid((unsigned)(ceil_div(rows, 32) * ceil_div(kz, 64)), (unsigned)(nb0 * nb1));
    pack_operand<T><<<grid, 256, 0, s>>>(p);
  }
  PNK_CHECK_LAUNCH();
}

void gemm_impl(const GemmDesc& d, const void* A, const void* B, const void* A2, const void* B2, Prec ap, Prec bp,
               void* C, Prec cp, Prec compute, hipStream_t s);

// FP32/BF16 product with FP64 operands rounded once into d.cast_ws (both
// products of a dual call side by side along k). Returns false when it does
// not apply or does not fit.
bool gemm_precast(const GemmDesc& d, const void* A, const void* B, const void* A2, const void* B2, Prec ap, Prec bp,
                  void* C, Prec cp, Prec compute, hipStream_t s) {
  if (!d.cast_ws || (compute != Prec::F32 && compute != Prec::BF16)) return false;
  // an operand is rounded once only when more than one column (row) of
  // tiles reads it; a thin product (the o x o outputs of the Fock terms)
  // streams it once, and rounding it on load saves a pass over it
  const bool pa = ap == Prec::F64 && d.N > 64, pb = bp == Prec::F64 && d.M > 64;
  if (!pa && !pb) return false;
  const int64_t nb = (int64_t)d.nb0 * d.nb1;
  if ((double)d.M * d.N * d.K * nb < 1e7) return false;  // small: convert on load
  const bool dual = A2 != nullptr;
  if (dual && pa != pb) return false;
  const int64_t es = compute == Prec::BF16 ? 2 : 4;
  const int kt = dual ? 2 * d.K : d.K;
  // rows of the copies start on 16-byte boundaries (vector loads); BF16
  // rows are zero-padded to a multiple of 64 elements (whole panels of the
  // pipelined kernel)
  const int lq = compute == Prec::BF16 ? 64 : 16 / (int)es;
  const int ld = (int)((kt + lq - 1) / lq * lq);
  const int64_t need = es * nb * ((pa ? (int64_t)d.M * ld : 0) + (pb ? (int64_t)d.N * ld : 0)) + 256;
  if (need > d.cast_ws_bytes) return false;
  char* base = (char*)d.cast_ws;
  char* abuf = base;
  char* bbuf = base + (((pa ? es * nb * (int64_t)d.M * ld : 0) + 255) & ~int64_t(255));
  GemmDesc e = d;
  e.cast_ws = nullptr;
  const void *An = A, *Bn = B;
  Prec apn = ap, bpn = bp;
  // (the last segment of a row also writes the zeros up to ld)
  auto run_pack = [&](const void* src, bool is_a, int koff, void* dst) {
    const double* in = (const double*)src;
    const int rows = is_a ? d.M : d.N;
    const int64_t sr = is_a ? d.a_m : d.b_n, sk = is_a ? d.a_k : d.b_k;
    const int64_t sb0 = is_a ? d.a_b0 : d.b_b0, sb1 = is_a ? d.a_b1 : d.b_b1;
    const int kz = koff + d.K == kt ? ld - koff : d.K;
    if (es == 2) pack<uint16_t>(in, sr, sk, sb0, sb1, rows, d.K, kz, d.nb0, d.nb1, ld, koff, dst, s);
    else pack<float>(in, sr, sk, sb0, sb1, rows, d.K, kz, d.nb0, d.nb1, ld, koff, dst, s);
  };
  if (pa) {
    run_pack(A, true, 0, abuf);
    if (dual) run_pack(A2, true, d.K, abuf);
    An = abuf;
    apn = compute;
    e.a_m = ld; e.a_k = 1; e.a_b0 = (int64_t)d.M * ld; e.a_b1 = (int64_t)d.nb0 * d.M * ld;
  }
  if (pb) {
    run_pack(B, false, 0, bbuf);
    if (dual) run_pack(B2, false, d.K, bbuf);
    Bn = bbuf;
    bpn = compute;
    e.b_n = ld; e.b_k = 1; e.b_b0 = (int64_t)d.N * ld; e.b_b1 = (int64_t)d.nb0 * d.N * ld;
  }
  // both products of a dual call packed along k: one product of depth 2K;
  // with both operands zero-padded to ld the contraction runs over the
  // padding too
  const bool bpad = !pb && bp == compute && d.b_k == 1 && d.b_kzero >= ld;
  e.K = pa && (pb || bpad) ? ld : kt;
  gemm_impl(e, An, Bn, nullptr, nullptr, apn, bpn, C, cp, compute, s);
  return true;
}

void gemm_impl(const GemmDesc& d, const void* A, const void* B, const void* A2, const void* B2, Prec ap, Prec bp,
               void* C, Prec cp, Prec compute, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.nb0 <= 0 || d.nb1 <= 0) return;
  PNK_REQUIRE(cp == Prec::F64 || cp == Prec::F32, "gemm: C must be f64 or f32");
  PNK_REQUIRE(d.K > 0, "gemm: K must be positive");
  if (gemm_precast(d, A, B, A2, B2, ap, bp, C, cp, compute, s)) return;
#define PNK_GEMM_CASE(MMA, TA, TB, TC, BK) return launch_sized<MMA, TA, TB, TC, BK>(d, A, B, A2, B2, C, s)
  if (compute == Prec::F64) {
    PNK_REQUIRE(ap == Prec::F64 && bp == Prec::F64, "gemm: f64 compute needs f64 operands");
    PNK_REQUIRE(cp == Prec::F64, "gemm: f64 compute writes f64");
    if (d.K <= kSmallK && std::min(d.M, d.N) <= kSmallSide) {
      launch_smallk(d, A, B, C, s);
      if (A2) {
        GemmDesc e = d;
        e.beta = 1.0;
        launch_smallk(e, A2, B2, C, s);
      }
      return;
    }
    PNK_GEMM_CASE(MmaF64, double, double, double, 16);
  }
  if (compute == Prec::F32) {
    PNK_REQUIRE(cp == Prec::F64, "gemm: f32 compute writes f64");
    if (ap == Prec::F64 && bp == Prec::F64) PNK_GEMM_CASE(MmaF32, double, double, double, 16);
    if (ap == Prec::F64 && bp == Prec::F32) PNK_GEMM_CASE(MmaF32, double, float, double, 16);
    if (ap == Prec::F32 && bp == Prec::F64) PNK_GEMM_CASE(MmaF32, float, double, double, 16);
    if (ap == Prec::F32 && bp == Prec::F32) PNK_GEMM_CASE(MmaF32, float, float, double, 16);
  }
  if (compute == Prec::BF16) {
    PNK_REQUIRE(cp == Prec::F64, "gemm: bf16 compute writes f64");
    if (ap == Prec::F64 && bp == Prec::F64) PNK_GEMM_CASE(MmaBF16, double, double, double, 32);
    if (ap == Prec::F64 && bp == Prec::BF16) PNK_GEMM_CASE(MmaBF16, double, uint16_t, double, 32);
    if (ap == Prec::BF16 && bp == Prec::F64) PNK_GEMM_CASE(MmaBF16, uint16_t, double, double, 32);
    if (ap == Prec::BF16 && bp == Prec::BF16) PNK_GEMM_CASE(MmaBF16, uint16_t, uint16_t, double, 32);
  }
#undef PNK_GEMM_CASE
  PNK_REQUIRE(false, "gemm: unsupported precision combination");
}

}  // namespace

void gemm(const GemmDesc& d, const void* A, Prec ap, const void* B, Prec bp, void* C, Prec cp, Prec compute,
          hipStream_t s) {
  gemm_impl(d, A, B, nullptr, nullptr, ap, bp, C, cp, compute, s);
}

void gemm_sum(const GemmDesc& d, const void* A1, const void* B1, const void* A2, const void* B2, Prec ap, Prec bp,
              void* C, Prec cp, Prec compute, hipStream_t s) {
  PNK_REQUIRE(A2 && B2, "gemm_sum: second product missing");
  gemm_impl(d, A1, B1, A2, B2, ap, bp, C, cp, compute, s);
}

}  // namespace pnk
