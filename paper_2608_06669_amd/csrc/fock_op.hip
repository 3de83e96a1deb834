// Fused Fock operator (see fock_op.hpp).
//
// One workgroup computes a BM x BM block (a, b) of y_ij for one occupied
// pair (i, j). The two virtual contractions form a single matrix-core
// product over a contraction of length 2v: panels 0 .. nkp-1 multiply
// f_vv[a][c] by x_ij[c][b], panels nkp .. 2nkp-1 multiply x_ij[a][c] by
// f_vv[c][b] (f_vv is symmetric), so both accumulate into the same
// registers with the FP64 4x4x4 matrix-core instruction and LDS double
// buffering. The two occupied contractions are short (length o) and are
// added in the epilogue from global memory (the o slices x_kj and x_ik of
// the block are read once each per workgroup and hit L2), with the f_oo
// columns i and j staged in LDS. One extra row of workgroups computes the
// singles. With the Lanczos fusion the epilogue also forms
// p = y - beta v_{k-1} and a fixed-order per-workgroup partial of <v_k, p>.

#include "fock_op.hpp"
#include "mfma_tiles.hpp"

#include <algorithm>

namespace pnk {
namespace {

using namespace tiles;

struct FockKArgs {
  int o, v, tiles_m, tiles;
  int vec;  // 16-byte operand loads allowed
  const double* f_oo;
  const double* f_vv;
  const double* x1;  // singles and doubles blocks of the input
  const double* x2;
  double* y1;        // ... and of the output
  double* y2;
  const double* vprev1;
  const double* vprev2;
  const double* beta;
  double* partials;
};

template <int BM, int WGM, bool LZ>
__global__ __launch_bounds__(256) void fock_op_kernel(FockKArgs p) {
  using Mma = MmaF64;
  constexpr int BN = BM;
  constexpr int BK = 16;
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TMI = WTM / Mma::TM, TNI = WTN / Mma::TN;
  static_assert(WTM % Mma::TM == 0 && WTN % Mma::TN == 0, "wave tile must split into instruction tiles");
  constexpr int ALDS = lds_elems<Mma, BM, BK>();
  constexpr int BLDS = lds_elems<Mma, BN, BK>();
  __shared__ __attribute__((aligned(16))) double As[2][ALDS];
  __shared__ __attribute__((aligned(16))) double Bs[2][BLDS];
  __shared__ double fi[kFockOpMaxOcc];
  __shared__ double fj[kFockOpMaxOcc];
  __shared__ double red[256];

  const int o = p.o, v = p.v;
  const int64_t ov = (int64_t)o * v, vv = (int64_t)v * v;
  const double* __restrict__ x1 = p.x1;
  const double* __restrict__ x2 = p.x2;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int pair = blockIdx.y;
  double beta = 0.0;
  if constexpr (LZ) beta = *p.beta;
  double dot = 0.0;

  if (pair < o * o) {
    if ((int)blockIdx.x < p.tiles) {  // uniform over the workgroup
      const int i = pair / o, j = pair % o;
      for (int k = tid; k < o; k += 256) {
        fi[k] = p.f_oo[(int64_t)k * o + i];
        fj[k] = p.f_oo[(int64_t)k * o + j];
      }
      const int wm = wave / WGN, wn = wave % WGN;
      const int m0 = (blockIdx.x % p.tiles_m) * BM;
      const int n0 = (blockIdx.x / p.tiles_m) * BN;
      const double* __restrict__ X = x2 + (int64_t)pair * vv;
      const double* __restrict__ F = p.f_vv;
      const bool vec = p.vec != 0;
      const int nkp = (v + BK - 1) / BK;
      const int nk = 2 * nkp;

      double acc[TMI][TNI];
#pragma unroll
      for (int a = 0; a < TMI; ++a)
#pragma unroll
        for (int b = 0; b < TNI; ++b) acc[a][b] = 0.0;

      Panel<Mma, double, BM, BK, true> pa;   // A[a][c], contiguous along c
      Panel<Mma, double, BN, BK, false> pb;  // B[c][b], contiguous along b
      auto load = [&](int t) {
        const int ph = t >= nkp ? 1 : 0;
        const int k0 = (t - ph * nkp) * BK;
        pa.load(ph ? X : F, v, 1, m0, v, k0, v, vec, tid);
        pb.load(ph ? F : X, 1, v, n0, v, k0, v, vec, tid);
      };
      load(0);
      pa.store(As[0], tid);
      pb.store(Bs[0], tid);
      __syncthreads();
      for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load(kt + 1);
        const double* Ac = As[cur];
        const double* Bc = Bs[cur];
#pragma unroll
        for (int ks = 0; ks < BK; ks += Mma::KSTEP) {
          const int kk = ks + (lane >> 4);
          double af[TMI], bf[TNI];
#pragma unroll
          for (int a = 0; a < TMI; ++a) af[a] = Ac[kk * (BM + kPad) + wm * WTM + a * 4 + (lane & 3)];
#pragma unroll
          for (int b = 0; b < TNI; ++b) bf[b] = Bc[kk * (BN + kPad) + wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < TMI; ++a)
#pragma unroll
            for (int b = 0; b < TNI; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        if (kt + 1 < nk) {
          pa.store(As[cur ^ 1], tid);
          pb.store(Bs[cur ^ 1], tid);
        }
        __syncthreads();
      }

      const double* __restrict__ xkj = x2 + (int64_t)j * vv;           // + k o v^2
      const double* __restrict__ xik = x2 + (int64_t)i * o * vv;       // + k v^2
      const int64_t step_kj = (int64_t)o * vv;
#pragma unroll
      for (int a = 0; a < TMI; ++a)
#pragma unroll
        for (int b = 0; b < TNI; ++b) {
          const int ga = m0 + wm * WTM + a * 4 + (lane >> 4);
          const int gb = n0 + wn * WTN + b * 16 + (lane & 15);
          if (ga >= v || gb >= v) continue;
          const int64_t ab = (int64_t)ga * v + gb;
          double y = acc[a][b];
          for (int k = 0; k < o; ++k) y -= fi[k] * xkj[k * step_kj + ab] + fj[k] * xik[k * vv + ab];
          const int64_t idx = (int64_t)pair * vv + ab;
          if constexpr (LZ) {
            const double q = y - beta * p.vprev2[idx];
            p.y2[idx] = q;
            dot += x2[idx] * q;
          } else {
            p.y2[idx] = y;
          }
        }
    }
  } else {
    const int64_t e = (int64_t)blockIdx.x * 256 + tid;
    if (e < ov) {
      const int i = (int)(e / v), a = (int)(e % v);
      double y = 0.0;
      for (int c = 0; c < v; ++c) y += p.f_vv[(int64_t)a * v + c] * x1[(int64_t)i * v + c];
      for (int k = 0; k < o; ++k) y -= p.f_oo[(int64_t)k * o + i] * x1[(int64_t)k * v + a];
      if constexpr (LZ) {
        const double q = y - beta * p.vprev1[e];
        p.y1[e] = q;
        dot += x1[e] * q;
      } else {
        p.y1[e] = y;
      }
    }
  }

  if constexpr (LZ) {
    red[tid] = dot;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) p.partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  }
}

bool aligned16(const void* q) { return ((uintptr_t)q & 15u) == 0; }

template <bool LZ>
void launch(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, const double* vprev1,
            const double* vprev2, const double* beta, double* partials, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0, "fock_op: not planned");
  PNK_REQUIRE(x1 != y1 && x2 != y2, "fock_op: output must not alias the input");
  FockKArgs a;
  a.o = op.o;
  a.v = op.v;
  a.tiles_m = (int)ceil_div(op.v, op.bm);
  a.tiles = op.tiles;
  a.vec = (op.v % 2 == 0 && aligned16(x2) && aligned16(op.f_vv)) ? 1 : 0;
  a.f_oo = op.f_oo;
  a.f_vv = op.f_vv;
  a.x1 = x1;
  a.x2 = x2;
  a.y1 = y1;
  a.y2 = y2;
  a.vprev1 = vprev1;
  a.vprev2 = vprev2;
  a.beta = beta;
  a.partials = partials;
  dim3 grid((unsigned)op.gx, (unsigned)op.gy);
  switch (op.bm) {
    case 32: fock_op_kernel<32, 2, LZ><<<grid, 256, 0, s>>>(a); break;
    case 48: fock_op_kernel<48, 4, LZ><<<grid, 256, 0, s>>>(a); break;
    default: fock_op_kernel<64, 2, LZ><<<grid, 256, 0, s>>>(a); break;
  }
  PNK_CHECK_LAUNCH();
}

}  // namespace

// Tile: the block edge among 32 / 48 / 64 that wastes the fewest padded
// outputs (v^2 / (tiles * bm^2)); among near-ties the largest edge that
// still gives at least 512 workgroups (two per CU), else the smallest.
bool fock_op_plan(FockOp& op) {
  if (op.o < 1 || op.v < 1 || op.o >= kFockOpMaxOcc) return false;
  const int cand[3] = {32, 48, 64};
  double util[3], best = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double t = (double)ceil_div(op.v, cand[c]) * cand[c];
    util[c] = (double)op.v * op.v / (t * t);
    best = std::max(best, util[c]);
  }
  int pick = -1;
  for (int c = 2; c >= 0; --c) {
    if (util[c] < 0.98 * best) continue;
    const int64_t tiles = ceil_div(op.v, cand[c]) * ceil_div(op.v, cand[c]);
    if ((int64_t)op.o * op.o * tiles >= 512) { pick = c; break; }
  }
  if (pick < 0)
    for (int c = 0; c < 3; ++c)
      if (util[c] >= 0.98 * best) { pick = c; break; }
  op.bm = cand[pick];
  const int64_t tm = ceil_div(op.v, op.bm);
  op.tiles = (int)(tm * tm);
  const int64_t singles = ceil_div((int64_t)op.o * op.v, 256);
  op.gx = (int)std::max<int64_t>(op.tiles, singles);
  op.gy = op.o * op.o + 1;
  return op.gx <= 65535 && op.gy <= 65535;
}

bool fock_op_is_lanczos_kernel(const void* func) {
  return func == reinterpret_cast<const void*>(&fock_op_kernel<32, 2, true>) ||
         func == reinterpret_cast<const void*>(&fock_op_kernel<48, 4, true>) ||
         func == reinterpret_cast<const void*>(&fock_op_kernel<64, 2, true>);
}

void fock_op_apply(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, hipStream_t s) {
  launch<false>(op, x1, x2, y1, y2, nullptr, nullptr, nullptr, nullptr, s);
}

void fock_op_lanczos(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                     double* partials, hipStream_t s) {
  const int64_t ov = (int64_t)op.o * op.v;
  launch<true>(op, v, v + ov, p, p + ov, vprev, vprev + ov, beta, partials, s);
}

}  // namespace pnk
