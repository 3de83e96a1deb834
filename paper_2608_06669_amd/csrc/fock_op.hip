// Fock operator A_F in two launches (see fock_op.hpp).
//
// Virtual kernel: one workgroup computes a bm x bm block (a, b) of
// y_ij = f_vv x_ij + x_ij f_vv for one occupied pair (i, j). The two
// contractions form a single matrix-core product over a contraction of
// length 2v: panels 0 .. nkp-1 multiply f_vv[a][c] by x_ij[c][b], panels
// nkp .. 2nkp-1 multiply x_ij[a][c] by f_vv[c][b] (f_vv is symmetric), so
// both accumulate into the same registers (FP64 4x4x4 matrix-core
// instruction, LDS double buffering).
//
// Occupied kernel: the two occupied contractions are short (length o) but
// touch o slices of x per output; done per output they re-read x 2o times.
// Instead one workgroup stages x[:, :, chunk] (all o^2 pairs for a chunk of
// ch consecutive (a, b)) in LDS once and forms both sums for every pair
// from there, so x is read from memory once. The same launch adds the
// virtual part, applies the Lanczos update and sums <v_k, p>, <p, p> and
// <v_k, v_k> per workgroup.
// Trailing workgroups compute the singles, 16 lanes per output.

#include "fock_op.hpp"
#include "block_sum.hpp"
#include "mfma_tiles.hpp"

#include <algorithm>

namespace pnk {
namespace {

using namespace tiles;

struct VirArgs {
  int v, tiles_m, tiles, units, per_xcd;
  int vec;  // 16-byte operand loads allowed
  const double* f_vv;
  const double* x2;
  double* y2;
  const double* done;  // when set and nonzero on entry, the launch does nothing
};

template <int BM, int WGM, int BK>
__global__ __launch_bounds__(256) void fock_vir_kernel(VirArgs p) {
  using Mma = MmaF64;
  constexpr int BN = BM;
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TMI = WTM / Mma::TM, TNI = WTN / Mma::TN;
  static_assert(WTM % Mma::TM == 0 && WTN % Mma::TN == 0, "wave tile must split into instruction tiles");
  constexpr int ALDS = lds_elems<Mma, BM, BK>();
  constexpr int BLDS = lds_elems<Mma, BN, BK>();
  __shared__ __attribute__((aligned(16))) double As[2][ALDS];
  __shared__ __attribute__((aligned(16))) double Bs[2][BLDS];

  if (p.done && *p.done != 0.0) return;
  const int v = p.v;
  const int64_t vv = (int64_t)v * v;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  // Workgroups are dispatched round-robin over the 8 XCDs; consecutive
  // units (the tiles of one pair) are given to one XCD so the pair's slab
  // of x is fetched into that XCD's L2 once.
  const int u = (int)(blockIdx.x % 8) * p.per_xcd + (int)(blockIdx.x / 8);
  if (u >= p.units) return;
  const int pair = u / p.tiles, tile = u % p.tiles;
  const int m0 = (tile % p.tiles_m) * BM;
  const int n0 = (tile / p.tiles_m) * BN;
  const double* __restrict__ X = p.x2 + (int64_t)pair * vv;
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

  double* __restrict__ Y = p.y2 + (int64_t)pair * vv;
#pragma unroll
  for (int a = 0; a < TMI; ++a)
#pragma unroll
    for (int b = 0; b < TNI; ++b) {
      const int ga = m0 + wm * WTM + a * 4 + (lane >> 4);
      const int gb = n0 + wn * WTN + b * 16 + (lane & 15);
      if (ga < v && gb < v) Y[(int64_t)ga * v + gb] = acc[a][b];
    }
}

struct OccArgs {
  int o, v, ch, nchunks;
  const double* f_oo;
  const double* f_vv;
  const double* x1;
  const double* x2;
  double* y1;
  double* y2;  // holds the virtual part on entry
  const double* vprev1;
  const double* vprev2;
  const double* beta;
  double* partials;
  double s1;           // factor on the A_F part of the singles
  const double* done;  // when set and nonzero on entry, the launch does nothing
};

// Singles rows of A_F (f_ov-free part): 16 outputs per workgroup (its
// index among the singles workgroups is sb), 16 lanes per output, summed by
// a fixed-order butterfly. The A_F part is scaled by s1; in the Lanczos
// form the update and the shares of the three sums are added to dot, nrm,
// vv2 (weight 1).
template <bool LZ, int PER = 16>
__device__ inline void singles_part(int o, int v, const double* __restrict__ f_oo, const double* __restrict__ f_vv,
                                    const double* __restrict__ x1, double* __restrict__ y1,
                                    const double* __restrict__ vprev1, double beta, double s1, int sb, double& dot,
                                    double& nrm, double& vv2) {
  const int tid = threadIdx.x;
  const int64_t ov = (int64_t)o * v;
  const int w = tid >> 4, l = tid & 15;
  const int64_t out = (int64_t)sb * PER + w;
  double part = 0.0;
  if (out < ov) {
    const int i = (int)(out / v), a = (int)(out % v);
    for (int c = l; c < v; c += 16) part += f_vv[(int64_t)a * v + c] * x1[(int64_t)i * v + c];
    for (int k = l; k < o; k += 16) part -= f_oo[(int64_t)k * o + i] * x1[(int64_t)k * v + a];
  }
  for (int m = 8; m > 0; m >>= 1) part += __shfl_xor(part, m, 16);
  part *= s1;
  if (out < ov && l == 0) {
    if constexpr (LZ) {
      const double q = part - beta * vprev1[out];
      const double vk = x1[out];
      y1[out] = q;
      dot += vk * q;
      nrm += q * q;
      vv2 += vk * vk;
    } else {
      y1[out] = part;
    }
  }
}

// ---- packed Lanczos step, virtual part fused with the previous update ----
struct VirLzArgs {
  int v, tiles_m, tiles, units, per_xcd, vec, npair, nsw;  // nsw: workgroups for the singles
  int64_t ov;
  const double* f_vv;
  const double* P;  // p_{k-1} (raw product of the last step)
  const double* V;  // v_{k-1}
  double* Vn;       // v_k (out)
  double* Y;        // virtual part of A_F v_k (out, doubles)
  double* w1;       // w_{k-2}
  double* w2;       // w_{k-3}, overwritten with w_{k-1}
  double* x;        // MINRES iterate
  const double* partials;  // shares of <v,p>, <p,p>, <v,v> from the last occupied launch
  int nparts;
  const double* st;  // state after step k-1
  double* stn;       // state after step k (written by workgroup 0)
  double* fin;
};

// Step k of the packed symmetric solve, first launch. Every workgroup sums
// the shares of the last occupied launch (fixed order) into alpha_{k-1} =
// <v,p>/<v,v> and beta_k = ||p - alpha v|| and takes step k-1's Givens
// rotation of the tridiagonal QR and the stopping test (the work of a
// separate update launch). Each workgroup then writes, for the elements of
// its own output tile (or, for the trailing workgroups, of the singles),
// v_k = (p - alpha v_{k-1}) / beta_k and the MINRES updates w_{k-1} =
// (v_{k-1} - delta w_{k-2} - eps w_{k-3}) / rho, x += phi w_{k-1}; and
// forms y_k = f_vv v_k + v_k f_vv for its tile with v_k built while the
// panels load. The first step of a solve (flag in the state) only
// normalises: p is the start vector, v_{-1} is zero and the shares are
// (0, ||p||^2, 0). A step whose test holds skips the matrix product.
// BK >= 64 is launched only for v <= BK: each phase's contraction is then
// one panel, and the first phase's panels are read with the element batch.
template <int BM, int WGM, int BK>
__global__ __launch_bounds__(256) void fock_vir_lz_kernel(VirLzArgs p) {
  using Mma = MmaF64;
  constexpr int BN = BM;
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TMI = WTM / Mma::TM, TNI = WTN / Mma::TN;
  constexpr int ALDS = lds_elems<Mma, BM, BK>();
  constexpr int BLDS = lds_elems<Mma, BN, BK>();
  // ONE: the whole contraction (v <= BK, checked by the launcher) in one
  // panel per phase, one LDS buffer; the phase-0 panels are read before the
  // scalars are formed
  constexpr bool ONE = BK >= 64;
  constexpr int NBUF = ONE ? 1 : 2;
  __shared__ __attribute__((aligned(16))) double As[NBUF][ALDS];
  __shared__ __attribute__((aligned(16))) double Bs[NBUF][BLDS];
  __shared__ double red[3][4];

  const int tid = threadIdx.x;
  if (p.st[kLzDone] != 0.0) {
    if (blockIdx.x == 0 && tid == 0) p.stn[kLzDone] = 1.0;
    return;
  }
  const int dwg = 8 * p.per_xcd;
  const int u = (int)(blockIdx.x % 8) * p.per_xcd + (int)(blockIdx.x / 8);
  if ((int)blockIdx.x < dwg && u >= p.units) return;  // padding of the XCD grouping

  // The elements this workgroup updates: its own output tile, or for the
  // trailing workgroups 1024 singles, in batches of EB per thread. The
  // first batch's loads are issued before the scalars are formed, so both
  // latencies overlap; larger tiles stream their further batches after.
  constexpr int EB = 4;
  constexpr int NB = (BM * BN + 256 * EB - 1) / (256 * EB);
  const int v = p.v;
  const int64_t vv = (int64_t)v * v;
  const bool singles_wg = (int)blockIdx.x >= dwg;
  const int pair = singles_wg ? 0 : u / p.tiles, tile = singles_wg ? 0 : u % p.tiles;
  const int m0 = (tile % p.tiles_m) * BM;
  const int n0 = (tile / p.tiles_m) * BN;
  const int64_t off = p.ov + (int64_t)pair * vv;
  const double* __restrict__ gP = p.P;
  const double* __restrict__ gV = p.V;
  const double* __restrict__ gW1 = p.w1;
  double* __restrict__ gW2 = p.w2;
  double* __restrict__ gX = p.x;
  double* __restrict__ gVn = p.Vn;
  int64_t idx[EB];
  double ep[EB], ev[EB], e1[EB], e2[EB], ex[EB];
  auto load_batch = [&](int bt) {
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      const int q = tid + 256 * (bt * EB + j);
      idx[j] = -1;
      if (singles_wg) {
        const int64_t e = (int64_t)(blockIdx.x - dwg) * 1024 + q;
        if (q < 1024 && e < p.ov) idx[j] = e;
      } else {
        const int gm = m0 + q / BN, gn = n0 + q % BN;
        if (q < BM * BN && gm < v && gn < v) idx[j] = off + (int64_t)gm * v + gn;
      }
      ep[j] = ev[j] = e1[j] = e2[j] = ex[j] = 0.0;
      if (idx[j] >= 0) {
        ep[j] = gP[idx[j]];
        ev[j] = gV[idx[j]];
        e1[j] = gW1[idx[j]];
        e2[j] = gW2[idx[j]];
        ex[j] = gX[idx[j]];
      }
    }
  };
  load_batch(0);
  const double* __restrict__ Xp = p.P + off;
  const double* __restrict__ Xv = p.V + off;
  const double* __restrict__ F = p.f_vv;
  const bool vec = p.vec != 0;
  // phase 0 of ONE: F rows m0.. and the p, v columns n0.. (v_k is formed
  // from them once alpha and beta are known)
  Panel<Mma, double, BM, BK, true> fa;
  Panel<Mma, double, BN, BK, false> pbp, pbv;
  if constexpr (ONE) {
    if (!singles_wg) {
      fa.load(F, v, 1, m0, v, 0, v, vec, tid);
      pbp.load(Xp, 1, v, n0, v, 0, v, vec, tid);
      pbv.load(Xv, 1, v, n0, v, 0, v, vec, tid);
    }
  }

  // scalars (every workgroup, same bits)
  double r3[3] = {0.0, 0.0, 0.0};
  for (int k = tid; k < p.nparts; k += 256) {
    r3[0] += p.partials[k];
    r3[1] += p.partials[p.nparts + k];
    r3[2] += p.partials[2 * p.nparts + k];
  }
  block_sum256<3>(r3, red);
  const double vp = r3[0], pp = r3[1], vnorm2 = r3[2];
  const double alpha = vnorm2 > 0.0 ? vp / vnorm2 : 0.0;
  const double betan = sqrt(fmax(pp - alpha * vp, 0.0));
  const double invb = betan != 0.0 ? 1.0 / betan : 0.0;
  const bool first = p.st[kLzFirst] != 0.0;
  double delta = 0.0, eps = 0.0, ir = 0.0, phi = 0.0;
  bool done_now;
  if (first) {
    done_now = !(betan > p.fin[kLzFinTol]) || betan == 0.0;
    if (blockIdx.x == 0 && tid == 0) {
      for (int q = 0; q < kLzNState; ++q) p.stn[q] = 0.0;
      p.stn[kLzBeta] = betan;
      p.stn[kLzC2] = 1.0;
      p.stn[kLzC1] = 1.0;
      p.stn[kLzPhiBar] = betan;
      p.stn[kLzRes] = betan;
      p.stn[kLzDone] = done_now ? 1.0 : 0.0;
      p.fin[kLzFinRes] = betan;
      p.fin[kLzFinBeta] = betan;
    }
  } else {
    const double beta = p.st[kLzBeta];
    const double c2 = p.st[kLzC2], s2 = p.st[kLzS2], c1 = p.st[kLzC1], s1 = p.st[kLzS1];
    eps = s2 * beta;
    const double dbar = c2 * beta;
    delta = c1 * dbar + s1 * alpha;
    const double gbar = -s1 * dbar + c1 * alpha;
    const double rho1 = hypot(gbar, betan);
    const double c = rho1 != 0.0 ? gbar / rho1 : 1.0;
    const double s = rho1 != 0.0 ? betan / rho1 : 0.0;
    const double phibar = p.st[kLzPhiBar];
    phi = c * phibar;
    ir = rho1 != 0.0 ? 1.0 / rho1 : 0.0;
    const double res = fabs(s * phibar);
    done_now = res <= p.fin[kLzFinTol] || betan == 0.0;
    if (blockIdx.x == 0 && tid == 0) {
      p.stn[kLzBeta] = betan;
      p.stn[kLzAlpha] = alpha;
      p.stn[kLzBetaN] = betan;
      p.stn[kLzC2] = c1; p.stn[kLzS2] = s1;
      p.stn[kLzC1] = c; p.stn[kLzS1] = s;
      p.stn[kLzPhiBar] = -s * phibar;
      p.stn[kLzRho1] = rho1;
      p.stn[kLzDelta] = delta;
      p.stn[kLzEps] = eps;
      p.stn[kLzPhi] = phi;
      p.stn[kLzRes] = res;
      p.stn[kLzInvB] = invb;
      p.stn[kLzDone] = done_now ? 1.0 : 0.0;
      p.stn[kLzFirst] = 0.0;
      p.fin[kLzFinSteps] += 1.0;
      p.fin[kLzFinRes] = res;
      p.fin[kLzFinBeta] = betan;
    }
  }
  auto apply_batch = [&]() {
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      if (idx[j] < 0) continue;
      gVn[idx[j]] = (ep[j] - alpha * ev[j]) * invb;
      if (!first) {
        const double w = (ev[j] - delta * e1[j] - eps * e2[j]) * ir;
        gW2[idx[j]] = w;
        gX[idx[j]] = ex[j] + phi * w;
      }
    }
  };
  apply_batch();
  if (singles_wg) return;  // 1024 singles: one batch
  for (int bt = 1; bt < NB; ++bt) {
    load_batch(bt);
    apply_batch();
  }
  if (done_now) return;  // converged: y_k is not needed

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  double acc[TMI][TNI];
#pragma unroll
  for (int a = 0; a < TMI; ++a)
#pragma unroll
    for (int b = 0; b < TNI; ++b) acc[a][b] = 0.0;
  auto mma = [&](const double* Ac, const double* Bc) {
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
  };
  if constexpr (ONE) {
    // phase 0: F[m0.., :] x v_k[:, n0..]; phase 1: v_k[m0.., :] x F[:, n0..]
#pragma unroll
    for (int i = 0; i < (int)(sizeof(pbp.r) / sizeof(double)); ++i) pbp.r[i] = (pbp.r[i] - alpha * pbv.r[i]) * invb;
    fa.store(As[0], tid);
    pbp.store(Bs[0], tid);
    Panel<Mma, double, BM, BK, true> pap, pav;
    Panel<Mma, double, BN, BK, false> fb;
    pap.load(Xp, v, 1, m0, v, 0, v, vec, tid);
    pav.load(Xv, v, 1, m0, v, 0, v, vec, tid);
    fb.load(F, 1, v, n0, v, 0, v, vec, tid);
    __syncthreads();
    mma(As[0], Bs[0]);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(pap.r) / sizeof(double)); ++i) pap.r[i] = (pap.r[i] - alpha * pav.r[i]) * invb;
    __syncthreads();
    pap.store(As[0], tid);
    fb.store(Bs[0], tid);
    __syncthreads();
    mma(As[0], Bs[0]);
  } else {
    const int nkp = (v + BK - 1) / BK;
    const int nk = 2 * nkp;
    // phase 0: F[a][c] x v_k[c][b]; phase 1: v_k[a][c] x F[c][b]; the v_k
    // panel is (p - alpha v) / beta of the two loaded panels
    Panel<Mma, double, BM, BK, true> pa;
    Panel<Mma, double, BN, BK, false> pb;
    auto load = [&](int t) {
      if (t >= nkp) {
        const int k0 = (t - nkp) * BK;
        pa.load_diff(Xp, Xv, alpha, invb, v, 1, m0, v, k0, v, vec, tid);
        pb.load(F, 1, v, n0, v, k0, v, vec, tid);
      } else {
        const int k0 = t * BK;
        pa.load(F, v, 1, m0, v, k0, v, vec, tid);
        pb.load_diff(Xp, Xv, alpha, invb, 1, v, n0, v, k0, v, vec, tid);
      }
    };
    load(0);
    pa.store(As[0], tid);
    pb.store(Bs[0], tid);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) load(kt + 1);
      mma(As[cur], Bs[cur]);
      if (kt + 1 < nk) {
        pa.store(As[cur ^ 1], tid);
        pb.store(Bs[cur ^ 1], tid);
      }
      __syncthreads();
    }
  }
  double* __restrict__ Yo = p.Y + off;
#pragma unroll
  for (int a = 0; a < TMI; ++a)
#pragma unroll
    for (int b = 0; b < TNI; ++b) {
      const int ga = m0 + wm * WTM + a * 4 + (lane >> 4);
      const int gb = n0 + wn * WTN + b * 16 + (lane & 15);
      if (ga < v && gb < v) Yo[(int64_t)ga * v + gb] = acc[a][b];
    }
}

// Dynamic LDS: xs[o*o][ch] then fo[o][o].
template <bool LZ>
__global__ __launch_bounds__(256) void fock_occ_kernel(OccArgs p) {
  extern __shared__ double lds[];
  __shared__ double red[3][4];
  if (p.done && *p.done != 0.0) return;
  const int o = p.o, v = p.v, ch = p.ch;
  const int oo = o * o;
  const int64_t vv = (int64_t)v * v;
  const int tid = threadIdx.x;
  double beta = 0.0;
  if constexpr (LZ) beta = *p.beta;
  double dot = 0.0, nrm = 0.0, vv2 = 0.0;

  if ((int)blockIdx.x < p.nchunks) {
    double* xs = lds;
    double* fo = lds + (int64_t)oo * ch;
    const int64_t ab0 = (int64_t)blockIdx.x * ch;
    for (int q = tid; q < oo * ch; q += 256) {
      const int pr = q / ch, e = q % ch;
      xs[q] = ab0 + e < vv ? p.x2[(int64_t)pr * vv + ab0 + e] : 0.0;
    }
    for (int q = tid; q < oo; q += 256) fo[q] = p.f_oo[q];
    __syncthreads();
    const int e = tid % ch;
    const int groups = 256 / ch;
    if (ab0 + e < vv) {
      // four pairs per round: their global loads are issued together
      constexpr int R = 4;
      for (int pr0 = tid / ch; pr0 < oo; pr0 += R * groups) {
        double yin[R], vin[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int pr = pr0 + r * groups;
          const int64_t idx = (int64_t)(pr < oo ? pr : 0) * vv + ab0 + e;
          yin[r] = p.y2[idx];
          if constexpr (LZ) vin[r] = p.vprev2[idx];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int pr = pr0 + r * groups;
          if (pr >= oo) break;
          const int i = pr / o, j = pr % o;
          double occ = 0.0;
          for (int k = 0; k < o; ++k)
            occ += fo[k * o + i] * xs[(k * o + j) * ch + e] + fo[k * o + j] * xs[(i * o + k) * ch + e];
          const int64_t idx = (int64_t)pr * vv + ab0 + e;
          const double y = yin[r] - occ;
          if constexpr (LZ) {
            const double q = y - beta * vin[r];
            const double vk = xs[pr * ch + e];
            p.y2[idx] = q;
            dot += vk * q;
            nrm += q * q;
            vv2 += vk * vk;
          } else {
            p.y2[idx] = y;
          }
        }
      }
    }
  } else {
    singles_part<LZ>(p.o, p.v, p.f_oo, p.f_vv, p.x1, p.y1, p.vprev1, beta, p.s1, blockIdx.x - p.nchunks, dot, nrm,
                     vv2);
  }

  if constexpr (LZ) {
    double r[3] = {dot, nrm, vv2};
    block_sum256<3>(r, red);
    if (tid == 0)
      for (int c = 0; c < 3; ++c) p.partials[c * gridDim.x + blockIdx.x] = r[c];
  }
}

// Packed pair layout (pairs i <= j only, P(i, j) = i o - i (i - 1) / 2 +
// j - i, each a v x v block; x_ji = x_ij^T is implied): the occupied terms
// need x_kj for k > j, which is x_jk transposed. A workgroup therefore
// takes a tile A = [a0, a0 + t) x [b0, b0 + t) of the upper tile triangle
// together with its mirror A^T, stages both for every packed pair, and
// forms the outputs of both tiles for every packed pair from there.
struct OccPackedArgs {
  int o, v, t, ntile, nchunks, npair, psplit, dwg;  // dwg: workgroups of the doubles part (a multiple of 8)
  const double* f_oo;
  const double* f_vv;
  const double* x1;
  const double* x2;  // packed
  double* y1;
  double* y2;  // packed; holds the virtual part on entry
  const double* vprev1;
  const double* vprev2;
  const double* beta;
  double* partials;
  double s1;
  const double* done;
};

__device__ inline int packed_pair(int i, int j, int o) { return i * o - i * (i - 1) / 2 + (j - i); }  // i <= j

// Tile c (0 <= c < ntile (ntile + 1) / 2) of the upper tile triangle in
// block order: the triangle is cut into blocks of S x S tiles (S t = 16
// elements, one 128-byte line of doubles per row), taken row by row over
// the upper block triangle, and the tiles of a block (ta <= tb within a
// diagonal block) row by row. Consecutive tiles run on one XCD, so the
// lines of x2 that neighbouring tiles and their mirrors share are fetched
// into that XCD's L2 once.
__device__ inline void block_order_tile(int c, int ntile, int S, int* ta, int* tb) {
  const int nst = (ntile + S - 1) / S;
  for (int sa = 0; sa < nst; ++sa) {
    const int ra = min(S, ntile - sa * S);
    for (int sb = sa; sb < nst; ++sb) {
      const int rb = min(S, ntile - sb * S);
      const int cnt = sa == sb ? ra * (ra + 1) / 2 : ra * rb;
      if (c < cnt) {
        if (sa == sb) {
          int r = 0;
          while (c >= ra - r) {
            c -= ra - r;
            ++r;
          }
          *ta = sa * S + r;
          *tb = *ta + c;
        } else {
          *ta = sa * S + c / rb;
          *tb = sb * S + c % rb;
        }
        return;
      }
      c -= cnt;
    }
  }
  *ta = *tb = 0;  // c out of range (not reached)
}

// Dynamic LDS: xs[npair][ns] then fo[o][o]; ns = t^2 (diagonal tile) or
// 2 t^2. The first dwg workgroups do the doubles: workgroup b takes the
// unit c = (b % 8) (dwg / 8) + b / 8, i.e. tile c / psplit (in block order)
// and the packed pairs pr = c % psplit + psplit m. Workgroups are dispatched round-robin
// over the 8 XCDs, so the psplit workgroups of a tile run on one XCD and
// its staged blocks are fetched into that L2 once. Units past
// nchunks * psplit only write zero partial sums; the remaining workgroups
// compute the singles.
__global__ __launch_bounds__(256) void fock_occ_packed_kernel(OccPackedArgs p) {
  extern __shared__ double lds[];
  __shared__ double red[3][4];
  // (k, j) -> 2 P(min, max) + (k > j): where x_kj sits among the staged
  // blocks, and whether it is read through the mirror tile
  __shared__ int tab[kFockOpMaxOcc * kFockOpMaxOcc];
  __shared__ unsigned char pi_[kFockOpMaxOcc * (kFockOpMaxOcc + 1) / 2], pj_[kFockOpMaxOcc * (kFockOpMaxOcc + 1) / 2];
  if (p.done && *p.done != 0.0) return;
  const int o = p.o, v = p.v, t = p.t, npair = p.npair, ps = p.psplit;
  const int64_t vv = (int64_t)v * v;
  const int tid = threadIdx.x;
  const double beta = *p.beta;
  double dot = 0.0, nrm = 0.0, vv2 = 0.0;

  const int unit = (int)(blockIdx.x % 8) * (p.dwg / 8) + (int)(blockIdx.x / 8);
  if ((int)blockIdx.x < p.dwg && unit < p.nchunks * ps) {
    // tile (ta, tb), ta <= tb, in block order
    int ta, tb;
    block_order_tile(unit / ps, p.ntile, 16 / p.t, &ta, &tb);
    const int part = unit % ps;
    const int a0 = ta * t, b0 = tb * t, tt = t * t;
    const bool diag = ta == tb;
    const int ns = diag ? tt : 2 * tt;
    double* xs = lds;
    double* fo = lds + (int64_t)npair * ns;
    const int groups = 256 / ns;
    const int s = tid % ns, g0 = tid / ns;
    // staged element s: s < tt is (a0 + s / t, b0 + s % t) of A, else
    // (b0 + r / t, a0 + r % t), r = s - tt, of A^T
    const int r = s < tt ? s : s - tt;
    const int a = (s < tt ? a0 : b0) + r / t, b = (s < tt ? b0 : a0) + r % t;
    const int sT = diag ? (r % t) * t + r / t : (s < tt ? tt : 0) + (r % t) * t + r / t;
    const bool active = g0 < groups && a < v && b < v;
    const int64_t e = active ? (int64_t)a * v + b : 0;
    // this thread's outputs: pairs part + ps (g0 + groups m), m = 0, 1, ...
    const int stride = ps * groups;
    constexpr int R = 4;
    double yin[R], vin[R];
    auto fetch = [&](int pr0) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int pr = pr0 + u * stride;
        const int64_t idx = (int64_t)(pr < npair ? pr : 0) * vv + e;
        yin[u] = p.y2[idx];
        vin[u] = p.vprev2[idx];
      }
    };
    const int first = part + ps * g0;
    if (active) fetch(first);  // in flight during the staging
    {
      // ns divides 256 (ns = t^2 or 2 t^2, t in {2, 4, 8}), so this thread
      // stages the same tile element s of packed pairs g0, g0 + 256 / ns, ...
      const bool inb = a < v && b < v;
      const double* src = p.x2 + (int64_t)g0 * vv + (int64_t)a * v + b;
      const int64_t step = (int64_t)groups * vv;
      for (int pr = g0; pr < npair; pr += groups, src += step) {
        double x = 0.0;
        if (inb) x = *src;
        xs[pr * ns + s] = x;
      }
    }
    for (int q = tid; q < o * o; q += 256) {
      fo[q] = p.f_oo[q];
      const int k = q / o, j = q % o;
      tab[q] = 2 * (k <= j ? packed_pair(k, j, o) : packed_pair(j, k, o)) + (k > j ? 1 : 0);
      if (k <= j) {
        pi_[packed_pair(k, j, o)] = (unsigned char)k;
        pj_[packed_pair(k, j, o)] = (unsigned char)j;
      }
    }
    __syncthreads();
    if (active) {
      for (int pr0 = first; pr0 < npair; pr0 += R * stride) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int pr = pr0 + u * stride;
          if (pr >= npair) break;
          const int i = pi_[pr], j = pj_[pr];
          double occ = 0.0;
          for (int k = 0; k < o; ++k) {
            const int t1 = tab[k * o + j], t2 = tab[i * o + k];
            const double xkj = xs[(t1 >> 1) * ns + ((t1 & 1) ? sT : s)];
            const double xik = xs[(t2 >> 1) * ns + ((t2 & 1) ? sT : s)];
            occ += fo[k * o + i] * xkj + fo[k * o + j] * xik;
          }
          const double q = (yin[u] - occ) - beta * vin[u];
          const double vk = xs[pr * ns + s];
          const double w = i == j ? 1.0 : 2.0;  // x_ij and x_ji = x_ij^T both count
          p.y2[(int64_t)pr * vv + e] = q;
          dot += w * vk * q;
          nrm += w * q * q;
          vv2 += w * vk * vk;
        }
        if (pr0 + R * stride < npair) fetch(pr0 + R * stride);
      }
    }
  } else if ((int)blockIdx.x >= p.dwg) {
    singles_part<true>(p.o, p.v, p.f_oo, p.f_vv, p.x1, p.y1, p.vprev1, beta, p.s1, blockIdx.x - p.dwg, dot, nrm,
                       vv2);
  }

  double rr[3] = {dot, nrm, vv2};
  block_sum256<3>(rr, red);
  if (tid == 0)
    for (int c = 0; c < 3; ++c) p.partials[c * gridDim.x + blockIdx.x] = rr[c];
}

// Register-blocked form of the packed occupied part. For one (a, b)
// position e, the occupied terms are Y^e = -(F^T M^e + M^e F) with M^e the
// o x o matrix M^e_ij = x_ij^ab, whose lower triangle the packed layout
// keeps at the transposed position: M^e_ij = x_ji^ba for i > j. A workgroup
// takes a set of 64 positions closed under transposition, one per lane
// (occ_set_lane), stages x at them for every packed pair in LDS
// (xs[pair][lane]), and each wave forms 4 x 4 blocks (I, J), I <= J, of the
// upper triangle of Y^e for its lane's e: per k it reads M^e_kJ and M^e_Ik
// (8 LDS reads, the lane or its transposed lane depending on k <= j) and
// f_kI, f_kJ (4 broadcast LDS reads) for 32 fused multiply-adds.
struct OccSetArgs {
  int o, v, npair, nb, units, bsplit, nblk, dwg;
  const double* f_oo;
  const double* f_vv;
  const double* x1;
  const double* x2;  // packed
  double* y1;
  double* y2;  // packed; holds the virtual part on entry
  const double* vprev1;
  const double* vprev2;
  const double* beta;
  double* partials;
  double s1;
  const double* done;
};

// With nb odd, the blocks of the last row and column are the second half
// of a 2 x 2 group. When the v x v grid ends at most 4 elements into that
// last block (edge), the set of an off-diagonal block pair (Ta, nb - 1) is
// instead the 4 valid rows 8 (nb - 1) .. + 4 by the 8 columns of block Ta
// together with its transpose (all 64 positions in range, one set in place
// of two half-empty ones): at v = 180, 507 sets in place of 529, which two
// rounds of one workgroup per compute unit cover.
__host__ __device__ inline bool occ_set_edge(int v, int nb) { return (nb & 1) && v - 8 * (nb - 1) <= 4; }
__host__ __device__ inline int occ_set_count(int v, int nb) { return nb * nb - (occ_set_edge(v, nb) ? nb - 1 : 0); }

// Position set u (0 <= u < occ_set_count(v, nb)) over the 8 x 8 blocks of
// the v x v grid (nb = ceil(v / 8) per side): a diagonal block (T, T), or
// half h of an off-diagonal block pair (Ta < Tb): rows 8 Ta + 4 h .. + 4 by
// columns 8 Tb .. + 8 together with its transpose (the edge sets above
// aside). The blocks are taken in 2 x 2 groups (16 x 16 elements: two
// 128-byte lines of doubles per row), the upper group triangle row by row,
// so that the sets of a group, which share the lines they touch, run one
// after another on one XCD. A diagonal group holds 4 sets: (2g, 2g), (2g,
// 2g + 1) halves 0 and 1, (2g + 1, 2g + 1); an off-diagonal one 8: w = 4
// dTa + 2 dTb + h; with nb odd the last diagonal group holds 1 and the last
// column's groups 4 (dTb = 0; w = 2 dTa + h), or 2 edge sets (w = dTa).
__host__ __device__ inline bool occ_set_decode(int u, int nb, bool edge, bool* diag, int* a0, int* b0) {
  const int ng = (nb + 1) / 2;
  const bool odd = nb & 1;
  const int nhalf = edge ? 2 : 4;  // sets of a group in the last column (nb odd)
  for (int ga = 0; ga < ng; ++ga) {
    const int cd = odd && ga == ng - 1 ? 1 : 4, noff = ng - 1 - ga;
    const int row = cd + 8 * noff - (odd && noff > 0 ? 8 - nhalf : 0);
    if (u >= row) {
      u -= row;
      continue;
    }
    const int T = 2 * ga;
    if (u < cd) {
      *diag = u == 0 || u == 3;
      *a0 = *diag ? 8 * (T + (u == 3 ? 1 : 0)) : 8 * T + 4 * (u - 1);
      *b0 = *diag ? *a0 : 8 * (T + 1);
      return true;
    }
    u -= cd;
    const int gb = ga + 1 + u / 8, w = u % 8;
    const bool half = odd && gb == ng - 1;
    *diag = false;
    if (half && edge) {
      *a0 = 8 * (nb - 1);
      *b0 = 8 * (T + w);
      return true;
    }
    const int dTa = half ? w >> 1 : w >> 2, dTb = half ? 0 : (w >> 1) & 1, h = w & 1;
    *a0 = 8 * (T + dTa) + 4 * h;
    *b0 = 8 * (2 * gb + dTb);
    return true;
  }
  return false;  // u out of range
}

// Lane l's position (a, b) in the set, and the lane lT holding (b, a).
__host__ __device__ inline void occ_set_lane(bool diag, int l, int a0, int b0, int* a, int* b, int* lT) {
  if (diag) {
    const int r = l >> 3, c = l & 7;
    *a = a0 + r;
    *b = a0 + c;
    *lT = 8 * c + r;
  } else if (l < 32) {
    const int r = l >> 3, c = l & 7;
    *a = a0 + r;
    *b = b0 + c;
    *lT = 32 + 4 * c + r;
  } else {
    const int m = l - 32, r = m >> 2, c = m & 3;
    *a = b0 + r;
    *b = a0 + c;
    *lT = 8 * c + r;
  }
}

// One k of the 4 x 4 block (I0, J0) of Y^e: acc_ij += f_ki M_kj + M_ik
// f_kj. M_kj is read from pair (k, j) at the lane's own position when k <=
// j, else from pair (j, k) at the transposed one; M_ik from pair (i, k) at
// its own position when i <= k, else from pair (k, i) transposed. With the
// packed index P(a, b) = R(a) + b, R(a) = a o - a (a - 1) / 2 - a, the
// four reads of a term are R(k) + J0 + q (one address, immediate offsets)
// or R(J0 + q) + k (and likewise with I0). T1 / T2 give the form of the two
// terms for the whole block: 0 own position, 1 transposed, 2 split at k =
// J0 + D (M_kj transposed for q < D) or k = I0 + D (M_ik own for q <= D).
// Own-form reads of M_kj at j = J0 + q >= o, and transposed-form reads of
// M_ik at i >= o, land up to three pairs past the last one (outputs that are
// not written; the staging area is padded for them).
template <int T1, int T2, int D, bool FENCE>
__device__ inline void occ_kstep(int k, int o, int I0, int J0, const double* xl, const double* xt, const double* fs,
                                 int ldf, double (&acc)[4][4]) {
  if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
  const double2 fi01 = *reinterpret_cast<const double2*>(fs + k * ldf + I0);
  const double2 fi23 = *reinterpret_cast<const double2*>(fs + k * ldf + I0 + 2);
  const double2 fj01 = *reinterpret_cast<const double2*>(fs + k * ldf + J0);
  const double2 fj23 = *reinterpret_cast<const double2*>(fs + k * ldf + J0 + 2);
  const double fi[4] = {fi01.x, fi01.y, fi23.x, fi23.y};
  const double fj[4] = {fj01.x, fj01.y, fj23.x, fj23.y};
  auto R = [o](int a) { return a * o - a * (a - 1) / 2 - a; };
  double mkj[4], mik[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (T1 == 1 || (T1 == 2 && q < D)) mkj[q] = xt[(R(J0 + q) + k) * 64];
    else mkj[q] = xl[(R(k) + J0 + q) * 64];
    if (T2 == 0 || (T2 == 2 && q <= D)) mik[q] = xl[(R(I0 + q) + k) * 64];
    else mik[q] = xt[(R(k) + I0 + q) * 64];
  }
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      acc[ii][jj] = fma(fi[ii], mkj[jj], acc[ii][jj]);
      acc[ii][jj] = fma(mik[ii], fj[jj], acc[ii][jj]);
    }
}

// The block's sum over k = 0 .. o - 1 in ranges of one read form each
// (diagonal blocks: I0 = J0). FENCE keeps the scheduler from hoisting the
// reads of later steps above earlier ones (register budget of 16-wave
// workgroups).
template <bool FENCE>
__device__ inline void occ_block(int o, int I0, int J0, const double* xl, const double* xt, const double* fs, int ldf,
                                 double (&acc)[4][4]) {
  int k = 0;
  for (; k < I0; ++k) occ_kstep<0, 1, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
  if (I0 == J0) {
    occ_kstep<2, 2, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 1 < o) occ_kstep<2, 2, 1, FENCE>(k + 1, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 2 < o) occ_kstep<2, 2, 2, FENCE>(k + 2, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 3 < o) occ_kstep<2, 2, 3, FENCE>(k + 3, o, I0, J0, xl, xt, fs, ldf, acc);
  } else {
    // k in [I0, I0 + 4) < J0 <= o - 1
    occ_kstep<0, 2, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
    occ_kstep<0, 2, 1, FENCE>(k + 1, o, I0, J0, xl, xt, fs, ldf, acc);
    occ_kstep<0, 2, 2, FENCE>(k + 2, o, I0, J0, xl, xt, fs, ldf, acc);
    occ_kstep<0, 2, 3, FENCE>(k + 3, o, I0, J0, xl, xt, fs, ldf, acc);
    for (k = I0 + 4; k < J0; ++k) occ_kstep<0, 0, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
    occ_kstep<2, 0, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 1 < o) occ_kstep<2, 0, 1, FENCE>(k + 1, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 2 < o) occ_kstep<2, 0, 2, FENCE>(k + 2, o, I0, J0, xl, xt, fs, ldf, acc);
    if (k + 3 < o) occ_kstep<2, 0, 3, FENCE>(k + 3, o, I0, J0, xl, xt, fs, ldf, acc);
  }
  for (k = J0 + 4; k < o; ++k) occ_kstep<1, 0, 0, FENCE>(k, o, I0, J0, xl, xt, fs, ldf, acc);
}

// Dynamic LDS: xs[npair + 3][64] (the last three rows only padding), then
// f_oo with rows padded to ldf = 4 ceil(o / 4) (zeros past o). NW waves per
// workgroup. Workgroup bid < dwg takes the unit u = (bid % 8) (dwg / 8) +
// bid / 8: position set u / bsplit, and of the nblk blocks of the upper
// block triangle those with index part NW + wave + NW bsplit m (part = u %
// bsplit). Units past units * bsplit only write zero partial sums; the
// remaining workgroups compute the singles, 4 NW outputs each.
template <int NW>
__global__ __launch_bounds__(64 * NW) void fock_occ_set_kernel(OccSetArgs p) {
  extern __shared__ __attribute__((aligned(16))) double xs[];
  __shared__ double red[3][NW];
  if (p.done && *p.done != 0.0) return;
  const int o = p.o, v = p.v, npair = p.npair;
  const int64_t vv = (int64_t)v * v;
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double beta = *p.beta;
  double dot = 0.0, nrm = 0.0, vv2 = 0.0;

  const int unit = (int)(blockIdx.x % 8) * (p.dwg / 8) + (int)(blockIdx.x / 8);
  bool diag = false;
  int a0 = 0, b0 = 0;
  if ((int)blockIdx.x < p.dwg && unit < p.units * p.bsplit &&
      occ_set_decode(unit / p.bsplit, p.nb, occ_set_edge(v, p.nb), &diag, &a0, &b0)) {
    int a, b, lT;
    occ_set_lane(diag, l, a0, b0, &a, &b, &lT);
    const int part = unit % p.bsplit;
    const bool valid = a < v && b < v;
    const int64_t e = valid ? (int64_t)a * v + b : 0;  // (invalid lanes read position 0 and discard it)
    const int bg = (o + 3) / 4, ldf = 4 * bg;
    double* fs = xs + (int64_t)(npair + 3) * 64;
    const int step = NW * p.bsplit;
    // PRE: the y and vprev elements of a wave's block of outputs are read
    // before its contractions (their latency hidden behind them) and kept
    // as pre = y - beta vprev; 16-wave workgroups (128 registers) read them
    // after the contractions instead. Outputs with i > j, i >= o or j >= o
    // are not written: a valid element is read in their place.
    constexpr bool PRE = NW < 16;
    double pre[4][4];
    auto block_of = [&](int blk, int* I0, int* J0) {
      int bi = 0, rem = blk;
      while (rem >= bg - bi) {
        rem -= bg - bi;
        ++bi;
      }
      *I0 = 4 * bi;
      *J0 = 4 * (bi + rem);
    };
    auto read_pre = [&](int I0, int J0) {
      double yin[4][4], vin[4][4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = min(I0 + ii, o - 1), j = max(min(J0 + jj, o - 1), i);
          const int64_t idx = (int64_t)(i * o - i * (i - 1) / 2 + (j - i)) * vv + e;
          yin[ii][jj] = p.y2[idx];
          vin[ii][jj] = p.vprev2[idx];
        }
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) pre[ii][jj] = yin[ii][jj] - beta * vin[ii][jj];
    };
    int blk = part * NW + wave;
    {
      // wave w stages pairs w, w + NW, ..., 16 loads in flight per lane
      // (clamped to the last pair), and f_oo; the first batch is issued
      // before the reads of the wave's first block of outputs
      const double* src = p.x2 + e;
      const int nf = o * ldf;
      const double fv = tid < nf && tid % ldf < o ? p.f_oo[(tid / ldf) * o + tid % ldf] : 0.0;
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = src[(int64_t)min(wave + NW * u, npair - 1) * vv];
      if constexpr (PRE) {
        int I0 = 0, J0 = 0;
        if (blk < p.nblk) block_of(blk, &I0, &J0);
        read_pre(I0, J0);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (wave + NW * u < npair) xs[(wave + NW * u) * 64 + l] = valid ? t[u] : 0.0;
      if (tid < nf) fs[tid] = fv;
      for (int pr0 = wave + 16 * NW; pr0 < npair; pr0 += 16 * NW) {
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = src[(int64_t)min(pr0 + NW * u, npair - 1) * vv];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (pr0 + NW * u < npair) xs[(pr0 + NW * u) * 64 + l] = valid ? t[u] : 0.0;
      }
      for (int q = tid + 64 * NW; q < nf; q += 64 * NW) {
        const int k = q / ldf, i = q % ldf;
        fs[q] = i < o ? p.f_oo[k * o + i] : 0.0;
      }
    }
    __syncthreads();
    const double* xl = xs + l;
    const double* xt = xs + lT;
    for (; blk < p.nblk; blk += step) {
      int I0, J0;
      block_of(blk, &I0, &J0);
      double acc[4][4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = 0.0;
      occ_block<NW == 16>(o, I0, J0, xl, xt, fs, ldf, acc);
      if constexpr (!PRE) read_pre(I0, J0);
      // outputs i <= j < o of valid positions; the sums weight the other
      // (padded) outputs by 0 and the blocks of pairs i < j by 2 (x_ij and
      // x_ji = x_ij^T both count)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = I0 + ii, j = J0 + jj;
          const bool out = i < o && j < o && i <= j;  // wave-uniform
          if (!out) continue;
          const int pr = i * o - i * (i - 1) / 2 + (j - i);
          const double q = pre[ii][jj] - acc[ii][jj];
          const double vk = xl[pr * 64];
          const double w = !valid ? 0.0 : (i == j ? 1.0 : 2.0);
          if (valid) p.y2[(int64_t)pr * vv + e] = q;
          dot += w * vk * q;
          nrm += w * q * q;
          vv2 += w * vk * vk;
        }
      if constexpr (PRE) {
        if (blk + step < p.nblk) {
          int I1, J1;
          block_of(blk + step, &I1, &J1);
          read_pre(I1, J1);
        }
      }
    }
  } else if ((int)blockIdx.x >= p.dwg) {
    singles_part<true, 4 * NW>(p.o, p.v, p.f_oo, p.f_vv, p.x1, p.y1, p.vprev1, beta, p.s1, blockIdx.x - p.dwg, dot,
                               nrm, vv2);
  }

  double rr[3] = {dot, nrm, vv2};
  block_sum_waves<3, NW>(rr, red);
  if (tid == 0)
    for (int c = 0; c < 3; ++c) p.partials[c * gridDim.x + blockIdx.x] = rr[c];
}

bool aligned16(const void* q) { return ((uintptr_t)q & 15u) == 0; }

// npairs: o^2 for the full layout, o (o + 1) / 2 for the packed one (the
// kernel only walks the v x v blocks one after another)
void launch_vir(const FockOp& op, int npairs, const double* x2, double* y2, const double* done, hipStream_t s) {
  VirArgs a;
  a.v = op.v;
  a.tiles_m = (int)ceil_div(op.v, op.bm);
  a.tiles = op.tiles;
  a.units = op.tiles * npairs;
  a.per_xcd = (int)ceil_div(a.units, 8);
  a.vec = (op.v % 2 == 0 && aligned16(x2) && aligned16(op.f_vv)) ? 1 : 0;
  a.f_vv = op.f_vv;
  a.x2 = x2;
  a.y2 = y2;
  a.done = done;
  dim3 grid((unsigned)(8 * a.per_xcd));
  // contraction panels of 32 for the 32-wide blocks when that pads v no
  // more than panels of 16 (measured: the wider blocks run better with 16)
  const bool bk32 = op.bm == 32 && ceil_div(op.v, 32) * 32 <= ceil_div(op.v, 16) * 16;
  switch (op.bm * 2 + (bk32 ? 1 : 0)) {
    case 64: fock_vir_kernel<32, 2, 16><<<grid, 256, 0, s>>>(a); break;
    case 65: fock_vir_kernel<32, 2, 32><<<grid, 256, 0, s>>>(a); break;
    case 96: fock_vir_kernel<48, 4, 16><<<grid, 256, 0, s>>>(a); break;
    case 97: fock_vir_kernel<48, 4, 32><<<grid, 256, 0, s>>>(a); break;
    case 128: fock_vir_kernel<64, 2, 16><<<grid, 256, 0, s>>>(a); break;
    default: fock_vir_kernel<64, 2, 32><<<grid, 256, 0, s>>>(a); break;
  }
  PNK_CHECK_LAUNCH();
}

size_t occ_lds_bytes(int o, int ch) { return sizeof(double) * ((size_t)o * o * ch + (size_t)o * o); }

template <bool LZ>
void launch_occ(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, const double* vprev1,
                const double* vprev2, const double* beta, double* partials, double s1, const double* done,
                hipStream_t s) {
  OccArgs a;
  a.o = op.o;
  a.v = op.v;
  a.ch = op.ch;
  a.nchunks = op.nchunks;
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
  a.s1 = s1;
  a.done = done;
  fock_occ_kernel<LZ><<<(unsigned)op.nparts(), 256, occ_lds_bytes(op.o, op.ch), s>>>(a);
  PNK_CHECK_LAUNCH();
}

size_t occ_set_lds_bytes(int o) {
  const size_t npair = (size_t)o * (o + 1) / 2, ldf = 4 * (size_t)((o + 3) / 4);
  return sizeof(double) * (64 * (npair + 3) + (size_t)o * ldf);
}

// Dynamic LDS a workgroup of the register-blocked occupied kernel may use:
// the device's per-workgroup maximum, opted into for that kernel (0 when
// the opt-in fails).
size_t occ_set_lds_limit() {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const size_t avail = (size_t)lim > 2048 ? (size_t)lim - 2048 : 0;  // the kernel's static reduction buffer
  const void* k[3] = {reinterpret_cast<const void*>(&fock_occ_set_kernel<4>),
                      reinterpret_cast<const void*>(&fock_occ_set_kernel<8>),
                      reinterpret_cast<const void*>(&fock_occ_set_kernel<16>)};
  for (const void* f : k)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)avail) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
  return avail;
}

}  // namespace

// Virtual kernel: the block edge among 32 / 48 / 64 that wastes the fewest
// padded outputs (v^2 / (tiles * bm^2)); among near-ties the largest edge
// that still gives at least 512 workgroups (two per CU), else the smallest.
// Occupied kernel: the widest chunk (64 .. 16 elements, 8 only when 16 does
// not fit) whose LDS stays within 64 KB (two workgroups per CU) and that
// still gives 512 workgroups.
int fock_op_set_positions(int v, int* a, int* b, int* lt, int64_t cap) {
  if (v < 1 || !a || !b || !lt) return -1;
  const int nb = (v + 7) / 8, n = occ_set_count(v, nb);
  if ((int64_t)n * 64 > cap) return -1;
  const bool edge = occ_set_edge(v, nb);
  for (int u = 0; u < n; ++u) {
    bool diag = false;
    int a0 = 0, b0 = 0;
    if (!occ_set_decode(u, nb, edge, &diag, &a0, &b0)) return -1;
    for (int l = 0; l < 64; ++l) occ_set_lane(diag, l, a0, b0, &a[u * 64 + l], &b[u * 64 + l], &lt[u * 64 + l]);
  }
  return n;
}

bool fock_op_plan(FockOp& op) {
  if (op.o < 1 || op.v < 1 || op.o > kFockOpMaxOcc) return false;
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

  const int64_t vv = (int64_t)op.v * op.v;
  // (at least 16 elements: a full 128-byte line per pair and chunk)
  op.ch = 0;
  for (int ch : {64, 32, 16, 8}) {
    if (occ_lds_bytes(op.o, ch) > 64 * 1024) continue;
    if (op.ch == 0) op.ch = ch;  // widest that fits, whatever the count
    if (ceil_div(vv, ch) >= 512 || ch == 16) { op.ch = ch; break; }
  }
  if (op.ch == 0) return false;
  op.nchunks = (int)ceil_div(vv, op.ch);
  op.nsingles = (int)ceil_div((int64_t)op.o * op.v, 16);
  // packed layout: tile edge 2 with the pairs unsplit when that gives 1024
  // to 8192 chunks; otherwise the widest tile edge among 8 / 4 / 2 whose
  // staging (two tiles per packed pair) stays within 64 KB and that gives at
  // least 256 chunks, else the widest that fits
  op.npair = op.o * (op.o + 1) / 2;
  op.pt = 0;
  // edge 2 unsplit when that alone gives 1024 chunks: measured per inner
  // product, 2.7 % faster than the rule below at o=10/v=90, 1 % at
  // o=16/v=144 and 8 % at o=20/v=180
  const int64_t nt2 = ceil_div(op.v, 2);
  const bool small_tiles = nt2 * (nt2 + 1) / 2 >= 1024 && nt2 * (nt2 + 1) / 2 <= 8192 &&
                           sizeof(double) * ((size_t)op.npair * 2 * 4 + (size_t)op.o * op.o) <= 64 * 1024;
  if (small_tiles) op.pt = 2;
  for (int tt : {8, 4, 2}) {
    if (small_tiles) break;
    const size_t lds = sizeof(double) * ((size_t)op.npair * 2 * tt * tt + (size_t)op.o * op.o);
    if (lds > 64 * 1024) continue;
    const int64_t nt = ceil_div(op.v, tt);
    if (op.pt == 0) op.pt = tt;
    if (nt * (nt + 1) / 2 >= 256) { op.pt = tt; break; }
  }
  if (op.pt > 0) {
    op.psingles = op.nsingles;
    op.pntile = (int)ceil_div(op.v, op.pt);
    op.pnchunks = op.pntile * (op.pntile + 1) / 2;
    // split the packed pairs of a tile over up to 4 workgroups (each stages
    // the whole tile) until there are about 1024 of them: the kernel is
    // bound by latency, which more resident waves hide
    op.psplit = 1;
    while (!small_tiles && op.psplit < 4 && (int64_t)op.pnchunks * op.psplit < 1024 && op.npair >= 8 * 2 * op.psplit)
      ++op.psplit;
    op.pdwg = (int)(8 * ceil_div((int64_t)op.pnchunks * op.psplit, 8));
    // the register-blocked form when 64 positions of every packed pair fit
    // in LDS (o <= 24 with 160 KB per workgroup): split each set's output
    // blocks over more workgroups while there are fewer than 512 and every
    // workgroup still gets a block
    const size_t set_lds = occ_set_lds_bytes(op.o), lds_limit = occ_set_lds_limit();
    if (set_lds <= lds_limit) {
      op.psets = 1;
      op.pnb = (int)ceil_div(op.v, 8);
      const int bg = (op.o + 3) / 4;
      op.pnblk = bg * (bg + 1) / 2;
      const int64_t units = occ_set_count(op.v, op.pnb);
      // waves per workgroup: 16 where the staging fills a CU's LDS (taken
      // as the per-workgroup maximum), else 8 when there are more than 4
      // blocks (measured at o=10/v=90: 2.5 % faster than 4 waves with the
      // blocks split over two workgroups), else 4
      const int per_cu = (int)((lds_limit + 2048) / set_lds);
      op.pnw = per_cu < 2 ? 16 : (op.pnblk > 4 ? 8 : 4);
      while (op.pnw > 4 && op.pnblk <= op.pnw / 2) op.pnw /= 2;
      op.pbsplit = 1;
      while (units * op.pbsplit < 512 && op.pnblk > op.pnw * op.pbsplit) ++op.pbsplit;
      op.pdwg = (int)(8 * ceil_div(units * op.pbsplit, 8));
      op.psingles = (int)ceil_div((int64_t)op.o * op.v, 4 * op.pnw);
    }
  }
  return (int64_t)op.tiles * op.o * op.o < (1ll << 31) - 8 && op.nparts() <= 0x7fffffff;
}

bool fock_op_fused_step(const FockOp& op) { return op.pt > 0 && op.bm == 32; }

bool fock_op_is_timed_lanczos_kernel(const void* func, bool fused) {
  if (!fused)
    return func == reinterpret_cast<const void*>(&fock_occ_kernel<true>) ||
           func == reinterpret_cast<const void*>(&fock_occ_packed_kernel) ||
           func == reinterpret_cast<const void*>(&fock_occ_set_kernel<4>) ||
           func == reinterpret_cast<const void*>(&fock_occ_set_kernel<8>) ||
           func == reinterpret_cast<const void*>(&fock_occ_set_kernel<16>);
  const void* timed[] = {reinterpret_cast<const void*>(&fock_vir_lz_kernel<32, 2, 16>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<32, 2, 32>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<32, 2, 64>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<32, 2, 96>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<48, 4, 16>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<48, 4, 32>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<64, 2, 16>),
                         reinterpret_cast<const void*>(&fock_vir_lz_kernel<64, 2, 32>)};
  for (const void* k : timed)
    if (func == k) return true;
  return false;
}

void fock_op_apply(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0, "fock_op: not planned");
  PNK_REQUIRE(x1 != y1 && x2 != y2, "fock_op: output must not alias the input");
  launch_vir(op, op.o * op.o, x2, y2, nullptr, s);
  launch_occ<false>(op, x1, x2, y1, y2, nullptr, nullptr, nullptr, nullptr, 1.0, nullptr, s);
}

void fock_op_lanczos_vir(const FockOp& op, const double* v, double* p, const double* done, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0, "fock_op: not planned");
  PNK_REQUIRE(v != p, "fock_op: output must not alias the input");
  const int64_t ov = (int64_t)op.o * op.v;
  launch_vir(op, op.o * op.o, v + ov, p + ov, done, s);
}

void fock_op_lanczos_occ(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                         double* partials, double singles_scale, const double* done, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0, "fock_op: not planned");
  PNK_REQUIRE(v != p, "fock_op: output must not alias the input");
  const int64_t ov = (int64_t)op.o * op.v;
  launch_occ<true>(op, v, v + ov, p, p + ov, vprev, vprev + ov, beta, partials, singles_scale, done, s);
}

void fock_op_lanczos_vir_packed(const FockOp& op, const double* v, double* p, const double* done, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0 && op.pt > 0, "fock_op: packed form not planned");
  PNK_REQUIRE(v != p, "fock_op: output must not alias the input");
  const int64_t ov = (int64_t)op.o * op.v;
  launch_vir(op, op.npair, v + ov, p + ov, done, s);
}

void fock_op_lanczos_vir_fused(const FockOp& op, const double* P, const double* V, double* Vn, double* Y, double* w1,
                               double* w2, double* x, const double* partials, int nparts, const double* st,
                               double* stn, double* fin, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0 && op.pt > 0, "fock_op: packed form not planned");
  PNK_REQUIRE(Vn != P && Vn != V && Y != P && Y != V && Y != Vn, "fock_op: fused step buffers must be distinct");
  VirLzArgs a;
  a.v = op.v;
  a.tiles_m = (int)ceil_div(op.v, op.bm);
  a.tiles = op.tiles;
  a.units = op.tiles * op.npair;
  a.per_xcd = (int)ceil_div(a.units, 8);
  a.npair = op.npair;
  a.ov = (int64_t)op.o * op.v;
  a.nsw = (int)ceil_div(a.ov, 1024);
  a.vec = (op.v % 2 == 0 && aligned16(P) && aligned16(V) && aligned16(op.f_vv)) ? 1 : 0;
  a.f_vv = op.f_vv;
  a.P = P;
  a.V = V;
  a.Vn = Vn;
  a.Y = Y;
  a.w1 = w1;
  a.w2 = w2;
  a.x = x;
  a.partials = partials;
  a.nparts = nparts;
  a.st = st;
  a.stn = stn;
  a.fin = fin;
  dim3 grid((unsigned)(8 * a.per_xcd + a.nsw));
  // 32 < v <= 96 on 32-wide blocks: the whole contraction in one panel per
  // phase (two dependent panel reads per workgroup instead of up to six)
  if (op.bm == 32 && op.v > 32 && op.v <= 96) {  // v <= BK, as the one-panel form needs
    if (op.v <= 64) fock_vir_lz_kernel<32, 2, 64><<<grid, 256, 0, s>>>(a);
    else fock_vir_lz_kernel<32, 2, 96><<<grid, 256, 0, s>>>(a);
    PNK_CHECK_LAUNCH();
    return;
  }
  const bool bk32 = op.bm == 32 && ceil_div(op.v, 32) * 32 <= ceil_div(op.v, 16) * 16;
  switch (op.bm * 2 + (bk32 ? 1 : 0)) {
    case 64: fock_vir_lz_kernel<32, 2, 16><<<grid, 256, 0, s>>>(a); break;
    case 65: fock_vir_lz_kernel<32, 2, 32><<<grid, 256, 0, s>>>(a); break;
    case 96: fock_vir_lz_kernel<48, 4, 16><<<grid, 256, 0, s>>>(a); break;
    case 97: fock_vir_lz_kernel<48, 4, 32><<<grid, 256, 0, s>>>(a); break;
    case 128: fock_vir_lz_kernel<64, 2, 16><<<grid, 256, 0, s>>>(a); break;
    default: fock_vir_lz_kernel<64, 2, 32><<<grid, 256, 0, s>>>(a); break;
  }
  PNK_CHECK_LAUNCH();
}

void fock_op_lanczos_occ_packed(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                                double* partials, double singles_scale, const double* done, hipStream_t s) {
  PNK_REQUIRE(op.bm > 0 && op.pt > 0, "fock_op: packed form not planned");
  PNK_REQUIRE(v != p, "fock_op: output must not alias the input");
  const int64_t ov = (int64_t)op.o * op.v;
  OccPackedArgs a;
  a.o = op.o;
  a.v = op.v;
  a.t = op.pt;
  a.ntile = op.pntile;
  a.nchunks = op.pnchunks;
  a.npair = op.npair;
  a.psplit = op.psplit;
  a.dwg = op.pdwg;
  a.f_oo = op.f_oo;
  a.f_vv = op.f_vv;
  a.x1 = v;
  a.x2 = v + ov;
  a.y1 = p;
  a.y2 = p + ov;
  a.vprev1 = vprev;
  a.vprev2 = vprev + ov;
  a.beta = beta;
  a.partials = partials;
  a.s1 = singles_scale;
  a.done = done;
  if (op.psets) {
    OccSetArgs c;
    c.o = op.o;
    c.v = op.v;
    c.npair = op.npair;
    c.nb = op.pnb;
    c.units = occ_set_count(op.v, op.pnb);
    c.bsplit = op.pbsplit;
    c.nblk = op.pnblk;
    c.dwg = op.pdwg;
    c.f_oo = op.f_oo;
    c.f_vv = op.f_vv;
    c.x1 = a.x1;
    c.x2 = a.x2;
    c.y1 = a.y1;
    c.y2 = a.y2;
    c.vprev1 = a.vprev1;
    c.vprev2 = a.vprev2;
    c.beta = beta;
    c.partials = partials;
    c.s1 = singles_scale;
    c.done = done;
    const unsigned grid = (unsigned)op.nparts_packed();
    const size_t lds = occ_set_lds_bytes(op.o);
    switch (op.pnw) {
      case 4: fock_occ_set_kernel<4><<<grid, 256, lds, s>>>(c); break;
      case 8: fock_occ_set_kernel<8><<<grid, 512, lds, s>>>(c); break;
      default: fock_occ_set_kernel<16><<<grid, 1024, lds, s>>>(c); break;
    }
    PNK_CHECK_LAUNCH();
    return;
  }
  const size_t lds = sizeof(double) * ((size_t)op.npair * 2 * op.pt * op.pt + (size_t)op.o * op.o);
  fock_occ_packed_kernel<<<(unsigned)op.nparts_packed(), 256, lds, s>>>(a);
  PNK_CHECK_LAUNCH();
}

}  // namespace pnk
