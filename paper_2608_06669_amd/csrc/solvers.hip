// PNK (Appendix F algorithm with Eisenstat-Walker forcing) and FP+DIIS.
//
// All vectors live on the device in the packed layout [t1 (o*v) | t2
// (o*o*v*v)]. The outer Newton residual, the energy, the Arnoldi
// orthogonalisation, the Hessenberg least-squares problem and the
// amplitude update are FP64 whatever precision the Jacobian products use.
//
// Orthogonalisation: classical Gram-Schmidt applied twice (CGS2) with fused
// multi-vector dot and update kernels. It builds the same Arnoldi relation
// as the modified Gram-Schmidt of the paper's algorithm (identical in exact
// arithmetic, at least as orthogonal in floating point) and needs one
// device-to-host transfer per Krylov step instead of one per basis vector.
// The small Hessenberg problem (Givens rotations, back substitution) is
// solved on the host.

#include "solvers.hpp"
#include "block_sum.hpp"
#include "eig.hpp"
#include "fock_op.hpp"

#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cmath>
#include <vector>

#include "cc_kernels.hpp"
#include "tensor_ops.hpp"

namespace pnk {

namespace {
constexpr int kMaxBasis = 256;  // multi_axpy limit
constexpr int kScal = 4 * kMaxBasis + 8;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Givens rotation zeroing b in (a, b): returns (c, s) with c a + s b = rho
void givens(double a, double b, double* c, double* s) {
  const double rho = std::hypot(a, b);
  if (rho == 0.0) { *c = 1.0; *s = 0.0; return; }
  *c = a / rho;
  *s = b / rho;
}

// Solve the upper-triangular k x k system R y = g (R column-major in H with
// leading dimension ldh).
std::vector<double> back_substitute(const std::vector<double>& H, int ldh, const std::vector<double>& g, int k) {
  std::vector<double> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double acc = g[i];
    for (int j = i + 1; j < k; ++j) acc -= H[i + (size_t)j * ldh] * y[j];
    const double d = H[i + (size_t)i * ldh];
    y[i] = d != 0.0 ? acc / d : 0.0;
  }
  return y;
}

}  // namespace

size_t Solver::bytes(int64_t n, int m_max, int restart, int diis, int64_t outer_cap) {
  const int64_t cap = std::max(n, outer_cap);
  const size_t outer = (size_t)(m_max + 1) + 3 + 2 * (size_t)diis;
  const size_t inner = (size_t)(restart + 1) + 1;
  return (outer * cap + inner * n) * sizeof(double) + (kScal + reduce_partials_size(kMaxBasis)) * sizeof(double) +
         16 * 256;
}

Solver::Solver(Engine& eng, int m_max, int restart, int diis, hipStream_t alloc_stream, bool stream_ordered,
               int64_t outer_cap)
    : eng_(eng), n_(eng.nvec()), cap_(std::max(eng.nvec(), outer_cap)), nv_(eng.nvec()), vo_(eng.o()),
      vv_(eng.v()), m_max_(m_max), restart_(restart), diis_(diis), alloc_stream_(alloc_stream),
      async_(stream_ordered) {
  PNK_REQUIRE(m_max >= 1 && m_max < kMaxBasis && restart >= 1 && restart < kMaxBasis && diis >= 0 && diis < 64,
              "solver: Krylov or DIIS size out of range");
  auto alloc = [&](size_t count) {
    double* p = nullptr;
    if (count == 0) return p;
    hipError_t e = async_ ? hipMallocAsync((void**)&p, count * sizeof(double), alloc_stream_)
                          : hipMalloc(&p, count * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw OomError("solver allocation failed");
    }
    return p;
  };
  Qo_ = alloc((size_t)(m_max + 1) * cap_);
  Qi_ = alloc((size_t)(restart + 1) * n_);
  r_ = alloc(cap_);
  ri_ = alloc(n_);
  w_ = alloc(cap_);
  w2_ = alloc(cap_);
  hx_ = alloc((size_t)diis * cap_);
  he_ = alloc((size_t)diis * cap_);
  dsc_ = alloc(kScal);
  partials_ = alloc(reduce_partials_size(kMaxBasis));
  PNK_HIP(hipHostMalloc(&host_, kScal * sizeof(double), hipHostMallocDefault));
}

Solver::~Solver() {
  for (auto& layout : lz_graphs_)
    for (auto& row : layout)
      for (hipGraphExec_t e : row)
        if (e) (void)hipGraphExecDestroy(e);
  for (hipEvent_t e : lz_ev_)
    if (e) (void)hipEventDestroy(e);
  for (double* p : {Qo_, Qi_, r_, ri_, w_, w2_, hx_, he_, dsc_, partials_})
    if (p) (void)(async_ ? hipFreeAsync(p, alloc_stream_) : hipFree(p));
  if (host_) (void)hipHostFree(host_);
}

// Host-to-device copy through pinned staging (host_ + 3 * kMaxBasis). Every
// upload is followed by a stream synchronisation before the staging area is
// written again.
void Solver::upload(double* dev, const double* src, int n, hipStream_t s) {
  PNK_REQUIRE(n <= kMaxBasis, "upload: too many scalars");
  double* stage = host_ + 3 * kMaxBasis;
  for (int i = 0; i < n; ++i) stage[i] = src[i];
  PNK_HIP(hipMemcpyAsync(dev, stage, n * sizeof(double), hipMemcpyHostToDevice, s));
}

void Solver::read_scalars(double* host, const double* dev, int n, hipStream_t s) {
  PNK_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
}

void Solver::set_gauge(const Gauge* g) {
  if (g) {
    PNK_REQUIRE(g->nvec() <= cap_, "solver: the gauge's vectors exceed the outer capacity");
    nv_ = g->nvec();
    vo_ = g->mo;
    vv_ = g->mv;
  } else {
    nv_ = n_;
    vo_ = eng_.o();
    vv_ = eng_.v();
  }
  gauge_ = g;
}

void Solver::norms(int64_t n, const double* r, double* ninf, double* n2, hipStream_t s) {
  nrm_inf(n, r, dsc_ + 0, partials_, s);
  nrm2(n, r, dsc_ + 1, partials_ + kReduceBlocks, s);
  read_scalars(host_, dsc_, 2, s);
  *ninf = host_[0];
  *n2 = host_[1];
}

double Solver::orthogonalise(int64_t n, double* Q, int64_t ldq, int m, double* w, std::vector<double>& h,
                             hipStream_t s) {
  double* h1 = dsc_;
  double* h2 = dsc_ + kMaxBasis;
  double* hn = dsc_ + 2 * kMaxBasis;
  multi_dot(n, m, Q, ldq, w, h1, partials_, s);
  multi_axpy(n, m, Q, ldq, h1, w, s);
  multi_dot(n, m, Q, ldq, w, h2, partials_, s);
  multi_axpy(n, m, Q, ldq, h2, w, s);
  nrm2(n, w, hn, partials_, s);
  read_scalars(host_, dsc_, 2 * kMaxBasis + 1, s);
  h.assign(m, 0.0);
  for (int i = 0; i < m; ++i) h[i] = host_[i] + host_[kMaxBasis + i];
  return host_[2 * kMaxBasis];
}

namespace {

// ---- short-recurrence (Lanczos) GMRES for symmetric A_F, all on the device ----
// Three kernels per step. Global sums are never a kernel of their own: the
// kernel that needs a sum adds the previous kernel's per-workgroup partial
// sums itself, every workgroup in the same fixed order (so every workgroup
// gets the same bits), and the scalar recurrences are evaluated redundantly
// by every workgroup of the last kernel. The state therefore has two slots:
// step k reads slot k % 2 and workgroup 0 writes slot (k + 1) % 2.
// state: [0] beta_k  [1] alpha_k  [2] beta_{k+1}  [3] c_{k-2} [4] s_{k-2}
//        [5] c_{k-1} [6] s_{k-1}  [7] phibar      [8] rho1    [9] delta
//        [10] eps    [11] phi     [12] |phibar|   [13] 1/beta_{k+1}
//        [14] done (the stopping test held at an earlier step)
// A third, fixed slot after the two holds what the host reads: steps run,
// the last residual estimate and beta, the absolute tolerance, ||b||.
// (the layout is shared with the fused packed step in fock_op)
constexpr int kBeta = kLzBeta, kAlpha = kLzAlpha, kBetaN = kLzBetaN, kC2 = kLzC2, kS2 = kLzS2, kC1 = kLzC1,
              kS1 = kLzS1, kPhiBar = kLzPhiBar, kRho1 = kLzRho1, kDelta = kLzDelta, kEps = kLzEps, kPhi = kLzPhi,
              kRes = kLzRes, kInvB = kLzInvB, kDone = kLzDone, kFirst = kLzFirst, kNState = kLzNState;
constexpr int kFinSteps = kLzFinSteps, kFinRes = kLzFinRes, kFinBeta = kLzFinBeta, kFinTol = kLzFinTol,
              kFinBNorm = kLzFinBNorm, kFinBHat = kLzFinBHat, kFinCount = kLzFinCount;
constexpr int kStateStride = kLzStateStride;
constexpr int kLzBlocks = 512;
// With f_ov = 0, A_F is block diagonal and its doubles block is the
// Kronecker sum of the singles block with itself (A_F, equation
// Preconditioner and its working equations): its spectrum spans exactly
// [2 lmin, 2 lmax] when the singles spectrum spans [lmin, lmax]. The
// symmetric inner solve therefore runs on D^1/2 A_F D^1/2 with D = 2 on
// the singles, which brings both blocks onto [2 lmin, 2 lmax] and halves
// the condition number (about 1/sqrt(2) as many Lanczos steps).
constexpr double kInnerSinglesScale = 2.0;

constexpr int kMaxFusedParts = 16384;  // workgroups of the fused A_F launch (three partials each)

// p = S p - beta_k v_{k-1} (S scales the first n1 entries by s1); partial
// sums of <v_k, p>, <p, p> and <v_k, v_k> (part1[b], part1[G + b],
// part1[2 G + b], G = gridDim.x)
__global__ __launch_bounds__(256) void lz_step1(int64_t n, double* __restrict__ p, const double* __restrict__ vprev,
                                                const double* __restrict__ v, const double* __restrict__ st,
                                                double* __restrict__ part1, int64_t n1, double s1) {
  if (st[kDone] != 0.0) return;
  __shared__ double sm[3][4];
  const double beta = st[kBeta];
  double dot = 0.0, nrm = 0.0, vv2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double x = (i < n1 ? s1 : 1.0) * p[i] - beta * vprev[i];
    const double vk = v[i];
    p[i] = x;
    dot += vk * x;
    nrm += x * x;
    vv2 += vk * vk;
  }
  double r[3] = {dot, nrm, vv2};
  block_sum256<3>(r, sm);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) part1[c * gridDim.x + blockIdx.x] = r[c];
}

// alpha_k = <v_k, p> / <v_k, v_k> and beta_{k+1} = ||p - alpha_k v_k||,
// from ||p||^2 - <v_k, p>^2 / <v_k, v_k> (p - alpha_k v_k is orthogonal to
// v_k), all from the partials of the launch before. Measuring <v_k, v_k>
// rather than taking it as 1 keeps a rounding error in the norm of v_k from
// growing from step to step. Then one Givens rotation of the tridiagonal
// QR, and
// w_k = (v_k - delta w_{k-1} - eps w_{k-2}) / rho1 (into the w_{k-2} slot),
// x += phi w_k, v_{k+1} = (p - alpha_k v_k) / beta_{k+1} (in place).
// The stopping test (|phibar| <= tolerance, or beta_{k+1} = 0) is taken
// here after every step; once it holds, the later steps of the queue pass
// the done flag on and write nothing else.
__global__ __launch_bounds__(256) void lz_update(int64_t n, const double* __restrict__ v,
                                                 const double* __restrict__ w1, double* __restrict__ w2,
                                                 double* __restrict__ x, double* __restrict__ p,
                                                 const double* __restrict__ part1, int nparts1,
                                                 const double* __restrict__ st, double* __restrict__ stn,
                                                 double* __restrict__ fin) {
  if (st[kDone] != 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) stn[kDone] = 1.0;
    return;
  }
  __shared__ double sm[3][4];
  double r[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nparts1; k += 256) {
    r[0] += part1[k];
    r[1] += part1[nparts1 + k];
    r[2] += part1[2 * nparts1 + k];
  }
  block_sum256<3>(r, sm);
  const double vp = r[0], pp = r[1], vv = r[2];
  const double alpha = vv > 0.0 ? vp / vv : 0.0;
  const double betan = sqrt(fmax(pp - alpha * vp, 0.0));
  const double beta = st[kBeta];
  const double c2 = st[kC2], s2 = st[kS2], c1 = st[kC1], s1 = st[kS1];
  const double eps = s2 * beta;
  const double dbar = c2 * beta;
  const double delta = c1 * dbar + s1 * alpha;
  const double gbar = -s1 * dbar + c1 * alpha;
  const double rho1 = hypot(gbar, betan);
  const double c = rho1 != 0.0 ? gbar / rho1 : 1.0;
  const double s = rho1 != 0.0 ? betan / rho1 : 0.0;
  const double phibar = st[kPhiBar];
  const double phi = c * phibar;
  const double invb = betan != 0.0 ? 1.0 / betan : 0.0;
  const double ir = rho1 != 0.0 ? 1.0 / rho1 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    stn[kBeta] = betan;
    stn[kAlpha] = alpha;
    stn[kBetaN] = betan;
    stn[kC2] = c1; stn[kS2] = s1;
    stn[kC1] = c; stn[kS1] = s;
    stn[kPhiBar] = -s * phibar;
    stn[kRho1] = rho1;
    stn[kDelta] = delta;
    stn[kEps] = eps;
    stn[kPhi] = phi;
    const double res = fabs(s * phibar);
    stn[kRes] = res;
    stn[kInvB] = invb;
    stn[kDone] = (res <= fin[kFinTol] || betan == 0.0) ? 1.0 : 0.0;
    fin[kFinSteps] += 1.0;
    fin[kFinRes] = res;
    fin[kFinBeta] = betan;
  }
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double vi = v[i];
    const double w = (vi - delta * w1[i] - eps * w2[i]) * ir;
    w2[i] = w;
    x[i] += phi * w;
    p[i] = (p[i] - alpha * vi) * invb;
  }
}

// bnorm: norm of the (scaled) start vector; rhs_norm: ||b||, which with
// rtol sets the absolute tolerance on the residual estimate.
__global__ void lz_init(double* st, const double* bnorm, const double* rhs_norm, double rtol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int k = 0; k < kNState; ++k) st[k] = 0.0;
  st[kC2] = 1.0; st[kC1] = 1.0;
  st[kPhiBar] = *bnorm;
  st[kRes] = *bnorm;
  st[kBeta] = 0.0;
  st[kStateStride + kDone] = 0.0;
  double* fin = st + 2 * kStateStride;
  fin[kFinSteps] = 0.0;
  fin[kFinRes] = *bnorm;
  fin[kFinBeta] = 1.0;
  fin[kFinTol] = rtol * *rhs_norm;
  fin[kFinBNorm] = *rhs_norm;
}

// ---- packed pair layout for pair-symmetric vectors (pairs i <= j) ----

__device__ inline int lzp_pair(int i, int j, int o) { return i * o - i * (i - 1) / 2 + (j - i); }  // i <= j

__device__ inline void lzp_decode(int pr, int o, int& i, int& j) {
  i = 0;
  while (pr >= o - i) {
    pr -= o - i;
    ++i;
  }
  j = i + pr;
}

constexpr int kPackTile = 32;
constexpr int kPackBlocksX = 16;  // workgroups per pair block (grid-stride over its tiles)

// xp = packed D^1/2 sym(b): singles times rs; for i <= j the block
// (b_ij + b_ji^T) / 2 (the pair-symmetric part; b_ji^T staged through LDS).
// Each workgroup writes its shares of ||sym(b)||^2 and ||D^1/2 sym(b)||^2
// (blocks of pairs i < j counted twice) to parts[g], parts[G + g], g the
// workgroup's linear index, G the number of workgroups. The packed vectors
// of z (null entries skipped) are set to zero in the same pass.
struct ZeroList {
  double* p[4];
};

__global__ __launch_bounds__(256) void lzp_pack(int o, int v, const double* __restrict__ b, double rs,
                                                double* __restrict__ xp, double* __restrict__ parts, ZeroList z) {
  __shared__ double tile[kPackTile][kPackTile + 1];
  __shared__ double sm[2][4];
  const int npair = o * (o + 1) / 2;
  const int64_t vv = (int64_t)v * v, ov = (int64_t)o * v;
  const int tid = threadIdx.x;
  double s_plain = 0.0, s_scaled = 0.0;
  if ((int)blockIdx.y == npair) {
    for (int64_t e = blockIdx.x * (int64_t)256 + tid; e < ov; e += (int64_t)gridDim.x * 256) {
      const double x = b[e];
      xp[e] = rs * x;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (z.p[q]) z.p[q][e] = 0.0;
      s_plain += x * x;
      s_scaled += (rs * x) * (rs * x);
    }
  } else {
    int i, j;
    lzp_decode(blockIdx.y, o, i, j);
    const double w = i == j ? 1.0 : 2.0;
    const double* __restrict__ bij = b + ov + (int64_t)(i * o + j) * vv;
    const double* __restrict__ bji = b + ov + (int64_t)(j * o + i) * vv;
    double* __restrict__ out = xp + ov + (int64_t)blockIdx.y * vv;
    const int nt = (v + kPackTile - 1) / kPackTile;
    const int tx = tid % kPackTile, ty = tid / kPackTile;
    for (int tl = blockIdx.x; tl < nt * nt; tl += gridDim.x) {
      const int a0 = (tl / nt) * kPackTile, b0 = (tl % nt) * kPackTile;
      __syncthreads();
      for (int r = ty; r < kPackTile; r += 256 / kPackTile) {  // tile[r][c] = b_ji[b0 + r][a0 + c]
        const int rr = b0 + r, cc = a0 + tx;
        tile[r][tx] = (rr < v && cc < v) ? bji[(int64_t)rr * v + cc] : 0.0;
      }
      __syncthreads();
      for (int r = ty; r < kPackTile; r += 256 / kPackTile) {
        const int a = a0 + r, bb = b0 + tx;
        if (a < v && bb < v) {
          const double x = 0.5 * (bij[(int64_t)a * v + bb] + tile[tx][r]);
          out[(int64_t)a * v + bb] = x;
          const int64_t idx = ov + (int64_t)blockIdx.y * vv + (int64_t)a * v + bb;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (z.p[q]) z.p[q][idx] = 0.0;
          s_plain += w * x * x;
          s_scaled += w * x * x;
        }
      }
    }
  }
  double r2[2] = {s_plain, s_scaled};
  block_sum256<2>(r2, sm);
  const int g = blockIdx.y * gridDim.x + blockIdx.x, G = gridDim.x * gridDim.y;
  if (tid == 0) {
    parts[g] = r2[0];
    parts[G + g] = r2[1];
  }
}

// x (full layout) = D^1/2 unpack(xp): x_ij = xp_P(i,j) for i <= j, and
// xp_P(j,i)^T (through LDS) for i > j; singles times rs.
__global__ __launch_bounds__(256) void lzp_unpack(int o, int v, const double* __restrict__ xp, double rs,
                                                  double* __restrict__ x) {
  __shared__ double tile[kPackTile][kPackTile + 1];
  const int64_t vv = (int64_t)v * v, ov = (int64_t)o * v;
  const int tid = threadIdx.x;
  if ((int)blockIdx.y == o * o) {
    for (int64_t e = blockIdx.x * (int64_t)256 + tid; e < ov; e += (int64_t)gridDim.x * 256) x[e] = rs * xp[e];
    return;
  }
  const int i = blockIdx.y / o, j = blockIdx.y % o;
  double* __restrict__ out = x + ov + (int64_t)blockIdx.y * vv;
  if (i <= j) {
    const double* __restrict__ src = xp + ov + (int64_t)lzp_pair(i, j, o) * vv;
    for (int64_t e = blockIdx.x * (int64_t)256 + tid; e < vv; e += (int64_t)gridDim.x * 256) out[e] = src[e];
    return;
  }
  const double* __restrict__ src = xp + ov + (int64_t)lzp_pair(j, i, o) * vv;  // x_ij = x_ji^T
  const int nt = (v + kPackTile - 1) / kPackTile;
  const int tx = tid % kPackTile, ty = tid / kPackTile;
  for (int tl = blockIdx.x; tl < nt * nt; tl += gridDim.x) {
    const int a0 = (tl / nt) * kPackTile, b0 = (tl % nt) * kPackTile;
    __syncthreads();
    for (int r = ty; r < kPackTile; r += 256 / kPackTile) {  // tile[r][c] = x_ji[b0 + r][a0 + c]
      const int rr = b0 + r, cc = a0 + tx;
      tile[r][tx] = (rr < v && cc < v) ? src[(int64_t)rr * v + cc] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < kPackTile; r += 256 / kPackTile) {
      const int a = a0 + r, bb = b0 + tx;
      if (a < v && bb < v) out[(int64_t)a * v + bb] = tile[tx][r];
    }
  }
}

// Set-up of the packed solve: the two norms from lzp_pack's partials
// (nparts each, summed in a fixed order by one workgroup); the state before
// step 0 (slot 1) with the first flag; and, in place of the shares of an
// occupied launch (occ_parts, occ_nparts each), (0, ||start||^2, 0), from
// which the first fused step normalises the start vector.
// Packed three-launch form: the state before the first step (slot 0) from
// the packing's partial sums of ||b||^2 and ||D^1/2 b||^2; the start vector
// is then normalised by ||D^1/2 b|| (fin's kFinBHat).
__global__ __launch_bounds__(256) void lzp_init_normalised(const double* __restrict__ parts, int nparts, double* st,
                                                           double rtol) {
  __shared__ double sm[2][4];
  double r[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < nparts; k += 256) {
    r[0] += parts[k];
    r[1] += parts[nparts + k];
  }
  block_sum256<2>(r, sm);
  if (threadIdx.x != 0) return;
  const double bn = sqrt(r[0]), bhat = sqrt(r[1]);
  for (int k = 0; k < kNState; ++k) st[k] = 0.0;
  st[kC2] = 1.0;
  st[kC1] = 1.0;
  st[kPhiBar] = bhat;
  st[kRes] = bhat;
  st[kStateStride + kDone] = 0.0;
  double* fin = st + 2 * kStateStride;
  fin[kFinSteps] = 0.0;
  fin[kFinRes] = bhat;
  fin[kFinBeta] = 1.0;
  fin[kFinTol] = rtol * bn;
  fin[kFinBNorm] = bn;
  fin[kFinBHat] = bhat;
}

__global__ __launch_bounds__(256) void lzp_init_fused(const double* __restrict__ parts, int nparts, double* st,
                                                      double* __restrict__ occ_parts, int occ_nparts, double rtol) {
  __shared__ double sm[2][4];
  double r[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < nparts; k += 256) {
    r[0] += parts[k];
    r[1] += parts[nparts + k];
  }
  block_sum256<2>(r, sm);
  for (int k = threadIdx.x; k < 3 * occ_nparts; k += 256) occ_parts[k] = 0.0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double bn = sqrt(r[0]), bhat = sqrt(r[1]);
  occ_parts[occ_nparts] = r[1];
  double* s1 = st + kStateStride;  // the state before step 0
  for (int k = 0; k < kNState; ++k) s1[k] = 0.0;
  s1[kFirst] = 1.0;
  st[kDone] = 0.0;
  double* fin = st + 2 * kStateStride;
  fin[kFinSteps] = 0.0;
  fin[kFinRes] = bhat;
  fin[kFinBeta] = 1.0;
  fin[kFinTol] = rtol * bn;
  fin[kFinBNorm] = bn;
  fin[kFinBHat] = bhat;
}

inline int grid_n(int64_t n) {
  int64_t g = ceil_div(n, 256);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

}  // namespace

// A_F symmetric (f_ov = 0): the Arnoldi process of GMRES reduces to the
// three-term Lanczos recurrence and the Hessenberg least-squares problem to
// a tridiagonal one, updated with one Givens rotation per step (GMRES and
// MINRES coincide in exact arithmetic). Everything stays on the device,
// including the stopping test; the host reads the outcome once per batch
// of queued steps.
// One Lanczos step on fixed buffers (see precond_solve_sym).
// Device scalars: [0, kMaxBasis) and [kMaxBasis, 2 kMaxBasis) projections,
// then norms; the Lanczos state's three slots start at 3.5 kMaxBasis.
double* Solver::lanczos_state() const { return dsc_ + 3 * kMaxBasis + kMaxBasis / 2; }

void Solver::lanczos_step(double* vprev, double* v, double* p, double* w1, double* w2, double* x, double* st,
                          double* stn, hipStream_t s) {
  int64_t n = n_;
  const int64_t ov = (int64_t)eng_.o() * eng_.v();
  double* part1 = partials_;
  const FockOp* op = eng_.fock_op();
  int nparts1 = kLzBlocks;
  if (lz_mode_ == kLzPacked3) {
    // packed pair layout (see precond_solve_sym): the same three launches
    n = ov + (int64_t)op->npair * eng_.v() * eng_.v();
    Timers* tm = eng_.timers();
    fock_op_lanczos_vir_packed(*op, v, p, st + kDone, s);
    if (tm) tm->begin(kTimerFock, s);
    fock_op_lanczos_occ_packed(*op, v, vprev, st + kBeta, p, part1, kInnerSinglesScale, st + kDone, s);
    if (tm) tm->end(kTimerFock, s);
    nparts1 = (int)op->nparts_packed();
  } else if (op && op->nparts() <= kMaxFusedParts) {
    // p = A_F v_k - beta_k v_{k-1} and the partials of <v_k, p>; the timer
    // covers the occupied launch
    Timers* tm = eng_.timers();
    fock_op_lanczos_vir(*op, v, p, st + kDone, s);
    if (tm) tm->begin(kTimerFock, s);
    fock_op_lanczos_occ(*op, v, vprev, st + kBeta, p, part1, kInnerSinglesScale, st + kDone, s);
    if (tm) tm->end(kTimerFock, s);
    nparts1 = (int)op->nparts();
  } else {
    eng_.fock_apply(v, v + ov, p, p + ov, s);
    lz_step1<<<kLzBlocks, 256, 0, s>>>(n, p, vprev, v, st, part1, ov, kInnerSinglesScale);
  }
  lz_update<<<kLzBlocks, 256, 0, s>>>(n, v, w1, w2, x, p, part1, nparts1, st, stn,
                                      lanczos_state() + 2 * kStateStride);
  PNK_CHECK_LAUNCH();
}

// Six steps: the buffer rotation (v: period 3, w: period 2, state slot:
// period 2) returns to its start, so the block can be recorded once as a
// HIP graph and replayed.
int Solver::lz_block_len() const { return lz_mode_ == kLzFused ? kPackedBlock : kLanczosBlock; }

void Solver::lanczos_block(hipStream_t s) {
  const int64_t n = n_;
  double* st = lanczos_state();
  if (lz_mode_ == kLzFused) {
    // packed: two launches per step, the update fused into the next step's
    // virtual launch; four vectors rotate (P = p_{k-1}, V = v_{k-1}, N = v_k,
    // Y = y_k -> p_k), period 4; w rotates with period 2
    const FockOp& op = *eng_.fock_op();
    const int np = (int)op.nparts_packed();
    double *P = Qi_, *V = Qi_ + n, *N = Qi_ + 2 * n, *Y = Qi_ + 3 * n;
    double *w1 = Qi_ + 4 * n, *w2 = Qi_ + 5 * n, *x = Qi_ + 6 * n;
    double* fin = st + 2 * kStateStride;
    Timers* tm = eng_.timers();
    for (int k = 0; k < kPackedBlock; ++k) {
      double* prev = st + ((k + 1) % 2) * kStateStride;  // state after step k-1
      double* cur = st + (k % 2) * kStateStride;         // state after step k
      // the timer covers the fused launch (the larger of the two)
      if (tm) tm->begin(kTimerFock, s);
      fock_op_lanczos_vir_fused(op, P, V, N, Y, w1, w2, x, partials_, np, prev, cur, fin, s);
      if (tm) tm->end(kTimerFock, s);
      fock_op_lanczos_occ_packed(op, N, V, cur + kBeta, Y, partials_, kInnerSinglesScale, cur + kDone, s);
      double* oldP = P;
      P = Y;     // p_k
      Y = V;     // free
      V = N;     // v_k
      N = oldP;  // free
      std::swap(w1, w2);
    }
    return;
  }
  double *vprev = Qi_, *v = Qi_ + n, *p = Qi_ + 2 * n, *w1 = Qi_ + 3 * n, *w2 = Qi_ + 4 * n, *x = Qi_ + 5 * n;
  for (int k = 0; k < kLanczosBlock; ++k) {
    double* cur = st + (k % 2) * kStateStride;
    double* nxt = st + ((k + 1) % 2) * kStateStride;
    lanczos_step(vprev, v, p, w1, w2, x, cur, nxt, s);
    std::swap(vprev, v);  // v_{k-1} <- v_k
    std::swap(v, p);      // v_k <- v_{k+1}; p <- free buffer
    std::swap(w1, w2);    // w_{k-1} <- w_k
  }
}

namespace {

// The nodes of a graph recorded from one stream, in stream order: such a
// graph is a chain (one root, one dependent per node). Empty if it is not.
std::vector<hipGraphNode_t> chain_order(hipGraph_t g) {
  size_t nn = 0;
  if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess || nn == 0) return {};
  size_t nr = 0;
  if (hipGraphGetRootNodes(g, nullptr, &nr) != hipSuccess || nr != 1) return {};
  hipGraphNode_t node;
  if (hipGraphGetRootNodes(g, &node, &nr) != hipSuccess) return {};
  std::vector<hipGraphNode_t> out;
  out.reserve(nn);
  while (true) {
    out.push_back(node);
    size_t ns = 0;
    if (hipGraphNodeGetDependentNodes(node, nullptr, &ns) != hipSuccess || ns > 1) return {};
    if (ns == 0) break;
    if (hipGraphNodeGetDependentNodes(node, &node, &ns) != hipSuccess) return {};
  }
  if (out.size() != nn) return {};
  return out;
}

// Inserts event record nodes before and after each timed A_F kernel node
// (fock_op_is_timed_lanczos_kernel) of a chain graph: pair k (events ev[2k],
// ev[2k+1]) brackets the k-th such launch in stream order, so its duration
// can be read after a replay. Returns the number of pairs, -1 on failure.
int bracket_fock_nodes(hipGraph_t g, const hipEvent_t* ev, int max_pairs, bool fused) {
  const std::vector<hipGraphNode_t> nodes = chain_order(g);
  if (nodes.empty()) return -1;
  int k = 0;
  for (hipGraphNode_t node : nodes) {
    hipGraphNodeType type;
    if (hipGraphNodeGetType(node, &type) != hipSuccess) return -1;
    if (type != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    if (hipGraphKernelNodeGetParams(node, &kp) != hipSuccess) return -1;
    if (!fock_op_is_timed_lanczos_kernel(kp.func, fused)) continue;
    if (k >= max_pairs) return -1;
    size_t nd = 0, ns = 0;
    if (hipGraphNodeGetDependencies(node, nullptr, &nd) != hipSuccess) return -1;
    std::vector<hipGraphNode_t> deps(nd);
    if (nd && hipGraphNodeGetDependencies(node, deps.data(), &nd) != hipSuccess) return -1;
    if (hipGraphNodeGetDependentNodes(node, nullptr, &ns) != hipSuccess) return -1;
    std::vector<hipGraphNode_t> succ(ns);
    if (ns && hipGraphNodeGetDependentNodes(node, succ.data(), &ns) != hipSuccess) return -1;
    hipGraphNode_t e1, e2;
    if (hipGraphAddEventRecordNode(&e1, g, deps.data(), nd, ev[2 * k]) != hipSuccess) return -1;
    for (hipGraphNode_t d : deps)
      if (hipGraphRemoveDependencies(g, &d, &node, 1) != hipSuccess) return -1;
    if (hipGraphAddDependencies(g, &e1, &node, 1) != hipSuccess) return -1;
    if (hipGraphAddEventRecordNode(&e2, g, &node, 1, ev[2 * k + 1]) != hipSuccess) return -1;
    for (hipGraphNode_t sn : succ) {
      if (hipGraphRemoveDependencies(g, &node, &sn, 1) != hipSuccess) return -1;
      if (hipGraphAddDependencies(g, &e2, &sn, 1) != hipSuccess) return -1;
    }
    ++k;
  }
  return k;
}

}  // namespace

// Records nb six-step blocks as one HIP graph. The timed variant also holds
// event record nodes around each fused A_F launch (used only while the
// engine's timers are on).
bool Solver::ensure_lanczos_graph(bool timed, int nb) {
  if (nb < 1 || nb > kMaxBatchBlocks) return false;
  hipGraphExec_t& exec = lz_graphs_[lz_mode_][timed ? 1 : 0][nb];
  bool& failed = lz_graph_failed_[lz_mode_][timed ? 1 : 0][nb];
  if (exec) return true;
  if (failed) return false;
  const int pairs = nb * lz_block_len();
  if (timed) {
    while ((int)lz_ev_.size() < 2 * pairs) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) { failed = true; return false; }
      lz_ev_.push_back(e);
    }
  }
  Timers* tm = eng_.timers();
  eng_.set_timers(nullptr);  // no host-side timer events inside a graph
  bool ok = false;
  hipStream_t cs = nullptr;
  hipGraph_t g = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
      hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    // a failure while recording must not leave a partial graph behind
    bool threw = false;
    try {
      for (int q = 0; q < nb; ++q) lanczos_block(cs);
    } catch (const std::exception& e) {
      threw = true;
      if (std::getenv("PNK_DEBUG")) std::fprintf(stderr, "pnk: graph capture failed: %s\n", e.what());
    }
    if (hipStreamEndCapture(cs, &g) == hipSuccess && g && !threw &&
        (!timed || bracket_fock_nodes(g, lz_ev_.data(), pairs, lz_mode_ == kLzFused) == pairs) &&
        hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess)
      ok = true;
  }
  if (g) (void)hipGraphDestroy(g);
  if (cs) (void)hipStreamDestroy(cs);
  (void)hipGetLastError();
  eng_.set_timers(tm);
  if (!ok) {
    if (std::getenv("PNK_DEBUG"))
      std::fprintf(stderr, "pnk: no %s inner-solve graph of %d blocks\n", timed ? "timed" : "plain", nb);
    exec = nullptr;
    failed = true;
  }
  return ok;
}

// A_F symmetric (f_ov = 0): the Arnoldi process of GMRES reduces to the
// three-term Lanczos recurrence and the Hessenberg least-squares problem to
// a tridiagonal one, updated with one Givens rotation per step (GMRES and
// MINRES coincide in exact arithmetic). Everything stays on the device:
// blocks of six steps are replayed as one HIP graph, and the host reads the
// residual estimate after each block (so up to five extra steps run past
// convergence; they only lower the residual further).
int Solver::precond_solve_sym(const double* b, double* x, double rtol, int maxit, hipStream_t s, bool* converged,
                              bool packed) {
  const int64_t n = n_;
  const int o = eng_.o(), vir = eng_.v();
  const int64_t ov = (int64_t)o * vir;
  const double rs = std::sqrt(kInnerSinglesScale);
  double* st = lanczos_state();
  const double* fin = st + 2 * kStateStride;
  const FockOp* op = eng_.fock_op();
  const int mode = !packed ? kLzFull : (fock_op_fused_step(*op) ? kLzFused : kLzPacked3);
  lz_mode_ = mode;
  // scaled system D^1/2 A_F D^1/2 z = D^1/2 b, x = D^1/2 z, D = diag(s I, I).
  // ||b|| stays on the device (b = 0 gives a zero start and a stop at the
  // first step).
  double* xi;  // the iterate z
  if (mode == kLzPacked3) {
    // pair-symmetric b: the recurrence runs on pairs i <= j, with inner
    // products that count the blocks of pairs i < j twice (those of the full
    // vectors), so its steps are those of the full-layout recurrence; the
    // buffers are those of the full layout, n_l of each used
    const int64_t nl = ov + (int64_t)op->npair * vir * vir;
    double *vprev = Qi_, *v = Qi_ + n, *w1 = Qi_ + 3 * n, *w2 = Qi_ + 4 * n;
    xi = Qi_ + 5 * n;
    double* parts = partials_ + 3 * kMaxFusedParts;
    lzp_pack<<<dim3(kPackBlocksX, op->npair + 1), 256, 0, s>>>(o, vir, b, rs, xi, parts,
                                                                 ZeroList{{vprev, w1, w2, nullptr}});
    lzp_init_normalised<<<1, 256, 0, s>>>(parts, kPackBlocksX * (op->npair + 1), st, rtol);
    scale_by_inverse(nl, xi, fin + kFinBHat, v, s);  // v_1 = D^1/2 b / ||D^1/2 b||
    fill(nl, 0.0, xi, s);
  } else if (mode == kLzFused) {
    // the same on the two-launch form: the first fused step normalises the
    // start vector P = D^1/2 b (V = 0)
    double *P0 = Qi_, *V0 = Qi_ + n, *w1 = Qi_ + 4 * n, *w2 = Qi_ + 5 * n;
    xi = Qi_ + 6 * n;
    double* parts = partials_ + 3 * kMaxFusedParts;
    lzp_pack<<<dim3(kPackBlocksX, op->npair + 1), 256, 0, s>>>(o, vir, b, rs, P0, parts,
                                                                 ZeroList{{V0, w1, w2, xi}});
    lzp_init_fused<<<1, 256, 0, s>>>(parts, kPackBlocksX * (op->npair + 1), st, partials_,
                                      (int)op->nparts_packed(), rtol);
  } else {
    double *vprev = Qi_, *v = Qi_ + n, *w1 = Qi_ + 3 * n, *w2 = Qi_ + 4 * n;
    xi = Qi_ + 5 * n;
    nrm2(n, b, dsc_ + 2, partials_, s);
    copy(n, b, xi, s);
    axpby(ov, rs, b, 0.0, xi, s);
    nrm2(n, xi, dsc_ + 1, partials_, s);
    lz_init<<<1, 1, 0, s>>>(st, dsc_ + 1, dsc_ + 2, rtol);
    scale_by_inverse(n, xi, dsc_ + 1, v, s);  // v_1 = D^1/2 b / ||D^1/2 b||
    fill(n, 0.0, vprev, s);
    fill(n, 0.0, w1, s);
    fill(n, 0.0, w2, s);
    fill(n, 0.0, xi, s);
  }
  PNK_CHECK_LAUNCH();
  Timers* tm = eng_.timers();
  // the event pairs are read for a sample of the solves: each bracketed
  // launch pays for its two event nodes, which would slow every solve
  const bool timeable = (packed || (op && op->nparts() <= kMaxFusedParts)) && lz_solves_++ % kTimedEvery == 0;
  const int len = lz_block_len();
  // The first batch queues as many blocks as the last solve needed steps
  // (as one recorded graph), later ones a block each. The device stops the
  // recurrence at the first step that meets the test, so the batch size
  // changes the cost only, never the result. With timing on, the event
  // pairs of the timed launches that ran are read: the occupied launches
  // of the three-launch forms (one per step), the fused first launches of
  // the two-launch form (one per step plus the normalising first launch; a
  // step's update completes in the next step's first launch).
  const bool two = mode == kLzFused;
  int batch = std::min(std::max(1, (int)ceil_div(lz_steps_hint_ + (two ? 1 : 0), len)), (int)kMaxBatchBlocks);
  int launched = 0, steps = 0;
  bool conv = false;
  while (launched < maxit) {
    const int nb = (int)std::min<int64_t>(batch, ceil_div(maxit - launched, len));
    bool timed = false, graph = false;
    if (use_graphs_) {
      timed = tm && timeable && ensure_lanczos_graph(true, nb);
      graph = timed || ensure_lanczos_graph(false, nb);
    }
    if (graph) PNK_HIP(hipGraphLaunch(lz_graphs_[mode][timed ? 1 : 0][nb], s));
    else
      for (int q = 0; q < nb; ++q) lanczos_block(s);
    const int before = launched;
    launched += nb * len;
    batch = 1;
    read_scalars(host_, fin, kFinCount, s);  // synchronises the stream
    steps = (int)host_[kFinSteps];
    // ||b - A_F x|| <= ||D^1/2 (b - A_F x)|| = the scaled residual (D >= I)
    const double res = host_[kFinRes], bn = host_[kFinBNorm];
    const bool ok = std::isfinite(res) && (res <= rtol * bn || host_[kFinBeta] == 0.0);
    if (timed) {
      const int ran_total = std::min(launched, two ? steps + 1 : steps);
      const int ran = std::min(nb * len, ran_total - before);
      for (int k = 0; k < ran; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, lz_ev_[2 * k], lz_ev_[2 * k + 1]) == hipSuccess) tm->add(kTimerFock, 1, ms);
        else (void)hipGetLastError();
      }
    }
    if (!std::isfinite(res)) break;
    if (ok) { conv = true; break; }
  }
  lz_steps_hint_ = steps;
  if (packed) {
    lzp_unpack<<<dim3(kPackBlocksX, o * o + 1), 256, 0, s>>>(o, vir, xi, rs, x);
    PNK_CHECK_LAUNCH();
  } else {
    copy(n, xi, x, s);
    axpby(ov, rs, xi, 0.0, x, s);
  }
  if (converged) *converged = conv;
  return steps;
}

int Solver::precond_solve(const double* b, double* x, double rtol, int maxit, int restart, hipStream_t s,
                          bool* converged, bool pair_symmetric) {
  PNK_REQUIRE(restart >= 1 && restart <= restart_, "precond_solve: restart exceeds the allocated basis");
  const int64_t n = n_;
  const int64_t ov = (int64_t)eng_.o() * eng_.v();
  Timers* tm = eng_.timers();
  if (tm) tm->begin(kTimerPrecond, s);
  struct EndTimer {
    Timers* t; hipStream_t s;
    ~EndTimer() { if (t) t->end(kTimerPrecond, s); }
  } end_timer{tm, s};
  if (eng_.fov_zero() && sym_inner_ && restart_ >= 5) {
    const FockOp* op = eng_.fock_op();
    const bool packed = pair_symmetric && op && op->pt > 0 && op->nparts_packed() <= kMaxFusedParts && restart_ >= 6;
    return precond_solve_sym(b, x, rtol, maxit, s, converged, packed);
  }
  double bn, dummy;
  norms(n, b, &dummy, &bn, s);
  fill(n, 0.0, x, s);
  if (converged) *converged = true;
  if (bn == 0.0) return 0;
  int total = 0;
  copy(n, b, ri_, s);  // r = b - A x with x = 0
  double beta = bn;
  std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h;
  while (true) {
    if (beta <= rtol * bn || total >= maxit || !std::isfinite(beta)) {
      if (converged) *converged = beta <= rtol * bn;
      return total;
    }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // Q_0 = r / beta
    scale_by_inverse(n, ri_, dsc_ + 1, Qi_, s);  // ||r|| from the last norms()
    int k_done = 0;
    bool done = false;
    for (int k = 0; k < restart; ++k) {
      double* q = Qi_ + (size_t)k * n;
      double* wv = Qi_ + (size_t)(k + 1) * n;
      eng_.fock_apply(q, q + ov, wv, wv + ov, s);
      ++total;
      const double hn = orthogonalise(n, Qi_, n, k + 1, wv, h, s);
      for (int i = 0; i <= k; ++i) H[i + (size_t)k * (restart + 1)] = h[i];
      H[k + 1 + (size_t)k * (restart + 1)] = hn;
      for (int i = 0; i < k; ++i) {
        double& a = H[i + (size_t)k * (restart + 1)];
        double& c = H[i + 1 + (size_t)k * (restart + 1)];
        const double t = cs[i] * a + sn[i] * c;
        c = -sn[i] * a + cs[i] * c;
        a = t;
      }
      givens(H[k + (size_t)k * (restart + 1)], hn, &cs[k], &sn[k]);
      H[k + (size_t)k * (restart + 1)] = cs[k] * H[k + (size_t)k * (restart + 1)] + sn[k] * hn;
      H[k + 1 + (size_t)k * (restart + 1)] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      k_done = k + 1;
      if (std::fabs(g[k + 1]) <= rtol * bn || total >= maxit || hn == 0.0 || !std::isfinite(hn)) {
        done = std::fabs(g[k + 1]) <= rtol * bn || hn == 0.0;
        break;
      }
      scale_by_inverse(n, wv, dsc_ + 2 * kMaxBasis, wv, s);  // hn, still on the device
    }
    std::vector<double> y = back_substitute(H, restart + 1, g, k_done);
    upload(dsc_ + 3 * kMaxBasis, y.data(), k_done, s);
    combine(n, k_done, Qi_, n, dsc_ + 3 * kMaxBasis, 1.0, x, s);
    if (done) {
      // the Givens estimate already meets the tolerance
      PNK_HIP(hipStreamSynchronize(s));
      if (converged) *converged = true;
      return total;
    }
    // true residual for the restart
    eng_.fock_apply(x, x + ov, ri_, ri_ + ov, s);
    axpby(n, 1.0, b, -1.0, ri_, s);
    double rinf;
    norms(n, ri_, &rinf, &beta, s);
  }
}

namespace {
double forcing(int k, double rn, double rn_prev, double eta_prev, double tol, const PnkOptions& o) {
  double eta;
  if (k == 0) {
    eta = o.eta0;
  } else {
    eta = o.gamma * std::pow(rn / rn_prev, o.alpha);
    const double sg = o.gamma * std::pow(eta_prev, o.alpha);
    if (sg > 0.1) eta = std::max(eta, sg);
  }
  eta = std::min(eta, o.eta_max);
  eta = std::max(eta, 0.5 * tol / rn);
  return std::min(eta, o.eta_max);
}
}  // namespace

// In a gauge: r(theta) = (W^T)^(x4) r(t), t = (C^T)^(x4) theta (kept in
// gauge_->t, the point J v is linearised at); A_F of the gauge is inverted
// on the range of (W^T)^(x4) as (W^T)^(x4) A_F^-1 (C^T)^(x4); the energy is
// that of t.
void Solver::g_residual(const double* x, double* r, hipStream_t s) {
  const int o = eng_.o(), vir = eng_.v();
  const int64_t ov = (int64_t)o * vir;
  if (!gauge_) {
    eng_.residual(x, x + ov, r, r + ov, s);
    return;
  }
  const Gauge& g = *gauge_;
  const int64_t gov = (int64_t)g.mo * g.mv;
  gauge_apply(g.mo, g.mv, o, vir, g.bwd_o, g.bwd_v, x, x + gov, g.t, g.t + ov, g.ta, g.tb, s);
  eng_.residual(g.t, g.t + ov, g.w1, g.w1 + ov, s);
  gauge_apply(o, vir, g.mo, g.mv, g.fwd_o, g.fwd_v, g.w1, g.w1 + ov, r, r + gov, g.ta, g.tb, s);
}

int Solver::g_precond(const double* b, double* x, double rtol, int maxit, int restart, hipStream_t s, bool* conv) {
  if (!gauge_) return precond_solve(b, x, rtol, maxit, restart, s, conv, true);
  const Gauge& g = *gauge_;
  const int o = eng_.o(), vir = eng_.v();
  const int64_t ov = (int64_t)o * vir, gov = (int64_t)g.mo * g.mv;
  gauge_apply(g.mo, g.mv, o, vir, g.bwd_o, g.bwd_v, b, b + gov, g.w2, g.w2 + ov, g.ta, g.tb, s);
  const int it = precond_solve(g.w2, g.w1, rtol, maxit, restart, s, conv, true);
  gauge_apply(o, vir, g.mo, g.mv, g.fwd_o, g.fwd_v, g.w1, g.w1 + ov, x, x + gov, g.ta, g.tb, s);
  return it;
}

void Solver::g_energy(const double* x, double* e_dev, hipStream_t s) {
  const int o = eng_.o(), vir = eng_.v();
  const int64_t ov = (int64_t)o * vir;
  if (!gauge_) {
    eng_.energy(x, x + ov, e_dev, s);
    return;
  }
  const Gauge& g = *gauge_;
  const int64_t gov = (int64_t)g.mo * g.mv;
  gauge_apply(g.mo, g.mv, o, vir, g.bwd_o, g.bwd_v, x, x + gov, g.w1, g.w1 + ov, g.ta, g.tb, s);
  eng_.energy(g.w1, g.w1 + ov, e_dev, s);
}

const double* Solver::g_zeros(hipStream_t s) {
  if (!gauge_) return eng_.zeros();
  fill(nv_, 0.0, w2_, s);
  return w2_;
}

void Solver::solve_pnk(double* x, const PnkOptions& opt, SolveStats* st, hipStream_t s) {
  const double t0 = now_s();
  *st = SolveStats();
  hist_.clear();
  PNK_REQUIRE(opt.m_max >= 1 && opt.m_max <= m_max_, "pnk: m_max exceeds the allocated basis");
  // outer vectors: length n with singles of gov elements over (vo, vv)
  // (the orbital ones, or the gauge's); ov: the orbital singles
  const int64_t n = nv_;
  const int o = eng_.o(), vir = eng_.v(), vo = vo_, vv = vv_;
  const int64_t ov = (int64_t)o * vir, gov = (int64_t)vo * vv;
  PNK_REQUIRE(opt.protocol == PnkOptions::kPNK || opt.protocol == PnkOptions::kNK ||
                  opt.protocol == PnkOptions::kINK,
              "pnk: unknown protocol");
  // CCD level: every vector keeps zero singles
  auto mask = [&](double* y) {
    if (opt.ccd) fill(gov, 0.0, y, s);
  };
  auto mask_orb = [&](double* y) {
    if (opt.ccd) fill(ov, 0.0, y, s);
  };
  // tolerance of the inner solves of A_F^-1 J q inside the Krylov loop
  const double krylov_rtol = opt.inner_rtol_jv > 0.0 ? opt.inner_rtol_jv : opt.inner_rtol;
  auto Ainv = [&](const double* b, double* out, double rtol) {
    if (opt.protocol == PnkOptions::kNK) {
      // no preconditioner: the identity on pair-symmetric vectors, applied
      // as the projection (b2 + b2^T over pairs) / 2 so that rounding-level
      // antisymmetric parts do not enter the Krylov space
      copy(gov, b, out, s);
      fill(n - gov, 0.0, out + gov, s);
      pair_symmetrize_add(vo, vv, b + gov, 0.5, out + gov, s);
    } else {
      bool conv = true;
      const int it = g_precond(b, out, rtol, opt.inner_maxit, opt.inner_restart, s, &conv);
      st->n_afmv += it;
      st->n_inner_iters += it;
    }
    mask(out);
  };
  if (opt.init_mp2) {
    // MP2-type start for every protocol (NK included): -A_F^-1 r(0)
    g_residual(g_zeros(s), r_, s);
    st->n_residual++;
    mask(r_);
    bool conv = true;
    const int it = g_precond(r_, x, opt.inner_rtol, opt.inner_maxit, opt.inner_restart, s, &conv);
    st->n_afmv += it;
    st->n_inner_iters += it;
    axpby(n, 0.0, x, -1.0, x, s);
  }
  mask(x);
  double rn_prev = 0.0, eta = opt.eta0;
  double stall_ref = 0.0;
  int stall_k = 0;
  int k = 0;
  std::vector<double> H, cs, sn, g, h;
  while (true) {
    g_residual(x, r_, s);
    st->n_residual++;
    mask(r_);
    double rinf, rn;
    norms(n, r_, &rinf, &rn, s);
    hist_.push_back(rn);
    hist_.push_back(rinf);
    st->res_inf = rinf;
    st->res_2 = rn;
    if (verbose_)
      std::fprintf(stderr, "pnk newton %d: |r|_inf %.3e |r|_2 %.3e, %d J v, %d A_F products\n", k, rinf, rn,
                   st->n_jvp, st->n_afmv);
    if (!std::isfinite(rn)) { st->diverged = 1; break; }
    if (rinf < opt.tol_inf) { st->converged = 1; break; }
    if (opt.stall_window > 0) {
      if (k == 0 || rinf < opt.stall_factor * stall_ref) {
        stall_ref = rinf;
        stall_k = k;
      } else if (k - stall_k >= opt.stall_window) {
        st->stalled = 1;
        break;
      }
    }
    if (k >= opt.max_newton) break;
    if (opt.protocol == PnkOptions::kINK) {
      // A_F dt = -r(t): one inner solve per step, no Jacobian products
      if (rn > 1e6) break;  // diverging, as FP ends it
      Ainv(r_, w_, opt.inner_rtol);
      axpby(n, -1.0, w_, 1.0, x, s);
      rn_prev = rn;
      ++k;
      continue;
    }
    eta = forcing(k, rn, rn_prev, eta, opt.tol_inf, opt);
    // z = A_F^{-1} r, q_1 = z / beta
    Ainv(r_, w_, opt.inner_rtol);
    double zinf, beta;
    norms(n, w_, &zinf, &beta, s);
    if (!(beta > 0.0) || !std::isfinite(beta)) { st->diverged = !std::isfinite(beta); break; }
    scale_by_inverse(n, w_, dsc_ + 1, Qo_, s);  // beta from norms()
    const int M = opt.m_max;
    H.assign((size_t)(M + 1) * M, 0.0);
    cs.assign(M, 0.0);
    sn.assign(M, 0.0);
    g.assign(M + 1, 0.0);
    g[0] = beta;
    double delta = 0.0;
    if (opt.use_fd_jvp) {
      double xinf, xn;
      norms(n, x, &xinf, &xn, s);
      delta = std::sqrt(2.220446049250313e-16) * (1.0 + xn);
    }
    int m_done = 0;
    for (int m = 0; m < M; ++m) {
      double* q = Qo_ + (size_t)m * n;
      double* wv = Qo_ + (size_t)(m + 1) * n;
      if (gauge_ && !opt.use_fd_jvp && opt.protocol == PnkOptions::kPNK) {
        // A_F^-1 J in the gauge is (W^T)^(x4) A_F^-1 J (C^T)^(x4): the
        // transforms between the two products cancel
        const Gauge& g = *gauge_;
        gauge_apply(vo, vv, o, vir, g.bwd_o, g.bwd_v, q, q + gov, g.w1, g.w1 + ov, g.ta, g.tb, s);
        eng_.jvp(g.w1, g.w1 + ov, g.w2, g.w2 + ov, opt.jvp_prec, s);
        st->n_jvp++;
        mask_orb(g.w2);
        bool conv = true;
        const int it = precond_solve(g.w2, g.w1, krylov_rtol, opt.inner_maxit, opt.inner_restart, s, &conv, true);
        st->n_afmv += it;
        st->n_inner_iters += it;
        mask_orb(g.w1);
        gauge_apply(o, vir, vo, vv, g.fwd_o, g.fwd_v, g.w1, g.w1 + ov, wv, wv + gov, g.ta, g.tb, s);
      } else {
        if (opt.use_fd_jvp) {
          // (r(theta + delta q) - r(theta)) / delta, the paper's product
          copy(n, x, w2_, s);
          axpby(n, delta, q, 1.0, w2_, s);
          g_residual(w2_, w_, s);
          axpby(n, -1.0 / delta, r_, 1.0 / delta, w_, s);
        } else if (gauge_) {
          const Gauge& g = *gauge_;
          gauge_apply(vo, vv, o, vir, g.bwd_o, g.bwd_v, q, q + gov, g.w1, g.w1 + ov, g.ta, g.tb, s);
          eng_.jvp(g.w1, g.w1 + ov, g.w2, g.w2 + ov, opt.jvp_prec, s);
          gauge_apply(o, vir, vo, vv, g.fwd_o, g.fwd_v, g.w2, g.w2 + ov, w_, w_ + gov, g.ta, g.tb, s);
        } else {
          eng_.jvp(q, q + ov, w_, w_ + ov, opt.jvp_prec, s);
        }
        st->n_jvp++;
        mask(w_);
        Ainv(w_, wv, krylov_rtol);
      }
      const double hn = orthogonalise(n, Qo_, n, m + 1, wv, h, s);
      for (int i = 0; i <= m; ++i) H[i + (size_t)m * (M + 1)] = h[i];
      for (int i = 0; i < m; ++i) {
        double& a = H[i + (size_t)m * (M + 1)];
        double& c = H[i + 1 + (size_t)m * (M + 1)];
        const double t = cs[i] * a + sn[i] * c;
        c = -sn[i] * a + cs[i] * c;
        a = t;
      }
      givens(H[m + (size_t)m * (M + 1)], hn, &cs[m], &sn[m]);
      H[m + (size_t)m * (M + 1)] = cs[m] * H[m + (size_t)m * (M + 1)] + sn[m] * hn;
      g[m + 1] = -sn[m] * g[m];
      g[m] = cs[m] * g[m];
      m_done = m + 1;
      if (std::fabs(g[m + 1]) <= eta * beta || hn <= 1e-14 * beta || !std::isfinite(hn)) break;
      if (m + 1 < M) {
        scale_by_inverse(n, wv, dsc_ + 2 * kMaxBasis, wv, s);
      }
    }
    std::vector<double> y = back_substitute(H, M + 1, g, m_done);
    upload(dsc_ + 3 * kMaxBasis, y.data(), m_done, s);
    combine(n, m_done, Qo_, n, dsc_ + 3 * kMaxBasis, -1.0, x, s);
    rn_prev = rn;
    ++k;
  }
  st->newton_iters = k;
  g_energy(x, dsc_, s);
  read_scalars(host_, dsc_, 1, s);
  st->e_corr = host_[0];
  st->seconds = now_s() - t0;
}

// The FP map t -> t - r(t) / (D + s) has the Jacobian G = I - diag(D +
// s)^-1 J(t); its spectral radius below one is what makes (S)FP converge
// locally (Section "Regularization"; the shift is the Ridge term of
// Appendix D). Arnoldi with CGS2 on pair-symmetric vectors (the projection
// (x2 + x2^T over pairs) / 2 follows every product), Ritz values of the
// Hessenberg matrix on the host.
double Solver::fp_spectral_radius(const double* t, const double* q0, double shift, int m, hipStream_t s,
                                  std::vector<double>* ritz_re, std::vector<double>* ritz_im) {
  PNK_REQUIRE(m >= 1 && m <= m_max_, "fp_spectral_radius: m exceeds the allocated basis");
  PNK_REQUIRE(!gauge_, "fp_spectral_radius: orbital basis only");
  const int64_t n = n_;
  const int o = eng_.o(), vir = eng_.v();
  const int64_t ov = (int64_t)o * vir;
  eng_.residual(t, t + ov, r_, r_ + ov, s);  // linearise at t
  double qinf, qn;
  norms(n, q0, &qinf, &qn, s);
  PNK_REQUIRE(qn > 0.0 && std::isfinite(qn), "fp_spectral_radius: the start vector is zero or not finite");
  scale_by_inverse(n, q0, dsc_ + 1, Qo_, s);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), h;
  int k_done = 0;
  for (int k = 0; k < m; ++k) {
    double* q = Qo_ + (size_t)k * n;
    double* wv = Qo_ + (size_t)(k + 1) * n;
    eng_.jvp(q, q + ov, w_, w_ + ov, Prec::F64, s);
    copy(n, q, w2_, s);
    jacobi_update(o, vir, eng_.f_oo(), eng_.f_vv(), shift, w_, w2_, nullptr, s);  // q - J q / (D + s)
    copy(ov, w2_, wv, s);
    fill(n - ov, 0.0, wv + ov, s);
    pair_symmetrize_add(o, vir, w2_ + ov, 0.5, wv + ov, s);
    const double hn = orthogonalise(n, Qo_, n, k + 1, wv, h, s);
    for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = h[i];
    k_done = k + 1;
    if (!std::isfinite(hn)) break;
    double hmax = 0.0;
    for (int i = 0; i <= k; ++i) hmax = std::max(hmax, std::fabs(h[i]));
    if (hn <= 1e-12 * std::max(1.0, hmax)) break;  // invariant subspace
    if (k + 1 < m) {
      H[(size_t)(k + 1) * m + k] = hn;
      scale_by_inverse(n, wv, dsc_ + 2 * kMaxBasis, wv, s);
    }
  }
  // the leading k_done x k_done block, row-major
  std::vector<double> Hk((size_t)k_done * k_done), re(k_done), im(k_done);
  for (int i = 0; i < k_done; ++i)
    for (int j = 0; j < k_done; ++j) Hk[(size_t)i * k_done + j] = H[(size_t)i * m + j];
  PNK_REQUIRE(hessenberg_eigenvalues(Hk.data(), k_done, re.data(), im.data()),
              "fp_spectral_radius: the Hessenberg eigenvalue iteration did not converge");
  double rho = 0.0;
  for (int i = 0; i < k_done; ++i) rho = std::max(rho, std::hypot(re[i], im[i]));
  if (ritz_re) *ritz_re = re;
  if (ritz_im) *ritz_im = im;
  return rho;
}

namespace {
// Bordered Pulay system [B -1; -1 0][c; l] = [0; -1] in the least-squares,
// minimum-norm sense (the pseudo-inverse): the bordered matrix is
// symmetric, so its singular values are the moduli of its eigenvalues,
// found by cyclic Jacobi rotations; components along eigenvalues below
// eps (m + 1) times the largest modulus are dropped (the usual SVD cutoff
// of a least-squares solver). Near convergence B shrinks with the squared
// error norms while the border stays 1, so an elimination with an
// absolute pivot test would declare it singular long before it is.
// Returns false only for a non-finite result.
bool pulay_solve(const std::vector<double>& B, int m, std::vector<double>& c) {
  const int n = m + 1;
  std::vector<double> A((size_t)n * n, 0.0), V((size_t)n * n, 0.0), rhs(n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[(size_t)i * n + j] = B[(size_t)i * m + j];
  for (int i = 0; i < m; ++i) { A[(size_t)i * n + m] = -1.0; A[(size_t)m * n + i] = -1.0; }
  rhs[m] = -1.0;
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (!(off > 1e-32 * tot)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        // rotation that zeroes A[p][q] (Golub & Van Loan, symmetric Schur)
        const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + tt * tt), sn = tt * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = cs * akp - sn * akq;
          a(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = cs * apk - sn * aqk;
          a(q, k) = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  double smax = 0.0;
  for (int i = 0; i < n; ++i) smax = std::max(smax, std::fabs(a(i, i)));
  const double cut = 2.220446049250313e-16 * n * smax;
  std::vector<double> sol(n, 0.0);
  for (int e = 0; e < n; ++e) {
    const double lam = a(e, e);
    if (!(std::fabs(lam) > cut)) continue;
    double proj = 0.0;
    for (int k = 0; k < n; ++k) proj += V[(size_t)k * n + e] * rhs[k];
    for (int k = 0; k < n; ++k) sol[k] += V[(size_t)k * n + e] * proj / lam;
  }
  for (double x : sol)
    if (!std::isfinite(x)) return false;
  c.assign(sol.begin(), sol.begin() + m);
  return true;
}
}  // namespace

void Solver::solve_fp_diis(double* x, const FpOptions& opt, SolveStats* st, hipStream_t s) {
  const double t0 = now_s();
  *st = SolveStats();
  hist_.clear();
  PNK_REQUIRE(opt.diis_size <= diis_, "fp: DIIS size exceeds the allocated history");
  // outer vectors: the orbital ones or the gauge's (dimensions vo_, vv_)
  const int64_t n = nv_;
  const int64_t gov = (int64_t)vo_ * vv_;
  auto mask = [&](double* y) {
    if (opt.ccd) fill(gov, 0.0, y, s);
  };
  // Jacobi denominators from the diagonals of the Fock blocks of the
  // gauge the iteration runs in
  const double* fo = gauge_ ? gauge_->Fo : eng_.f_oo();
  const double* fv = gauge_ ? gauge_->Fv : eng_.f_vv();
  if (opt.init_mp2) {
    g_residual(g_zeros(s), r_, s);
    st->n_residual++;
    mask(r_);
    bool conv = true;
    const int it = g_precond(r_, x, opt.inner_rtol, 200, restart_, s, &conv);
    st->n_afmv += it;
    st->n_inner_iters += it;
    axpby(n, 0.0, x, -1.0, x, s);
  }
  mask(x);
  const int nd = opt.diis_size;
  std::vector<int> slots;  // slot ids in age order (oldest first)
  std::vector<double> Bfull((size_t)std::max(nd, 1) * std::max(nd, 1), 0.0);
  int it = 0;
  while (true) {
    g_residual(x, r_, s);
    st->n_residual++;
    mask(r_);
    double rinf, rn;
    norms(n, r_, &rinf, &rn, s);
    hist_.push_back(rn);
    hist_.push_back(rinf);
    st->res_inf = rinf;
    st->res_2 = rn;
    if (verbose_) std::fprintf(stderr, "fp+diis iteration %d: |r|_inf %.3e |r|_2 %.3e\n", it, rinf, rn);
    if (!std::isfinite(rn)) { st->diverged = 1; break; }
    if (rinf < opt.tol_inf) { st->converged = 1; break; }
    if (it >= opt.max_iter || rn > 1e6) break;
    if (nd == 0) {
      jacobi_update(vo_, vv_, fo, fv, opt.level_shift, r_, x, nullptr, s);
      ++it;
      continue;
    }
    // choose the slot: next free one, else the oldest
    int slot;
    if ((int)slots.size() < nd) {
      slot = (int)slots.size();
    } else {
      slot = slots.front();
      slots.erase(slots.begin());
    }
    slots.push_back(slot);
    double* xs = hx_ + (size_t)slot * n;
    double* es = he_ + (size_t)slot * n;
    copy(n, x, xs, s);
    jacobi_update(vo_, vv_, fo, fv, opt.level_shift, r_, xs, es, s);
    // B row of the new error vector against every stored one (slot order).
    // Slots are filled in order, so the m in use are 0 .. m - 1; the others
    // hold uninitialised memory and are never read (a zero weight times a
    // non-finite value there would still be NaN)
    const int m = (int)slots.size();
    const int mm = std::max(nd, 1);
    multi_dot(n, m, he_, n, es, dsc_, partials_, s);
    read_scalars(host_, dsc_, m, s);
    for (int q : slots) {
      Bfull[(size_t)slot * mm + q] = host_[q];
      Bfull[(size_t)q * mm + slot] = host_[q];
    }
    if (it + 1 >= opt.diis_start && m >= 2) {
      std::vector<double> B((size_t)m * m), c;
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) B[(size_t)a * m + b] = Bfull[(size_t)slots[a] * mm + slots[b]];
      if (pulay_solve(B, m, c)) {
        std::vector<double> cs(m, 0.0);
        for (int a = 0; a < m; ++a) cs[slots[a]] = c[a];
        upload(dsc_ + 3 * kMaxBasis, cs.data(), m, s);
        fill(n, 0.0, x, s);
        combine(n, m, hx_, n, dsc_ + 3 * kMaxBasis, 1.0, x, s);
      } else {
        copy(n, xs, x, s);
      }
    } else {
      copy(n, xs, x, s);
    }
    ++it;
  }
  st->newton_iters = it;
  g_energy(x, dsc_, s);
  read_scalars(host_, dsc_, 1, s);
  st->e_corr = host_[0];
  st->seconds = now_s() - t0;
}

}  // namespace pnk
