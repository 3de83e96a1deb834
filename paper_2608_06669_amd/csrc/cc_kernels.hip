// Small CCSD-specific kernels (HBM or launch-latency bound).

#include "cc_kernels.hpp"
#include "tensor_ops.hpp"

namespace pnk {
namespace {

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = ceil_div(n, 256);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__global__ void assemble_fock_kernel(int o, int v, const double* f_oo, const double* f_ov, const double* f_vv,
                                     double* f) {
  const int n = o + v;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int p = e / n, q = e % n;
    double x;
    if (p < o && q < o) x = f_oo[p * o + q];
    else if (p < o) x = f_ov[p * v + (q - o)];
    else if (q < o) x = f_ov[q * v + (p - o)];
    else x = f_vv[(p - o) * v + (q - o)];
    f[e] = x;
  }
}

__global__ void extract_occ_rows_kernel(int naux, int o, int n, const double* L, double* Lo) {
  const int64_t total = (int64_t)naux * o * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = e / ((int64_t)o * n);
    const int64_t r = e % ((int64_t)o * n);
    Lo[e] = L[P * n * n + r];
  }
}

__global__ void extract_blocks_kernel(int naux, int o, int v, const double* L, const double* h, double* Loo,
                                      double* Lov, double* Lvo, double* Lvv) {
  const int n = o + v;
  const int64_t nn = (int64_t)n * n;
  const int64_t total = (int64_t)(naux + 1) * nn;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = e / nn;
    const int r = (int)(e % nn);
    const int p = r / n, q = r % n;
    const double x = (P < naux) ? L[e] : h[r];
    if (p < o && q < o) Loo[(P * o + p) * o + q] = x;
    else if (p < o) Lov[(P * o + p) * v + (q - o)] = x;
    else if (q < o) Lvo[(P * v + (p - o)) * o + q] = x;
    else Lvv[(P * v + (p - o)) * v + (q - o)] = x;
  }
}

__global__ void trace_slices_kernel(int nslices, int o, const double* X, double* D) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < nslices; P += gridDim.x * blockDim.x) {
    double acc = 0.0;
    const double* x = X + (int64_t)P * o * o;
    for (int k = 0; k < o; ++k) acc += x[k * o + k];
    D[P] = acc;
  }
}

__global__ void trace_occ_kernel(int naux, int o, int n, const double* L, double* d) {
  for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < naux; P += gridDim.x * blockDim.x) {
    double acc = 0.0;
    const double* x = L + (int64_t)P * n * n;
    for (int k = 0; k < o; ++k) acc += x[k * n + k];
    d[P] = acc;
  }
}

__global__ __launch_bounds__(256) void energy_stage1(int o, int v, const double* __restrict__ f_ov,
                                                     const double* __restrict__ Itil, const double* __restrict__ t1,
                                                     const double* __restrict__ t2, double* partials) {
  __shared__ double sm[256];
  const int64_t ov = (int64_t)o * v;
  const int64_t N2 = ov * ov;
  const int64_t vv = (int64_t)v * v;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < N2; e += (int64_t)gridDim.x * 256) {
    const int64_t ij = e / vv;
    const int ab = (int)(e % vv);
    const int i = (int)(ij / o), j = (int)(ij % o);
    const int a = ab / v, b = ab % v;
    acc += Itil[e] * (t2[e] + t1[i * v + a] * t1[j * v + b]);
  }
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < ov; e += (int64_t)gridDim.x * 256)
    acc += 2.0 * f_ov[e] * t1[e];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void sum_partials(int nparts, const double* partials, double* out) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += partials[i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

__global__ void jacobi_kernel(int o, int v, const double* __restrict__ f_oo, const double* __restrict__ f_vv,
                              double shift, const double* __restrict__ r, double* __restrict__ t,
                              double* __restrict__ step) {
  const int64_t ov = (int64_t)o * v;
  const int64_t N = ov + ov * ov;
  const int64_t vv = (int64_t)v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    double D;
    if (e < ov) {
      const int i = (int)(e / v), a = (int)(e % v);
      D = f_vv[a * v + a] - f_oo[i * o + i];
    } else {
      const int64_t q = e - ov;
      const int64_t ij = q / vv;
      const int ab = (int)(q % vv);
      const int i = (int)(ij / o), j = (int)(ij % o);
      const int a = ab / v, b = ab % v;
      D = f_vv[a * v + a] + f_vv[b * v + b] - f_oo[i * o + i] - f_oo[j * o + j];
    }
    const double st = -r[e] / (D + shift);
    t[e] += st;
    if (step) step[e] = st;
  }
}

__global__ void scale_inv_kernel(int64_t n, const double* __restrict__ x, const double* __restrict__ s,
                                 double* __restrict__ y) {
  const double inv = *s != 0.0 ? 1.0 / *s : 0.0;  // a zero vector stays zero
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * inv;
}

__device__ inline int64_t upair(int x, int y, int n) {  // x <= y
  return (int64_t)x * n - (int64_t)x * (x - 1) / 2 + (y - x);
}
__device__ inline int64_t spair(int x, int y, int n) {  // x < y
  return (int64_t)x * (n - 1) - (int64_t)x * (x - 1) / 2 + (y - x - 1);
}
// Occupied pairs of the ladder, i <= j: the n(n-1)/2 pairs i < j first (in
// spair order), then the n diagonal pairs. The antisymmetric ladder
// vanishes on i = j for pair-symmetric t2, so its product runs over the
// first n(n-1)/2 rows only.
__device__ inline int64_t opair(int i, int j, int n) {  // i <= j
  return i < j ? spair(i, j, n) : (int64_t)n * (n - 1) / 2 + i;
}

__global__ void ppl_pack_w_kernel(int v, int a0, int na, const double* __restrict__ Wblk,
                                  const int* __restrict__ pa, const int* __restrict__ pb,
                                  const int* __restrict__ ma, const int* __restrict__ mb, double* __restrict__ S,
                                  double* __restrict__ A) {
  const int64_t P2 = (int64_t)v * (v + 1) / 2, P2m = (int64_t)v * (v - 1) / 2;
  const int64_t vv = (int64_t)v * v, v3 = vv * v;
  const int64_t p_lo = upair(a0, a0, v), p_hi = (a0 + na < v) ? upair(a0 + na, a0 + na, v) : P2;
  const int64_t m_lo = (a0 < v - 1) ? spair(a0, a0 + 1, v) : P2m;
  const int64_t m_hi = (a0 + na < v - 1) ? spair(a0 + na, a0 + na + 1, v) : P2m;
  const int64_t ns = (p_hi - p_lo) * P2, nm = (m_hi - m_lo) * P2m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns + nm; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < ns) {
      const int64_t p = p_lo + e / P2, q = e % P2;
      const int a = pa[p], b = pb[p], c = pa[q], d = pb[q];
      const double* w = Wblk + (a - a0) * v3 + (int64_t)b * vv;
      S[p * P2 + q] = w[(int64_t)c * v + d] + w[(int64_t)d * v + c];
    } else {
      const int64_t f = e - ns;
      const int64_t p = m_lo + f / P2m, q = f % P2m;
      const int a = ma[p], b = mb[p], c = ma[q], d = mb[q];
      const double* w = Wblk + (a - a0) * v3 + (int64_t)b * vv;
      A[p * P2m + q] = w[(int64_t)c * v + d] - w[(int64_t)d * v + c];
    }
  }
}

__global__ void ppl_pack_t_kernel(int o, int v, const double* __restrict__ t2, const int* __restrict__ pa,
                                  const int* __restrict__ pb, const int* __restrict__ ma,
                                  const int* __restrict__ mb, double* __restrict__ Tp, double* __restrict__ Tm) {
  const int64_t P2 = (int64_t)v * (v + 1) / 2, P2m = (int64_t)v * (v - 1) / 2;
  const int64_t O2 = (int64_t)o * (o + 1) / 2, O2m = (int64_t)o * (o - 1) / 2;
  const int64_t vv = (int64_t)v * v;
  const int64_t np = O2 * P2, nm = O2m * P2m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np + nm; e += (int64_t)gridDim.x * blockDim.x) {
    const bool plus = e < np;
    const int64_t f = plus ? e : e - np;
    const int64_t width = plus ? P2 : P2m;
    const int64_t ij = f / width, q = f % width;
    // occupied pair (i <= j) from its index (opair order)
    int i, j;
    if (ij < O2m) {
      i = 0;
      while (i + 2 < o && spair(i + 1, i + 2, o) <= ij) ++i;
      j = i + 1 + (int)(ij - spair(i, i + 1, o));
    } else {
      i = j = (int)(ij - O2m);
    }
    const double* t = t2 + ((int64_t)i * o + j) * vv;
    if (plus) {
      const int c = pa[q], d = pb[q];
      Tp[f] = (c == d) ? 0.5 * t[(int64_t)c * v + c] : 0.5 * (t[(int64_t)c * v + d] + t[(int64_t)d * v + c]);
    } else {
      const int c = ma[q], d = mb[q];
      Tm[f] = 0.5 * (t[(int64_t)c * v + d] - t[(int64_t)d * v + c]);
    }
  }
}

__global__ void ppl_unpack_kernel(int o, int v, const double* __restrict__ Rp, const double* __restrict__ Rm,
                                  double* __restrict__ R) {
  const int64_t P2 = (int64_t)v * (v + 1) / 2, P2m = (int64_t)v * (v - 1) / 2;
  const int64_t vv = (int64_t)v * v;
  const int64_t total = (int64_t)o * o * vv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ijx = e / vv;
    const int ab = (int)(e % vv);
    int i = (int)(ijx / o), j = (int)(ijx % o);
    int a = ab / v, b = ab % v;
    if (i > j) {  // X_ij^ab = X_ji^ba
      const int t = i; i = j; j = t;
      const int u = a; a = b; b = u;
    }
    const int64_t ij = opair(i, j, o);
    const bool offd = i < j;  // the antisymmetric part has rows i < j only
    double x;
    if (a <= b) {
      x = Rp[ij * P2 + upair(a, b, v)];
      if (a < b && offd) x += Rm[ij * P2m + spair(a, b, v)];
    } else {
      x = Rp[ij * P2 + upair(b, a, v)];
      if (offd) x -= Rm[ij * P2m + spair(b, a, v)];
    }
    R[e] += x;
  }
}

}  // namespace

void ppl_pack_w(int v, int a0, int na, const double* Wblk, const int* pair_a, const int* pair_b, const int* mpair_a,
                const int* mpair_b, double* S, double* A, hipStream_t s) {
  const int64_t P2 = (int64_t)v * (v + 1) / 2;
  ppl_pack_w_kernel<<<grid_for(na * (int64_t)v * P2, 32768), 256, 0, s>>>(v, a0, na, Wblk, pair_a, pair_b, mpair_a,
                                                                          mpair_b, S, A);
  PNK_CHECK_LAUNCH();
}
void ppl_pack_t(int o, int v, const double* t2, const int* pair_a, const int* pair_b, const int* mpair_a,
                const int* mpair_b, double* Tp, double* Tm, hipStream_t s) {
  const int64_t n = (int64_t)o * (o + 1) / 2 * ((int64_t)v * v);
  ppl_pack_t_kernel<<<grid_for(n, 16384), 256, 0, s>>>(o, v, t2, pair_a, pair_b, mpair_a, mpair_b, Tp, Tm);
  PNK_CHECK_LAUNCH();
}
void ppl_unpack_add(int o, int v, const double* Rp, const double* Rm, double* R, hipStream_t s) {
  const int64_t n = (int64_t)o * o * v * v;
  ppl_unpack_kernel<<<grid_for(n, 16384), 256, 0, s>>>(o, v, Rp, Rm, R);
  PNK_CHECK_LAUNCH();
}

void assemble_fock(int o, int v, const double* f_oo, const double* f_ov, const double* f_vv, double* f,
                   hipStream_t s) {
  const int n = o + v;
  assemble_fock_kernel<<<grid_for((int64_t)n * n), 256, 0, s>>>(o, v, f_oo, f_ov, f_vv, f);
  PNK_CHECK_LAUNCH();
}
void extract_occ_rows(int naux, int o, int n, const double* L, double* Lo, hipStream_t s) {
  extract_occ_rows_kernel<<<grid_for((int64_t)naux * o * n, 16384), 256, 0, s>>>(naux, o, n, L, Lo);
  PNK_CHECK_LAUNCH();
}
void extract_blocks(int naux, int o, int v, const double* L, const double* h, double* Loo, double* Lov,
                    double* Lvo, double* Lvv, hipStream_t s) {
  const int64_t n = o + v;
  extract_blocks_kernel<<<grid_for((naux + 1) * n * n, 16384), 256, 0, s>>>(naux, o, v, L, h, Loo, Lov, Lvo, Lvv);
  PNK_CHECK_LAUNCH();
}
void trace_slices(int nslices, int o, const double* X, double* D, hipStream_t s) {
  trace_slices_kernel<<<grid_for(nslices), 256, 0, s>>>(nslices, o, X, D);
  PNK_CHECK_LAUNCH();
}
void trace_occ(int naux, int o, int n, const double* L, double* d, hipStream_t s) {
  trace_occ_kernel<<<grid_for(naux), 256, 0, s>>>(naux, o, n, L, d);
  PNK_CHECK_LAUNCH();
}
void energy(int o, int v, const double* f_ov, const double* Itil, const double* t1, const double* t2, double* out,
            double* partials, hipStream_t s) {
  energy_stage1<<<kReduceBlocks, 256, 0, s>>>(o, v, f_ov, Itil, t1, t2, partials);
  sum_partials<<<1, 256, 0, s>>>(kReduceBlocks, partials, out);
  PNK_CHECK_LAUNCH();
}
void jacobi_update(int o, int v, const double* f_oo, const double* f_vv, double shift, const double* r, double* t,
                   double* step, hipStream_t s) {
  const int64_t ov = (int64_t)o * v;
  jacobi_kernel<<<grid_for(ov + ov * ov), 256, 0, s>>>(o, v, f_oo, f_vv, shift, r, t, step);
  PNK_CHECK_LAUNCH();
}
void scale_by_inverse(int64_t n, const double* x, const double* s_dev, double* y, hipStream_t s) {
  scale_inv_kernel<<<grid_for(n), 256, 0, s>>>(n, x, s_dev, y);
  PNK_CHECK_LAUNCH();
}

}  // namespace pnk
