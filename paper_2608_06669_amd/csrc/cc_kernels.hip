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
  const double inv = 1.0 / *s;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * inv;
}

}  // namespace

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
