// Bandwidth-bound tensor kernels (HBM roofline): permutations, vector
// updates and deterministic reductions.

#include "tensor_ops.hpp"

namespace pnk {
namespace {

constexpr int kTile = 32;

// ---- permutation with both fastest axes different: 32 x 32 LDS tile ----
struct PermArgs {
  const double* in;
  double* out;
  int E3, Eq;         // extents of output axis 3 and output axis q
  int64_t in_s3;      // input stride of output axis 3 (input stride of q is 1)
  int64_t out_sq;     // output stride of axis q (output stride of axis 3 is 1)
  int Eu, Ew;
  int64_t in_su, in_sw, out_su, out_sw;
  int tiles3;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void permute_tiled_kernel(PermArgs p) {
  __shared__ double tile[kTile][kTile + 1];
  const int t3 = blockIdx.x % p.tiles3;
  const int tq = blockIdx.x / p.tiles3;
  const int u = blockIdx.y;
  const int w = blockIdx.z;
  const double* in = p.in + u * p.in_su + w * p.in_sw;
  double* out = p.out + u * p.out_su + w * p.out_sw;
  const int tx = threadIdx.x & 31;
  const int ty = threadIdx.x >> 5;  // 0..7
  // read: x runs along q (input-contiguous), y along axis 3
#pragma unroll
  for (int r = 0; r < kTile; r += 8) {
    const int iq = tq * kTile + tx;
    const int i3 = t3 * kTile + ty + r;
    if (iq < p.Eq && i3 < p.E3) tile[ty + r][tx] = in[(int64_t)i3 * p.in_s3 + iq];
  }
  __syncthreads();
  // write: x runs along axis 3 (output-contiguous)
#pragma unroll
  for (int r = 0; r < kTile; r += 8) {
    const int i3 = t3 * kTile + tx;
    const int iq = tq * kTile + ty + r;
    if (iq < p.Eq && i3 < p.E3) {
      double* o = out + (int64_t)iq * p.out_sq + i3;
      const double v = p.alpha * tile[tx][ty + r];
      *o = (p.beta == 0.0) ? v : v + p.beta * *o;
    }
  }
}

// ---- permutation that keeps the fastest axis: plain streaming ----
struct PermFlatArgs {
  const double* in;
  double* out;
  int od[4];
  int64_t is[4];  // input stride of each output axis
  int64_t total;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void permute_flat_kernel(PermFlatArgs p) {
  if (p.total < (1ll << 31)) {
    // the same indices in 32-bit arithmetic (64-bit division is a long
    // instruction sequence); e + stride stays below 2^32
    const uint32_t od1 = (uint32_t)p.od[1], od2 = (uint32_t)p.od[2], od3 = (uint32_t)p.od[3];
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < (uint32_t)p.total; e += gridDim.x * blockDim.x) {
      uint32_t r = e;
      const uint32_t i3 = r % od3; r /= od3;
      const uint32_t i2 = r % od2; r /= od2;
      const uint32_t i1 = r % od1; r /= od1;
      const uint32_t i0 = r;
      const double v = p.alpha * p.in[i0 * p.is[0] + i1 * p.is[1] + i2 * p.is[2] + i3 * p.is[3]];
      p.out[e] = (p.beta == 0.0) ? v : v + p.beta * p.out[e];
    }
    return;
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < p.total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int i3 = (int)(r % p.od[3]); r /= p.od[3];
    const int i2 = (int)(r % p.od[2]); r /= p.od[2];
    const int i1 = (int)(r % p.od[1]); r /= p.od[1];
    const int i0 = (int)r;
    const double v = p.alpha * p.in[i0 * p.is[0] + i1 * p.is[1] + i2 * p.is[2] + i3 * p.is[3]];
    p.out[e] = (p.beta == 0.0) ? v : v + p.beta * p.out[e];
  }
}

__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
__global__ void fill_kernel(int64_t n, double v, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void copy_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}
__global__ void cast_f32_kernel(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__global__ void cast_bf16_kernel(int64_t n, const double* __restrict__ x, uint16_t* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f32_to_bf16_rne((float)x[i]);
}
// rows x cols row-major (row length cols) to rows of length ld >= cols; the
// ld - cols padding elements of each row are zero
template <typename T>
__global__ void cast_rows_kernel(int64_t rows, int64_t cols, int64_t ld, const double* __restrict__ x, T* __restrict__ y) {
  const int64_t n = rows * ld;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ld, c = i - r * ld;
    const double v = c < cols ? x[r * cols + c] : 0.0;
    if constexpr (sizeof(T) == 2) y[i] = f32_to_bf16_rne((float)v);
    else y[i] = (float)v;
  }
}

// R[i][j][a][b] += alpha * (X[i][j][a][b] + X[j][i][b][a]); one (i,j) pair and
// one 32 x 32 (a,b) tile per block
__global__ __launch_bounds__(256) void pair_sym_kernel(int o, int v, int tiles, const double* __restrict__ X,
                                                       double alpha, double* __restrict__ R) {
  __shared__ double tile[kTile][kTile + 1];
  const int ta = blockIdx.x / tiles;  // tile along a
  const int tb = blockIdx.x % tiles;  // tile along b
  const int ij = blockIdx.y;
  const int i = ij / o, j = ij % o;
  const int64_t vv = (int64_t)v * v;
  const double* Xji = X + ((int64_t)j * o + i) * vv;
  const double* Xij = X + (int64_t)ij * vv;
  double* Rij = R + (int64_t)ij * vv;
  const int tx = threadIdx.x & 31;
  const int ty = threadIdx.x >> 5;
  // tile[b_local][a_local] = X[j][i][b][a], read along a
#pragma unroll
  for (int r = 0; r < kTile; r += 8) {
    const int b = tb * kTile + ty + r;
    const int a = ta * kTile + tx;
    if (a < v && b < v) tile[ty + r][tx] = Xji[(int64_t)b * v + a];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kTile; r += 8) {
    const int a = ta * kTile + ty + r;
    const int b = tb * kTile + tx;
    if (a < v && b < v) {
      const int64_t off = (int64_t)a * v + b;
      Rij[off] += alpha * (Xij[off] + tile[tx][ty + r]);
    }
  }
}

// ---- reductions ----
template <int OP>  // 0: dot, 1: sum of squares, 2: max |x|
__global__ __launch_bounds__(256) void reduce_stage1(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y, double* partials) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (OP == 0) acc += x[i] * y[i];
    else if (OP == 1) acc += x[i] * x[i];
    else acc = fmax(acc, fabs(x[i]));
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      if (OP == 2) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
      else sm[threadIdx.x] += sm[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

// One workgroup per vector (a grid-stride loop over the vectors); each
// vector's sum runs in the same fixed order whatever the grid.
template <int OP>  // 0: sum, 1: sqrt(sum), 2: max
__global__ __launch_bounds__(256) void reduce_stage2(int nparts, const double* partials, int stride, int nvec,
                                                     double* out) {
  __shared__ double sm[256];
  for (int vct = blockIdx.x; vct < nvec; vct += gridDim.x) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
      const double p = partials[(int64_t)i * stride + vct];
      acc = (OP == 2) ? fmax(acc, p) : acc + p;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) sm[threadIdx.x] = (OP == 2) ? fmax(sm[threadIdx.x], sm[threadIdx.x + s])
                                                       : sm[threadIdx.x] + sm[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[vct] = (OP == 1) ? sqrt(sm[0]) : sm[0];
    __syncthreads();
  }
}

constexpr int kMD = 8;  // vectors per multi-dot pass

__global__ __launch_bounds__(256) void multi_dot_stage1(int64_t n, int m, const double* __restrict__ Q, int64_t ldq,
                                                        const double* __restrict__ w, double* partials) {
  __shared__ double sm[kMD][256];
  for (int c0 = 0; c0 < m; c0 += kMD) {
    const int mc = min(kMD, m - c0);
    double acc[kMD];
#pragma unroll
    for (int q = 0; q < kMD; ++q) acc[q] = 0.0;
    // four grid-stride iterations' loads are issued before their products
    // are added, in the same order as one iteration at a time
    const int64_t st = (int64_t)gridDim.x * 256;
    constexpr int U = 4;
    for (int64_t i0 = blockIdx.x * (int64_t)256 + threadIdx.x; i0 < n; i0 += U * st) {
      double wi[U], qv[U][kMD];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + u * st;
        wi[u] = i < n ? w[i] : 0.0;
#pragma unroll
        for (int q = 0; q < kMD; ++q) qv[u][q] = (q < mc && i < n) ? Q[(int64_t)(c0 + q) * ldq + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (i0 + u * st >= n) break;
#pragma unroll
        for (int q = 0; q < kMD; ++q)
          if (q < mc) acc[q] += qv[u][q] * wi[u];
      }
    }
#pragma unroll
    for (int q = 0; q < kMD; ++q) sm[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s)
#pragma unroll
        for (int q = 0; q < kMD; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x < mc) partials[(int64_t)blockIdx.x * m + c0 + threadIdx.x] = sm[threadIdx.x][0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void multi_axpy_kernel(int64_t n, int m, const double* __restrict__ Q, int64_t ldq,
                                                         const double* __restrict__ h, double sign,
                                                         double* __restrict__ w) {
  __shared__ double hs[256];
  for (int q = threadIdx.x; q < m && q < 256; q += 256) hs[q] = h[q];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int q = 0; q < m; ++q) acc += hs[q] * Q[(int64_t)q * ldq + i];
    w[i] += sign * acc;
  }
}

__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void hash_stage1(int64_t n, const double* __restrict__ x, uint64_t* partials) {
  __shared__ uint64_t sm[256];
  uint64_t acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t bits = (uint64_t)__double_as_longlong(x[i]);
    acc += mix64(bits ^ mix64((uint64_t)i + 0x9e3779b97f4a7c15ull));
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}
__global__ __launch_bounds__(256) void hash_stage2(int nparts, const uint64_t* partials, int64_t n, uint64_t* out) {
  // integer addition is exact, so the summation order does not matter
  __shared__ uint64_t sm[256];
  uint64_t acc = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += partials[i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = mix64(sm[0] + mix64((uint64_t)n));
}

inline int grid_for(int64_t n, int cap = 4096) {
  int64_t g = ceil_div(n, 256);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

void permute4(const double* in, double* out, const int d[4], const int perm[4], double alpha, double beta,
              hipStream_t s) {
  int64_t is[4];
  is[3] = 1;
  for (int k = 2; k >= 0; --k) is[k] = is[k + 1] * d[k + 1];
  int od[4];
  for (int k = 0; k < 4; ++k) od[k] = d[perm[k]];
  const int64_t total = (int64_t)od[0] * od[1] * od[2] * od[3];
  if (total == 0) return;
  int64_t os[4];
  os[3] = 1;
  for (int k = 2; k >= 0; --k) os[k] = os[k + 1] * od[k + 1];
  int q = 0;
  for (int k = 0; k < 4; ++k)
    if (perm[k] == 3) q = k;
  if (q == 3 || od[3] == 1 || od[q] == 1) {
    PermFlatArgs p;
    p.in = in; p.out = out; p.total = total; p.alpha = alpha; p.beta = beta;
    for (int k = 0; k < 4; ++k) { p.od[k] = od[k]; p.is[k] = is[perm[k]]; }
    permute_flat_kernel<<<grid_for(total, 16384), 256, 0, s>>>(p);
    PNK_CHECK_LAUNCH();
    return;
  }
  int rest[2], nr = 0;
  for (int k = 0; k < 3; ++k)
    if (k != q) rest[nr++] = k;
  PermArgs p;
  p.in = in; p.out = out;
  p.E3 = od[3]; p.Eq = od[q];
  p.in_s3 = is[perm[3]];
  p.out_sq = os[q];
  p.Eu = od[rest[0]]; p.Ew = od[rest[1]];
  p.in_su = is[perm[rest[0]]]; p.in_sw = is[perm[rest[1]]];
  p.out_su = os[rest[0]]; p.out_sw = os[rest[1]];
  p.tiles3 = (int)ceil_div(p.E3, kTile);
  p.alpha = alpha; p.beta = beta;
  const int64_t gx = (int64_t)p.tiles3 * ceil_div(p.Eq, kTile);
  PNK_REQUIRE(p.Eu <= 65535 && p.Ew <= 65535 && gx < (1ll << 31), "permute4: extents too large");
  permute_tiled_kernel<<<dim3((unsigned)gx, p.Eu, p.Ew), 256, 0, s>>>(p);
  PNK_CHECK_LAUNCH();
}

void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n <= 0) return;
  axpby_kernel<<<grid_for(n), 256, 0, s>>>(n, a, x, b, y);
  PNK_CHECK_LAUNCH();
}
void fill(int64_t n, double v, double* y, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<<<grid_for(n), 256, 0, s>>>(n, v, y);
  PNK_CHECK_LAUNCH();
}
void copy(int64_t n, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  copy_kernel<<<grid_for(n), 256, 0, s>>>(n, x, y);
  PNK_CHECK_LAUNCH();
}
void cast_f64_to_f32(int64_t n, const double* x, float* y, hipStream_t s) {
  if (n <= 0) return;
  cast_f32_kernel<<<grid_for(n, 16384), 256, 0, s>>>(n, x, y);
  PNK_CHECK_LAUNCH();
}
void cast_f64_to_bf16(int64_t n, const double* x, uint16_t* y, hipStream_t s) {
  if (n <= 0) return;
  cast_bf16_kernel<<<grid_for(n, 16384), 256, 0, s>>>(n, x, y);
  PNK_CHECK_LAUNCH();
}
void cast_f64_to_f32_rows(int64_t rows, int64_t cols, int64_t ld, const double* x, float* y, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  cast_rows_kernel<float><<<grid_for(rows * ld, 16384), 256, 0, s>>>(rows, cols, ld, x, y);
  PNK_CHECK_LAUNCH();
}
void cast_f64_to_bf16_rows(int64_t rows, int64_t cols, int64_t ld, const double* x, uint16_t* y, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  cast_rows_kernel<uint16_t><<<grid_for(rows * ld, 16384), 256, 0, s>>>(rows, cols, ld, x, y);
  PNK_CHECK_LAUNCH();
}

void pair_symmetrize_add(int o, int v, const double* X, double alpha, double* R, hipStream_t s) {
  if (o <= 0 || v <= 0) return;
  const int tiles = (int)ceil_div(v, kTile);
  PNK_REQUIRE((int64_t)o * o <= 65535, "pair_symmetrize_add: too many pairs");
  pair_sym_kernel<<<dim3(tiles * tiles, o * o), 256, 0, s>>>(o, v, tiles, X, alpha, R);
  PNK_CHECK_LAUNCH();
}

int64_t reduce_partials_size(int nvec) { return (int64_t)kReduceBlocks * (nvec < 1 ? 1 : nvec); }

void dot(int64_t n, const double* x, const double* y, double* out, double* partials, hipStream_t s) {
  reduce_stage1<0><<<kReduceBlocks, 256, 0, s>>>(n, x, y, partials);
  reduce_stage2<0><<<1, 256, 0, s>>>(kReduceBlocks, partials, 1, 1, out);
  PNK_CHECK_LAUNCH();
}
void nrm2(int64_t n, const double* x, double* out, double* partials, hipStream_t s) {
  reduce_stage1<1><<<kReduceBlocks, 256, 0, s>>>(n, x, nullptr, partials);
  reduce_stage2<1><<<1, 256, 0, s>>>(kReduceBlocks, partials, 1, 1, out);
  PNK_CHECK_LAUNCH();
}
void nrm_inf(int64_t n, const double* x, double* out, double* partials, hipStream_t s) {
  reduce_stage1<2><<<kReduceBlocks, 256, 0, s>>>(n, x, nullptr, partials);
  reduce_stage2<2><<<1, 256, 0, s>>>(kReduceBlocks, partials, 1, 1, out);
  PNK_CHECK_LAUNCH();
}
void multi_dot(int64_t n, int m, const double* Q, int64_t ldq, const double* w, double* out, double* partials,
               hipStream_t s) {
  if (m <= 0) return;
  multi_dot_stage1<<<kReduceBlocks, 256, 0, s>>>(n, m, Q, ldq, w, partials);
  reduce_stage2<0><<<m, 256, 0, s>>>(kReduceBlocks, partials, m, m, out);
  PNK_CHECK_LAUNCH();
}
void multi_axpy(int64_t n, int m, const double* Q, int64_t ldq, const double* h, double* w, hipStream_t s) {
  if (m <= 0) return;
  PNK_REQUIRE(m <= 256, "multi_axpy: at most 256 vectors");
  multi_axpy_kernel<<<grid_for(n), 256, 0, s>>>(n, m, Q, ldq, h, -1.0, w);
  PNK_CHECK_LAUNCH();
}
void combine(int64_t n, int m, const double* Q, int64_t ldq, const double* y, double sign, double* x,
             hipStream_t s) {
  if (m <= 0) return;
  PNK_REQUIRE(m <= 256, "combine: at most 256 vectors");
  multi_axpy_kernel<<<grid_for(n), 256, 0, s>>>(n, m, Q, ldq, y, sign, x);
  PNK_CHECK_LAUNCH();
}
void hash64(int64_t n, const double* x, uint64_t* out, uint64_t* partials, hipStream_t s) {
  hash_stage1<<<kReduceBlocks, 256, 0, s>>>(n, x, partials);
  hash_stage2<<<1, 256, 0, s>>>(kReduceBlocks, partials, n, out);
  PNK_CHECK_LAUNCH();
}

}  // namespace pnk
