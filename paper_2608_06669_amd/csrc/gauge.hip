// Four-index gauge transforms and the gauge's set-up (gauge.hpp).

#include "gauge.hpp"

#include <cmath>
#include <vector>

#include "gemm.hpp"

namespace pnk {

int64_t gauge_matrix_elems(int o, int v) { return 3 * ((int64_t)o * o + (int64_t)v * v); }

int64_t gauge_vector_elems(int o, int v) {
  const int64_t ov = (int64_t)o * v, n2 = ov * ov;
  return 3 * (ov + n2) + 2 * n2;
}

void gauge_apply(int o, int v, const double* Ao, const double* Av, const double* x, double* y, double* ta,
                 double* tb, hipStream_t s) {
  const int64_t O = o, V = v, ov = O * V, vv = V * V;
  PNK_REQUIRE(x != y && x != ta && x != tb && y != ta && y != tb && ta != tb, "gauge_apply: buffers overlap");
  GemmDesc d;
  // singles: Z[i][lam] = sum_a x1[i][a] Av[lam][a]; y1 = Ao Z
  d = GemmDesc();
  d.M = o; d.N = v; d.K = v;
  d.a_m = V; d.a_k = 1;
  d.b_k = 1; d.b_n = V;
  d.c_m = V; d.c_n = 1;
  gemm64(d, x, Av, ta, s);
  d = GemmDesc();
  d.M = o; d.N = v; d.K = o;
  d.a_m = O; d.a_k = 1;
  d.b_k = V; d.b_n = 1;
  d.c_m = V; d.c_n = 1;
  gemm64(d, Ao, ta, y, s);
  const double* x2 = x + ov;
  double* y2 = y + ov;
  // index b: ta[i][j][a][sig] = sum_b x2[i][j][a][b] Av[sig][b]
  d = GemmDesc();
  d.M = (int)(O * O * V); d.N = v; d.K = v;
  d.a_m = V; d.a_k = 1;
  d.b_k = 1; d.b_n = V;
  d.c_m = V; d.c_n = 1;
  gemm64(d, x2, Av, ta, s);
  // index a, per pair ij: tb[ij][lam][sig] = sum_a Av[lam][a] ta[ij][a][sig]
  d = GemmDesc();
  d.M = v; d.N = v; d.K = v;
  d.nb0 = o * o;
  d.a_m = V; d.a_k = 1; d.a_b0 = 0;
  d.b_k = V; d.b_n = 1; d.b_b0 = vv;
  d.c_m = V; d.c_n = 1; d.c_b0 = vv;
  gemm64(d, Av, ta, tb, s);
  // index j, per i: ta[i][nu][ls] = sum_j Ao[nu][j] tb[i][j][ls]
  d = GemmDesc();
  d.M = o; d.N = (int)vv; d.K = o;
  d.nb0 = o;
  d.a_m = O; d.a_k = 1; d.a_b0 = 0;
  d.b_k = vv; d.b_n = 1; d.b_b0 = O * vv;
  d.c_m = vv; d.c_n = 1; d.c_b0 = O * vv;
  gemm64(d, Ao, tb, ta, s);
  // index i: y2[mu][nu ls] = sum_i Ao[mu][i] ta[i][nu ls]
  d = GemmDesc();
  d.M = o; d.N = (int)(O * vv); d.K = o;
  d.a_m = O; d.a_k = 1;
  d.b_k = O * vv; d.b_n = 1;
  d.c_m = O * vv; d.c_n = 1;
  gemm64(d, Ao, ta, y2, s);
}

bool invert_matrix(int n, const double* A, double* Ainv) {
  std::vector<double> M((size_t)n * 2 * n, 0.0);
  double scale = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      M[(size_t)i * 2 * n + j] = A[(size_t)i * n + j];
      scale = std::max(scale, std::fabs(A[(size_t)i * n + j]));
    }
    M[(size_t)i * 2 * n + n + i] = 1.0;
  }
  if (!(scale > 0.0) || !std::isfinite(scale)) return false;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * 2 * n + c]) > std::fabs(M[(size_t)piv * 2 * n + c])) piv = r;
    const double p = M[(size_t)piv * 2 * n + c];
    if (!(std::fabs(p) > 1e-13 * scale)) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[(size_t)piv * 2 * n + j], M[(size_t)c * 2 * n + j]);
    const double ip = 1.0 / p;
    for (int j = 0; j < 2 * n; ++j) M[(size_t)c * 2 * n + j] *= ip;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[(size_t)r * 2 * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) M[(size_t)r * 2 * n + j] -= f * M[(size_t)c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ainv[(size_t)i * n + j] = M[(size_t)i * 2 * n + n + j];
  return true;
}

namespace {

// out = A B (host, row-major n x n)
void matmul(int n, const double* A, const double* B, double* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += A[(size_t)i * n + k] * B[(size_t)k * n + j];
      out[(size_t)i * n + j] = acc;
    }
}

// fwd = W^T, bwd = W^-T, F = W^T f W^-T for one block
void block_matrices(int n, const double* W, const double* f, double* fwd, double* bwd, double* F) {
  std::vector<double> Wi((size_t)n * n), tmp((size_t)n * n);
  PNK_REQUIRE(invert_matrix(n, W, Wi.data()), "gauge: W is singular or not finite");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      fwd[(size_t)i * n + j] = W[(size_t)j * n + i];
      bwd[(size_t)i * n + j] = Wi[(size_t)j * n + i];
    }
  matmul(n, fwd, f, tmp.data());
  matmul(n, tmp.data(), bwd, F);
}

}  // namespace

void gauge_setup(Gauge& g, const double* w_oo, const double* w_vv, const double* f_oo, const double* f_vv,
                 hipStream_t s) {
  const int o = g.o, v = g.v;
  const size_t oo = (size_t)o * o, vv = (size_t)v * v;
  std::vector<double> Wo(oo), Wv(vv), fo(oo), fv(vv);
  PNK_HIP(hipMemcpyAsync(Wo.data(), w_oo, oo * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(Wv.data(), w_vv, vv * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(fo.data(), f_oo, oo * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(fv.data(), f_vv, vv * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
  std::vector<double> h(3 * (oo + vv));
  double* fwd_o = h.data();
  double* bwd_o = fwd_o + oo;
  double* F_o = bwd_o + oo;
  double* fwd_v = F_o + oo;
  double* bwd_v = fwd_v + vv;
  double* F_v = bwd_v + vv;
  block_matrices(o, Wo.data(), fo.data(), fwd_o, bwd_o, F_o);
  block_matrices(v, Wv.data(), fv.data(), fwd_v, bwd_v, F_v);
  PNK_HIP(hipMemcpyAsync(g.fwd_o, fwd_o, oo * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.bwd_o, bwd_o, oo * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.Fo, F_o, oo * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.fwd_v, fwd_v, vv * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.bwd_v, bwd_v, vv * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.Fv, F_v, vv * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipStreamSynchronize(s));  // the host arrays go out of scope
}

}  // namespace pnk
