// Four-index gauge transforms and the gauge's set-up (gauge.hpp).

#include "gauge.hpp"

#include <cmath>
#include <vector>

#include "gemm.hpp"

namespace pnk {

int64_t gauge_matrix_elems(int o, int v, int mo, int mv) {
  return 2 * ((int64_t)o * mo + (int64_t)v * mv) + (int64_t)mo * mo + (int64_t)mv * mv;
}

int64_t gauge_vector_elems(int o, int v, int mo, int mv) {
  const int64_t ov = (int64_t)o * v, n = ov + ov * ov;
  const int64_t mm = (int64_t)mo * mv, ng = mm + mm * mm;
  return 3 * n + ng + 2 * mm * mm;
}

void gauge_apply(int qo, int qv, int po, int pv, const double* Ao, const double* Av, const double* x1,
                 const double* x2, double* y1, double* y2, double* ta, double* tb, hipStream_t s) {
  const int64_t QO = qo, QV = qv, PO = po, PV = pv, pvv = PV * PV;
  PNK_REQUIRE(x1 != y1 && x2 != y2 && x2 != ta && x2 != tb && y2 != ta && y2 != tb && ta != tb,
              "gauge_apply: buffers overlap");
  GemmDesc d;
  // singles: Z[i][lam] = sum_a x1[i][a] Av[lam][a]; y1 = Ao Z
  d = GemmDesc();
  d.M = qo; d.N = pv; d.K = qv;
  d.a_m = QV; d.a_k = 1;
  d.b_k = 1; d.b_n = QV;
  d.c_m = PV; d.c_n = 1;
  gemm64(d, x1, Av, ta, s);
  d = GemmDesc();
  d.M = po; d.N = pv; d.K = qo;
  d.a_m = QO; d.a_k = 1;
  d.b_k = PV; d.b_n = 1;
  d.c_m = PV; d.c_n = 1;
  gemm64(d, Ao, ta, y1, s);
  // index b: ta[i][j][a][sig] = sum_b x2[i][j][a][b] Av[sig][b]
  d = GemmDesc();
  d.M = (int)(QO * QO * QV); d.N = pv; d.K = qv;
  d.a_m = QV; d.a_k = 1;
  d.b_k = 1; d.b_n = QV;
  d.c_m = PV; d.c_n = 1;
  gemm64(d, x2, Av, ta, s);
  // index a, per pair ij: tb[ij][lam][sig] = sum_a Av[lam][a] ta[ij][a][sig]
  d = GemmDesc();
  d.M = pv; d.N = pv; d.K = qv;
  d.nb0 = qo * qo;
  d.a_m = QV; d.a_k = 1; d.a_b0 = 0;
  d.b_k = PV; d.b_n = 1; d.b_b0 = QV * PV;
  d.c_m = PV; d.c_n = 1; d.c_b0 = pvv;
  gemm64(d, Av, ta, tb, s);
  // index j, per i: ta[i][nu][ls] = sum_j Ao[nu][j] tb[i][j][ls]
  d = GemmDesc();
  d.M = po; d.N = (int)pvv; d.K = qo;
  d.nb0 = qo;
  d.a_m = QO; d.a_k = 1; d.a_b0 = 0;
  d.b_k = pvv; d.b_n = 1; d.b_b0 = QO * pvv;
  d.c_m = pvv; d.c_n = 1; d.c_b0 = PO * pvv;
  gemm64(d, Ao, tb, ta, s);
  // index i: y2[mu][nu ls] = sum_i Ao[mu][i] ta[i][nu ls]
  d = GemmDesc();
  d.M = po; d.N = (int)(PO * pvv); d.K = qo;
  d.a_m = QO; d.a_k = 1;
  d.b_k = PO * pvv; d.b_n = 1;
  d.c_m = PO * pvv; d.c_n = 1;
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

// out = A B (host, row-major; A n x k, B k x m)
void matmul(int n, int k, int m, const double* A, const double* B, double* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      double acc = 0.0;
      for (int q = 0; q < k; ++q) acc += A[(size_t)i * k + q] * B[(size_t)q * m + j];
      out[(size_t)i * m + j] = acc;
    }
}

// One block with W [n][m]: fwd = W^T [m][n], bwd = C^T [n][m] and
// F = W^T f C^T [m][m], C = W^+. For square W, C^T = W^-T from the inverse
// of W itself; otherwise C^T = (W W^T)^-1 W (W of full row rank makes
// W W^T positive definite).
void block_matrices(int n, int m, const double* W, const double* f, double* fwd, double* bwd, double* F) {
  for (int mu = 0; mu < m; ++mu)
    for (int i = 0; i < n; ++i) fwd[(size_t)mu * n + i] = W[(size_t)i * m + mu];
  if (m == n) {
    std::vector<double> Wi((size_t)n * n);
    PNK_REQUIRE(invert_matrix(n, W, Wi.data()), "gauge: W is singular or not finite");
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) bwd[(size_t)i * n + j] = Wi[(size_t)j * n + i];
  } else {
    std::vector<double> G((size_t)n * n), Gi((size_t)n * n);
    matmul(n, m, n, W, fwd, G.data());
    PNK_REQUIRE(invert_matrix(n, G.data(), Gi.data()), "gauge: W is not of full row rank or not finite");
    matmul(n, n, m, Gi.data(), W, bwd);
  }
  std::vector<double> tmp((size_t)m * n);
  matmul(m, n, n, fwd, f, tmp.data());
  matmul(m, n, m, tmp.data(), bwd, F);
}

}  // namespace

void gauge_setup(Gauge& g, const double* w_oo, const double* w_vv, const double* f_oo, const double* f_vv,
                 hipStream_t s) {
  const int o = g.o, v = g.v, mo = g.mo, mv = g.mv;
  const size_t oo = (size_t)o * o, vv = (size_t)v * v, om = (size_t)o * mo, vm = (size_t)v * mv;
  const size_t mmo = (size_t)mo * mo, mmv = (size_t)mv * mv;
  std::vector<double> Wo(om), Wv(vm), fo(oo), fv(vv);
  PNK_HIP(hipMemcpyAsync(Wo.data(), w_oo, om * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(Wv.data(), w_vv, vm * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(fo.data(), f_oo, oo * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipMemcpyAsync(fv.data(), f_vv, vv * sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
  std::vector<double> h(2 * (om + vm) + mmo + mmv);
  double* fwd_o = h.data();
  double* bwd_o = fwd_o + om;
  double* F_o = bwd_o + om;
  double* fwd_v = F_o + mmo;
  double* bwd_v = fwd_v + vm;
  double* F_v = bwd_v + vm;
  block_matrices(o, mo, Wo.data(), fo.data(), fwd_o, bwd_o, F_o);
  block_matrices(v, mv, Wv.data(), fv.data(), fwd_v, bwd_v, F_v);
  PNK_HIP(hipMemcpyAsync(g.fwd_o, fwd_o, om * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.bwd_o, bwd_o, om * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.Fo, F_o, mmo * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.fwd_v, fwd_v, vm * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.bwd_v, bwd_v, vm * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipMemcpyAsync(g.Fv, F_v, mmv * sizeof(double), hipMemcpyHostToDevice, s));
  PNK_HIP(hipStreamSynchronize(s));  // the host arrays go out of scope
}

}  // namespace pnk
