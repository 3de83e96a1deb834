// C boundary of the library (include/pnkcc.h): argument checks, workspace
// management, problem caching and status codes.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pnkcc.h"
#include "api_internal.hpp"
#include "eig.hpp"
#include "fock_op.hpp"
#include "gauge.hpp"
#include "gemm.hpp"
#include "tensor_ops.hpp"

using namespace pnk;

namespace pnk {

size_t workspace_bytes(int o, int v, int naux, int lowp, int m_max, int restart, int diis, int64_t outer_cap) {
  EngineOptions eo;
  eo.lowp_f32 = lowp & 1;
  eo.lowp_bf16 = (lowp >> 1) & 1;
  const int64_t nvec = (int64_t)o * v + (int64_t)o * o * v * v;
  return engine_bytes(o, v, naux, eo) + Solver::bytes(nvec, m_max, restart, diis, outer_cap) +
         2 * nvec * sizeof(double);
}

void check_problem(const cc_problem* p) {
  PNK_REQUIRE(p != nullptr, "problem is NULL");
  PNK_REQUIRE(p->nocc > 0 && p->nvir > 0 && p->naux > 0, "nocc, nvir and naux must be positive");
  PNK_REQUIRE(p->f_oo && p->f_ov && p->f_vv && p->L, "problem arrays must not be NULL");
  PNK_REQUIRE(p->nocc <= 255, "nocc above 255 is not supported");
  const int64_t ov = (int64_t)p->nocc * p->nvir;
  PNK_REQUIRE(ov <= 46000, "nocc * nvir above 46000 is not supported");
  PNK_REQUIRE((int64_t)p->nvir * p->nvir <= 1000000, "nvir above 1000 is not supported");
}

void* Handle::dev_alloc(size_t bytes) {
  void* p = nullptr;
  hipError_t e = stream_ordered ? hipMallocAsync(&p, bytes, alloc_stream) : hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw OomError("device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void Handle::dev_free(void* p) {
  if (!p) return;
  (void)(stream_ordered ? hipFreeAsync(p, alloc_stream) : hipFree(p));
}

Handle::~Handle() {
  sol.reset();
  eng.reset();
  dev_free(xa);
  dev_free(xb);
  dev_free(hash_buf);
  dev_free(gauge_mem);
}

Gauge* Handle::ensure_gauge(const cc_gauge* g, hipStream_t s) {
  PNK_REQUIRE(g && g->w_oo && g->w_vv, "gauge matrices must not be NULL");
  const int o = eng->o(), v = eng->v();
  PNK_REQUIRE(g->m_occ >= 0 && g->m_vir >= 0, "gauge sizes must not be negative");
  const int mo = g->m_occ ? g->m_occ : o, mv = g->m_vir ? g->m_vir : v;
  PNK_REQUIRE(mo >= o && mv >= v, "a gauge needs at least as many functions as its block has orbitals");
  PNK_REQUIRE(mo <= 255 && (int64_t)mo * mv <= 46000 && (int64_t)mv * mv <= 1000000,
              "gauge sizes above m_occ 255, m_occ m_vir 46000 or m_vir 1000 are not supported");
  const int64_t ng = (int64_t)mo * mv + (int64_t)mo * mo * mv * mv;
  const int lowp = (eng->options().lowp_f32 ? 1 : 0) | (eng->options().lowp_bf16 ? 2 : 0);
  const int64_t cap = std::max(sol_cap, ng);
  const int64_t me = gauge_matrix_elems(o, v, mo, mv), ve = gauge_vector_elems(o, v, mo, mv);
  const size_t gbytes = (size_t)(me + ve) * sizeof(double) + 16 * 256;
  if (limit && workspace_bytes(o, v, eng->naux(), lowp, sol_m, sol_r, sol_d, cap) + gbytes > limit)
    throw OomError("the gauge buffers (" + std::to_string(gbytes) + " bytes) and solver vectors of length " +
                   std::to_string(ng) + " exceed the handle limit");
  if (!gauge_mem || gauge.o != o || gauge.v != v || gauge.mo != mo || gauge.mv != mv) {
    dev_free(gauge_mem);
    gauge_mem = nullptr;
    gauge_mem = (double*)dev_alloc(gbytes);
    // 256-byte aligned pieces
    char* base = (char*)gauge_mem;
    auto take = [&](int64_t elems) {
      double* p = (double*)base;
      base += ((size_t)elems * sizeof(double) + 255) & ~(size_t)255;
      return p;
    };
    const int64_t ov = (int64_t)o * v, n = ov + ov * ov, mm = (int64_t)mo * mv;
    gauge.o = o;
    gauge.v = v;
    gauge.mo = mo;
    gauge.mv = mv;
    gauge.fwd_o = take((int64_t)o * mo); gauge.bwd_o = take((int64_t)o * mo); gauge.Fo = take((int64_t)mo * mo);
    gauge.fwd_v = take((int64_t)v * mv); gauge.bwd_v = take((int64_t)v * mv); gauge.Fv = take((int64_t)mv * mv);
    gauge.t = take(n); gauge.w1 = take(n); gauge.w2 = take(n);
    gauge.xg = take(ng); gauge.ta = take(mm * mm); gauge.tb = take(mm * mm);
  }
  if (sol->outer_capacity() < ng) {
    // the outer Krylov and DIIS vectors of a redundant gauge are longer
    // than the orbital ones
    sol.reset();
    sol = std::make_unique<Solver>(*eng, sol_m, sol_r, sol_d, alloc_stream, stream_ordered, ng);
    sol_cap = ng;
  }
  gauge_setup(gauge, g->w_oo, g->w_vv, eng->f_oo(), eng->f_vv(), s);
  return &gauge;
}

void Handle::ensure(const cc_problem* p, int lowp, int m_max, int restart, int diis, hipStream_t s) {
  check_problem(p);
  PNK_HIP(hipSetDevice(device));
  const int o = p->nocc, v = p->nvir, naux = p->naux;
  const bool want32 = (lowp & 1) || (eng && eng->options().lowp_f32 && eng->o() == o && eng->v() == v &&
                                     eng->naux() == naux);
  const bool want16 = ((lowp >> 1) & 1) || (eng && eng->options().lowp_bf16 && eng->o() == o && eng->v() == v &&
                                            eng->naux() == naux);
  const bool same_shape = eng && eng->o() == o && eng->v() == v && eng->naux() == naux;
  const bool have_lowp = same_shape && (!want32 || eng->options().lowp_f32) && (!want16 || eng->options().lowp_bf16);
  const bool have_solver = sol && same_shape && sol_m >= m_max && sol_r >= restart && sol_d >= diis;
  if (!same_shape || !have_lowp || !have_solver) {
    const int M = std::max(m_max, same_shape && sol ? sol_m : 0);
    const int R = std::max(restart, same_shape && sol ? sol_r : 0);
    const int Dd = std::max(diis, same_shape && sol ? sol_d : 0);
    const int lp = (want32 ? 1 : 0) | (want16 ? 2 : 0);
    // outer vectors keep a redundant gauge's length once one has been used
    const int64_t cap = same_shape ? sol_cap : 0;
    const size_t need = workspace_bytes(o, v, naux, lp, M, R, Dd, cap);
    if (limit && need > limit)
      throw OomError("problem needs " + std::to_string(need) + " workspace bytes; the handle limit is " +
                     std::to_string(limit));
    if (!same_shape || !have_lowp) {
      sol.reset();
      eng.reset();
      dev_free(xa);
      dev_free(xb);
      xa = xb = nullptr;
      EngineOptions eo;
      eo.lowp_f32 = want32;
      eo.lowp_bf16 = want16;
      eo.alloc_stream = alloc_stream;
      eo.stream_ordered = stream_ordered;
      eng = std::make_unique<Engine>(o, v, naux, eo);
      eng->set_timers(timers.get());
      prepared = false;
      const int64_t n = eng->nvec();
      xa = (double*)dev_alloc(n * sizeof(double));
      xb = (double*)dev_alloc(n * sizeof(double));
    }
    sol.reset();
    sol = std::make_unique<Solver>(*eng, M, R, Dd, alloc_stream, stream_ordered, cap);
    sol_cap = cap;
    sol_m = M;
    sol_r = R;
    sol_d = Dd;
  }
  if (!hash_buf) hash_buf = (uint64_t*)dev_alloc((kReduceBlocks + 8) * sizeof(uint64_t));
  // content key of the problem
  const int64_t n = o + v;
  uint64_t* parts = hash_buf + 8;
  hash64((int64_t)o * o, p->f_oo, hash_buf + 0, parts, s);
  hash64((int64_t)o * v, p->f_ov, hash_buf + 1, parts, s);
  hash64((int64_t)v * v, p->f_vv, hash_buf + 2, parts, s);
  hash64((int64_t)naux * n * n, p->L, hash_buf + 3, parts, s);
  uint64_t hv[4];
  PNK_HIP(hipMemcpyAsync(hv, hash_buf, sizeof(hv), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
  ProblemKey key{o, v, naux, p->f_oo, p->f_ov, p->f_vv, p->L, {hv[0], hv[1], hv[2], hv[3]}};
  if (!prepared || !(key == cached_key)) {
    ProblemView pv;
    pv.o = o; pv.v = v; pv.naux = naux;
    pv.f_oo = p->f_oo; pv.f_ov = p->f_ov; pv.f_vv = p->f_vv; pv.L = p->L;
    eng->prepare(pv, s);
    cached_key = key;
    prepared = true;
  }
}

void pack(int64_t ov, int64_t n2, const double* a1, const double* a2, double* x, hipStream_t s) {
  PNK_HIP(hipMemcpyAsync(x, a1, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
  PNK_HIP(hipMemcpyAsync(x + ov, a2, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
}
void unpack(int64_t ov, int64_t n2, const double* x, double* a1, double* a2, hipStream_t s) {
  PNK_HIP(hipMemcpyAsync(a1, x, ov * sizeof(double), hipMemcpyDeviceToDevice, s));
  PNK_HIP(hipMemcpyAsync(a2, x + ov, n2 * sizeof(double), hipMemcpyDeviceToDevice, s));
}

PnkOptions to_internal(const cc_pnk_opts& o) {
  PnkOptions r;
  r.tol_inf = o.tol_inf;
  r.max_newton = o.max_newton;
  r.m_max = o.m_max;
  r.gamma = o.gamma;
  r.alpha = o.alpha;
  r.eta0 = o.eta0;
  r.eta_max = o.eta_max;
  r.inner_rtol = o.inner_rtol;
  r.inner_maxit = o.inner_maxit;
  r.inner_restart = o.inner_restart;
  r.jvp_prec = (Prec)o.jvp_prec;
  r.use_fd_jvp = o.use_fd_jvp != 0;
  r.init_mp2 = o.init_mp2 != 0;
  r.protocol = (int)o.protocol;
  r.ccd = o.ccd != 0;
  r.stall_window = o.stall_window;
  r.stall_factor = o.stall_factor;
  r.inner_rtol_jv = o.inner_rtol_jv;
  return r;
}

void check_pnk_opts(const cc_pnk_opts& o) {
  PNK_REQUIRE(o.tol_inf > 0 && std::isfinite(o.tol_inf), "tol_inf must be positive");
  PNK_REQUIRE(o.max_newton >= 0, "max_newton must be >= 0");
  PNK_REQUIRE(o.m_max >= 1 && o.m_max <= 200, "m_max must be in 1..200");
  PNK_REQUIRE(o.inner_restart >= 1 && o.inner_restart <= 200, "inner_restart must be in 1..200");
  PNK_REQUIRE(o.inner_maxit >= 1, "inner_maxit must be >= 1");
  PNK_REQUIRE(o.inner_rtol > 0 && o.inner_rtol < 1, "inner_rtol must be in (0, 1)");
  PNK_REQUIRE(o.jvp_prec == CC_FP64 || o.jvp_prec == CC_FP32 || o.jvp_prec == CC_BF16, "unknown jvp_prec");
  PNK_REQUIRE(!(o.use_fd_jvp && o.jvp_prec != CC_FP64), "the finite-difference product is FP64 only");
  PNK_REQUIRE(o.eta_max > 0 && o.eta_max < 1 && o.eta0 > 0 && o.eta0 < 1, "forcing terms must be in (0, 1)");
  PNK_REQUIRE(o.protocol == CC_PNK || o.protocol == CC_NK || o.protocol == CC_INK, "unknown protocol");
  PNK_REQUIRE(o.stall_window >= 0, "stall_window must be >= 0");
  PNK_REQUIRE(o.stall_window == 0 || (o.stall_factor > 0 && o.stall_factor < 1), "stall_factor must be in (0, 1)");
  PNK_REQUIRE(o.inner_rtol_jv == 0 || (o.inner_rtol_jv > 0 && o.inner_rtol_jv < 1), "inner_rtol_jv must be 0 or in (0, 1)");
}

int lowp_for(cc_precision p) { return p == CC_FP32 ? 1 : (p == CC_BF16 ? 2 : 0); }

}  // namespace pnk

#define PNK_API_BEGIN(hp)                                   \
  if (!(hp)) return CC_ERR_ARG;                             \
  Handle* H = reinterpret_cast<Handle*>(hp);                \
  H->err.clear();                                           \
  try {
#define PNK_API_END                                         \
  }                                                         \
  catch (const ArgError& e) { H->err = e.what(); return CC_ERR_ARG; } \
  catch (const OomError& e) { H->err = e.what(); return CC_ERR_OOM; } \
  catch (const HipError& e) { H->err = e.what(); return CC_ERR_HIP; } \
  catch (const std::exception& e) { H->err = e.what(); return CC_ERR_INTERNAL; }

extern "C" {

cc_status cc_create(cc_handle** h, int device, size_t workspace_limit_bytes) {
  if (!h) return CC_ERR_ARG;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return CC_ERR_HIP;
  }
  Handle* H = new (std::nothrow) Handle();
  if (!H) return CC_ERR_OOM;
  H->device = device;
  H->limit = workspace_limit_bytes;
  *h = reinterpret_cast<cc_handle*>(H);
  return CC_OK;
}

void cc_destroy(cc_handle* h) {
  if (!h) return;
  Handle* H = reinterpret_cast<Handle*>(h);
  (void)hipSetDevice(H->device);
  delete H;
}

const char* cc_last_error(const cc_handle* h) {
  if (!h) return "null handle";
  return reinterpret_cast<const Handle*>(h)->err.c_str();
}

size_t cc_workspace_bytes(int32_t nocc, int32_t nvir, int32_t naux, int lowp_flags, int m_max, int inner_restart,
                          int diis_size) {
  if (nocc <= 0 || nvir <= 0 || naux <= 0 || m_max < 1 || inner_restart < 1 || diis_size < 0) return 0;
  return workspace_bytes(nocc, nvir, naux, lowp_flags, m_max, inner_restart, diis_size);
}

void cc_pnk_opts_default(cc_pnk_opts* o) {
  if (!o) return;
  o->tol_inf = 1e-8;
  o->max_newton = 100;
  o->m_max = 20;
  o->gamma = 0.9;
  o->alpha = 1.5;
  o->eta0 = 0.5;
  o->eta_max = 0.9;
  o->inner_rtol = 1e-12;
  o->inner_maxit = 200;
  o->inner_restart = 30;
  o->jvp_prec = CC_FP64;
  o->use_fd_jvp = 0;
  o->init_mp2 = 1;
  o->protocol = CC_PNK;
  o->ccd = 0;
  o->stall_window = 0;
  o->stall_factor = 0.5;
  o->inner_rtol_jv = 0.0;
}

void cc_fp_opts_default(cc_fp_opts* o) {
  if (!o) return;
  o->tol_inf = 1e-8;
  o->max_iter = 500;
  o->diis_size = 8;
  o->diis_start = 2;
  o->level_shift = 0.0;
  o->init_mp2 = 1;
  o->ccd = 0;
}

cc_status cc_residual(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, double* r1, double* r2,
                      double* e_corr_host, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2 && r1 && r2, "t1, t2, r1, r2 must not be NULL");
  H->ensure(p, 0, 1, 1, 0, s);
  H->eng->residual(t1, t2, r1, r2, s);
  if (e_corr_host) {
    H->eng->energy(t1, t2, H->eng->scratch_partials() + 1024, s);
    PNK_HIP(hipMemcpyAsync(e_corr_host, H->eng->scratch_partials() + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
    PNK_HIP(hipStreamSynchronize(s));
  }
  return CC_OK;
  PNK_API_END
}

cc_status cc_energy(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, double* e_corr_host,
                    void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2 && e_corr_host, "t1, t2, e_corr_host must not be NULL");
  H->ensure(p, 0, 1, 1, 0, s);
  H->eng->energy(t1, t2, H->eng->scratch_partials() + 1024, s);
  PNK_HIP(hipMemcpyAsync(e_corr_host, H->eng->scratch_partials() + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
  return CC_OK;
  PNK_API_END
}

cc_status cc_jvp(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, const double* v1,
                 const double* v2, double* jv1, double* jv2, cc_precision prec, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2 && v1 && v2 && jv1 && jv2, "array arguments must not be NULL");
  PNK_REQUIRE(prec == CC_FP64 || prec == CC_FP32 || prec == CC_BF16, "unknown precision");
  H->ensure(p, lowp_for(prec), 1, 1, 0, s);
  // linearise at t: the residual goes to the handle's scratch vector
  const int64_t ov = H->eng->o() * (int64_t)H->eng->v();
  H->eng->residual(t1, t2, H->xa, H->xa + ov, s);
  H->eng->jvp(v1, v2, jv1, jv2, (Prec)prec, s);
  return CC_OK;
  PNK_API_END
}

cc_status cc_fock_apply(cc_handle* h, const cc_problem* p, const double* x1, const double* x2, double* y1,
                        double* y2, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(x1 && x2 && y1 && y2, "array arguments must not be NULL");
  H->ensure(p, 0, 1, 1, 0, s);
  H->eng->fock_apply(x1, x2, y1, y2, s);
  return CC_OK;
  PNK_API_END
}

static cc_status precond_solve_impl(cc_handle* h, const cc_problem* p, const double* b1, const double* b2,
                                    double* x1, double* x2, double rtol, int maxit, int* iters_out, void* stream,
                                    bool pair_symmetric) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(b1 && b2 && x1 && x2, "array arguments must not be NULL");
  PNK_REQUIRE(rtol > 0 && rtol < 1 && maxit >= 1, "rtol must be in (0, 1) and maxit >= 1");
  H->ensure(p, 0, 1, 30, 0, s);
  const int64_t ov = H->eng->o() * (int64_t)H->eng->v(), n2 = H->eng->nvec() - ov;
  pack(ov, n2, b1, b2, H->xb, s);
  bool conv = true;
  const int it = H->sol->precond_solve(H->xb, H->xa, rtol, maxit, 30, s, &conv, pair_symmetric);
  unpack(ov, n2, H->xa, x1, x2, s);
  PNK_HIP(hipStreamSynchronize(s));
  if (iters_out) *iters_out = it;
  return conv ? CC_OK : CC_NOT_CONVERGED;
  PNK_API_END
}

cc_status cc_precond_solve(cc_handle* h, const cc_problem* p, const double* b1, const double* b2, double* x1,
                           double* x2, double rtol, int maxit, int* iters_out, void* stream) {
  return precond_solve_impl(h, p, b1, b2, x1, x2, rtol, maxit, iters_out, stream, false);
}

cc_status cc_precond_solve_pairsym(cc_handle* h, const cc_problem* p, const double* b1, const double* b2, double* x1,
                                   double* x2, double rtol, int maxit, int* iters_out, void* stream) {
  return precond_solve_impl(h, p, b1, b2, x1, x2, rtol, maxit, iters_out, stream, true);
}

cc_status cc_fp_spectral_radius(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, const double* q1,
                                const double* q2, double shift, int m, double* rho_out, double* ritz_re,
                                double* ritz_im, int* n_ritz, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2 && q1 && q2 && rho_out, "array arguments must not be NULL");
  PNK_REQUIRE(m >= 1 && m <= 200, "m must be in 1..200");
  PNK_REQUIRE(std::isfinite(shift), "shift must be finite");
  H->ensure(p, 0, m, 1, 0, s);
  const int64_t ov = H->eng->o() * (int64_t)H->eng->v(), n2 = H->eng->nvec() - ov;
  pack(ov, n2, t1, t2, H->xa, s);
  pack(ov, n2, q1, q2, H->xb, s);
  std::vector<double> re, im;
  *rho_out = H->sol->fp_spectral_radius(H->xa, H->xb, shift, m, s, &re, &im);
  for (size_t i = 0; i < re.size(); ++i) {
    if (ritz_re) ritz_re[i] = re[i];
    if (ritz_im) ritz_im[i] = im[i];
  }
  if (n_ritz) *n_ritz = (int)re.size();
  return CC_OK;
  PNK_API_END
}

static void fill_info(const SolveStats& st, cc_info* info) {
  if (!info) return;
  info->e_corr = st.e_corr;
  info->res_inf = st.res_inf;
  info->res_2 = st.res_2;
  info->converged = st.converged;
  info->newton_iters = st.newton_iters;
  info->n_residual = st.n_residual;
  info->n_jvp = st.n_jvp;
  info->n_afmv = st.n_afmv;
  info->n_inner_iters = st.n_inner_iters;
  info->seconds = st.seconds;
  info->stalled = st.stalled;
}

cc_status cc_solve_pnk(cc_handle* h, const cc_problem* p, const cc_pnk_opts* opts, double* t1, double* t2,
                       cc_info* info, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2, "t1, t2 must not be NULL");
  cc_pnk_opts o;
  cc_pnk_opts_default(&o);
  if (opts) o = *opts;
  check_pnk_opts(o);
  H->ensure(p, lowp_for(o.jvp_prec), o.m_max, o.inner_restart, 0, s);
  const int64_t ov = H->eng->o() * (int64_t)H->eng->v(), n2 = H->eng->nvec() - ov;
  if (!o.init_mp2) pack(ov, n2, t1, t2, H->xa, s);
  SolveStats st;
  H->sol->solve_pnk(H->xa, to_internal(o), &st, s);
  unpack(ov, n2, H->xa, t1, t2, s);
  PNK_HIP(hipStreamSynchronize(s));
  H->history = H->sol->history();
  fill_info(st, info);
  if (st.diverged) { H->err = "non-finite residual norm"; return CC_ERR_NAN; }
  return st.converged ? CC_OK : CC_NOT_CONVERGED;
  PNK_API_END
}

cc_status cc_solve_fp_diis(cc_handle* h, const cc_problem* p, const cc_fp_opts* opts, double* t1, double* t2,
                           cc_info* info, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(t1 && t2, "t1, t2 must not be NULL");
  cc_fp_opts o;
  cc_fp_opts_default(&o);
  if (opts) o = *opts;
  PNK_REQUIRE(o.tol_inf > 0 && o.max_iter >= 0 && o.diis_size >= 0 && o.diis_size <= 32 && o.diis_start >= 0,
              "invalid FP options");
  H->ensure(p, 0, 1, 30, std::max(o.diis_size, 1), s);
  const int64_t ov = H->eng->o() * (int64_t)H->eng->v(), n2 = H->eng->nvec() - ov;
  if (!o.init_mp2) pack(ov, n2, t1, t2, H->xa, s);
  FpOptions fo;
  fo.tol_inf = o.tol_inf;
  fo.max_iter = o.max_iter;
  fo.diis_size = o.diis_size;
  fo.diis_start = o.diis_start;
  fo.level_shift = o.level_shift;
  fo.init_mp2 = o.init_mp2 != 0;
  fo.ccd = o.ccd != 0;
  SolveStats st;
  H->sol->solve_fp_diis(H->xa, fo, &st, s);
  unpack(ov, n2, H->xa, t1, t2, s);
  PNK_HIP(hipStreamSynchronize(s));
  H->history = H->sol->history();
  fill_info(st, info);
  if (st.diverged) { H->err = "non-finite residual norm"; return CC_ERR_NAN; }
  return st.converged ? CC_OK : CC_NOT_CONVERGED;
  PNK_API_END
}

cc_status cc_gauge_transform(cc_handle* h, const cc_problem* p, const cc_gauge* g, int to_gauge, const double* x1,
                             const double* x2, double* y1, double* y2, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(x1 && x2 && y1 && y2, "array arguments must not be NULL");
  H->ensure(p, 0, 1, 1, 0, s);
  Gauge* G = H->ensure_gauge(g, s);
  const int o = H->eng->o(), v = H->eng->v();
  if (to_gauge) gauge_apply(o, v, G->mo, G->mv, G->fwd_o, G->fwd_v, x1, x2, y1, y2, G->ta, G->tb, s);
  else gauge_apply(G->mo, G->mv, o, v, G->bwd_o, G->bwd_v, x1, x2, y1, y2, G->ta, G->tb, s);
  PNK_HIP(hipStreamSynchronize(s));
  return CC_OK;
  PNK_API_END
}

cc_status cc_residual_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const double* th1,
                            const double* th2, double* r1, double* r2, double* e_corr_host, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(th1 && th2 && r1 && r2, "th1, th2, r1, r2 must not be NULL");
  H->ensure(p, 0, 1, 1, 0, s);
  Gauge* G = H->ensure_gauge(g, s);
  const int o = H->eng->o(), v = H->eng->v();
  const int64_t ov = (int64_t)o * v;
  gauge_apply(G->mo, G->mv, o, v, G->bwd_o, G->bwd_v, th1, th2, G->t, G->t + ov, G->ta, G->tb, s);
  H->eng->residual(G->t, G->t + ov, G->w1, G->w1 + ov, s);
  gauge_apply(o, v, G->mo, G->mv, G->fwd_o, G->fwd_v, G->w1, G->w1 + ov, r1, r2, G->ta, G->tb, s);
  if (e_corr_host) {
    H->eng->energy(G->t, G->t + ov, H->eng->scratch_partials() + 1024, s);
    PNK_HIP(hipMemcpyAsync(e_corr_host, H->eng->scratch_partials() + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  PNK_HIP(hipStreamSynchronize(s));
  return CC_OK;
  PNK_API_END
}

cc_status cc_jvp_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const double* th1, const double* th2,
                       const double* v1, const double* v2, double* jv1, double* jv2, cc_precision prec,
                       void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(th1 && th2 && v1 && v2 && jv1 && jv2, "array arguments must not be NULL");
  PNK_REQUIRE(prec == CC_FP64 || prec == CC_FP32 || prec == CC_BF16, "unknown precision");
  H->ensure(p, lowp_for(prec), 1, 1, 0, s);
  Gauge* G = H->ensure_gauge(g, s);
  const int o = H->eng->o(), v = H->eng->v();
  const int64_t ov = (int64_t)o * v;
  // linearise at t(theta), then J_theta v = (W^T)^(x4) J (C^T)^(x4) v
  gauge_apply(G->mo, G->mv, o, v, G->bwd_o, G->bwd_v, th1, th2, G->t, G->t + ov, G->ta, G->tb, s);
  H->eng->residual(G->t, G->t + ov, G->w1, G->w1 + ov, s);
  gauge_apply(G->mo, G->mv, o, v, G->bwd_o, G->bwd_v, v1, v2, G->w1, G->w1 + ov, G->ta, G->tb, s);
  H->eng->jvp(G->w1, G->w1 + ov, G->w2, G->w2 + ov, (Prec)prec, s);
  gauge_apply(o, v, G->mo, G->mv, G->fwd_o, G->fwd_v, G->w2, G->w2 + ov, jv1, jv2, G->ta, G->tb, s);
  PNK_HIP(hipStreamSynchronize(s));
  return CC_OK;
  PNK_API_END
}

namespace {
// Sets the solver's gauge for the lifetime of the object.
struct GaugeScope {
  Solver* sol;
  GaugeScope(Solver* s, const Gauge* g) : sol(s) { sol->set_gauge(g); }
  ~GaugeScope() { sol->set_gauge(nullptr); }
};
}  // namespace

cc_status cc_solve_pnk_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const cc_pnk_opts* opts,
                             double* th1, double* th2, cc_info* info, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(th1 && th2, "th1, th2 must not be NULL");
  cc_pnk_opts o;
  cc_pnk_opts_default(&o);
  if (opts) o = *opts;
  check_pnk_opts(o);
  H->ensure(p, lowp_for(o.jvp_prec), o.m_max, o.inner_restart, 0, s);
  Gauge* G = H->ensure_gauge(g, s);
  const int64_t gov = (int64_t)G->mo * G->mv, gn2 = G->nvec() - gov;
  if (!o.init_mp2) pack(gov, gn2, th1, th2, G->xg, s);
  SolveStats st;
  {
    GaugeScope scope(H->sol.get(), G);
    H->sol->solve_pnk(G->xg, to_internal(o), &st, s);
  }
  unpack(gov, gn2, G->xg, th1, th2, s);
  PNK_HIP(hipStreamSynchronize(s));
  H->history = H->sol->history();
  fill_info(st, info);
  if (st.diverged) { H->err = "non-finite residual norm"; return CC_ERR_NAN; }
  return st.converged ? CC_OK : CC_NOT_CONVERGED;
  PNK_API_END
}

cc_status cc_solve_fp_diis_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const cc_fp_opts* opts,
                                 double* th1, double* th2, cc_info* info, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(th1 && th2, "th1, th2 must not be NULL");
  cc_fp_opts o;
  cc_fp_opts_default(&o);
  if (opts) o = *opts;
  PNK_REQUIRE(o.tol_inf > 0 && o.max_iter >= 0 && o.diis_size >= 0 && o.diis_size <= 32 && o.diis_start >= 0,
              "invalid FP options");
  H->ensure(p, 0, 1, 30, std::max(o.diis_size, 1), s);
  Gauge* G = H->ensure_gauge(g, s);
  const int64_t gov = (int64_t)G->mo * G->mv, gn2 = G->nvec() - gov;
  if (!o.init_mp2) pack(gov, gn2, th1, th2, G->xg, s);
  FpOptions fo;
  fo.tol_inf = o.tol_inf;
  fo.max_iter = o.max_iter;
  fo.diis_size = o.diis_size;
  fo.diis_start = o.diis_start;
  fo.level_shift = o.level_shift;
  fo.init_mp2 = o.init_mp2 != 0;
  fo.ccd = o.ccd != 0;
  SolveStats st;
  {
    GaugeScope scope(H->sol.get(), G);
    H->sol->solve_fp_diis(G->xg, fo, &st, s);
  }
  unpack(gov, gn2, G->xg, th1, th2, s);
  PNK_HIP(hipStreamSynchronize(s));
  H->history = H->sol->history();
  fill_info(st, info);
  if (st.diverged) { H->err = "non-finite residual norm"; return CC_ERR_NAN; }
  return st.converged ? CC_OK : CC_NOT_CONVERGED;
  PNK_API_END
}

int cc_last_history(const cc_handle* h, double* pairs, int max_pairs) {
  if (!h) return 0;
  const Handle* H = reinterpret_cast<const Handle*>(h);
  const int avail = (int)(H->history.size() / 2);
  if (pairs)
    for (int i = 0; i < std::min(avail, max_pairs); ++i) {
      pairs[2 * i] = H->history[2 * i];
      pairs[2 * i + 1] = H->history[2 * i + 1];
    }
  return avail;
}

cc_status cc_diag_timing(cc_handle* h, int enable) {
  PNK_API_BEGIN(h)
  if (enable) {
    if (!H->timers) H->timers = std::make_unique<Timers>();
    H->timers->reset();
  } else if (H->timers) {
    H->timers->reset();
    if (H->eng) H->eng->set_timers(nullptr);
    H->timers.reset();
  }
  if (H->eng) H->eng->set_timers(H->timers.get());
  return CC_OK;
  PNK_API_END
}

cc_status cc_diag_timing_read(cc_handle* h, int slot, int* count, double* total_ms) {
  PNK_API_BEGIN(h)
  PNK_REQUIRE(count && total_ms && slot >= 0 && slot < kTimerSlots, "invalid timing query");
  if (!H->timers) { *count = 0; *total_ms = 0.0; return CC_OK; }
  H->timers->read(slot, count, total_ms);
  return CC_OK;
  PNK_API_END
}

cc_status cc_diag_contraction_flops(cc_handle* h, const cc_problem* p, cc_precision prec, double* residual_flops,
                                    double* jvp_flops, void* stream) {
  PNK_API_BEGIN(h)
  hipStream_t s = (hipStream_t)stream;
  PNK_REQUIRE(residual_flops && jvp_flops, "output pointers must not be NULL");
  PNK_REQUIRE(prec == CC_FP64 || prec == CC_FP32 || prec == CC_BF16, "unknown precision");
  H->ensure(p, lowp_for(prec), 1, 1, 0, s);
  Engine& E = *H->eng;
  const int64_t ov = (int64_t)E.o() * E.v();
  // eager evaluations: a recorded graph's replay launches nothing the host
  // could count
  E.set_graphs(false);
  try {
    E.reset_contraction_flops();
    E.residual(E.zeros(), E.zeros() + ov, H->xa, H->xa + ov, s);
    *residual_flops = E.contraction_flops();
    E.reset_contraction_flops();
    E.jvp(E.zeros(), E.zeros() + ov, H->xb, H->xb + ov, (Prec)prec, s);
    *jvp_flops = E.contraction_flops();
  } catch (...) {
    E.set_graphs(true);
    throw;
  }
  E.set_graphs(true);
  PNK_HIP(hipStreamSynchronize(s));
  return CC_OK;
  PNK_API_END
}

cc_status cc_diag_hessenberg_eigenvalues(int m, const double* H, double* re, double* im) {
  if (m < 1 || !H || !re || !im) return CC_ERR_ARG;
  return hessenberg_eigenvalues(H, m, re, im) ? CC_OK : CC_NOT_CONVERGED;
}

cc_status cc_diag_occ_sets(int nvir, int* a, int* b, int* lane_t, int64_t cap, int* nsets) {
  if (nvir < 1 || !a || !b || !lane_t || !nsets || cap < 0) return CC_ERR_ARG;
  const int n = fock_op_set_positions(nvir, a, b, lane_t, cap);
  if (n < 0) return CC_ERR_ARG;
  *nsets = n;
  return CC_OK;
}

cc_status cc_diag_gemm(int M, int N, int K, const double* A, int64_t a_m, int64_t a_k, const double* B,
                       int64_t b_k, int64_t b_n, double* C, int64_t c_m, int64_t c_n, double alpha, double beta,
                       cc_precision prec, void* stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return CC_ERR_ARG;
  if (prec != CC_FP64 && prec != CC_FP32 && prec != CC_BF16) return CC_ERR_ARG;
  try {
    GemmDesc d;
    d.M = M; d.N = N; d.K = K;
    d.a_m = a_m; d.a_k = a_k; d.b_k = b_k; d.b_n = b_n; d.c_m = c_m; d.c_n = c_n;
    d.alpha = alpha; d.beta = beta;
    gemm(d, A, Prec::F64, B, Prec::F64, C, Prec::F64, (Prec)prec, (hipStream_t)stream);
  } catch (const ArgError&) {
    return CC_ERR_ARG;
  } catch (const std::exception&) {
    return CC_ERR_HIP;
  }
  return CC_OK;
}

}  // extern "C"

namespace pnk {
int64_t diag_splitk_elems(int64_t nbatch, int M, int N) {
  return std::min<int64_t>(64 * nbatch * (int64_t)M * N, kDiagSplitElems);
}
int64_t diag_cast_bytes(int64_t nbatch, int M, int N, int K, cc_precision prec) {
  // rows of the copies padded to 16 bytes (BF16: to 64 elements, whole
  // panels of the pipelined kernel)
  const int64_t es = prec == CC_BF16 ? 2 : 4, per = prec == CC_BF16 ? 64 : 16 / es;
  return es * nbatch * ((int64_t)M + N) * ((K + per - 1) / per * per) + 512;
}
}  // namespace pnk

extern "C" {

cc_status cc_diag_gemm_batched(int M, int N, int K, int nbatch, const double* A, int64_t a_m, int64_t a_k,
                               int64_t a_b, const double* B, int64_t b_k, int64_t b_n, int64_t b_b, double* C,
                               int64_t c_m, int64_t c_n, int64_t c_b, double alpha, double beta, cc_precision prec,
                               int flags, void* stream) {
  if (M < 1 || N < 1 || K < 1 || nbatch < 1 || !A || !B || !C) return CC_ERR_ARG;
  if (prec != CC_FP64 && prec != CC_FP32 && prec != CC_BF16) return CC_ERR_ARG;
  if (flags & ~3) return CC_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  void* cast = nullptr;
  double* ws = nullptr;
  cc_status st = CC_OK;
  try {
    GemmDesc d;
    d.M = M; d.N = N; d.K = K;
    d.nb0 = nbatch;
    d.a_m = a_m; d.a_k = a_k; d.a_b0 = a_b;
    d.b_k = b_k; d.b_n = b_n; d.b_b0 = b_b;
    d.c_m = c_m; d.c_n = c_n; d.c_b0 = c_b;
    d.alpha = alpha; d.beta = beta;
    if ((flags & 1) && prec != CC_FP64) {
      d.cast_ws_bytes = diag_cast_bytes(nbatch, M, N, K, prec);
      if (hipMalloc(&cast, d.cast_ws_bytes) != hipSuccess) throw OomError("diag_gemm: cast scratch");
      d.cast_ws = cast;
    }
    if (flags & 2) {
      d.ws_elems = diag_splitk_elems(nbatch, M, N);
      if (hipMalloc((void**)&ws, d.ws_elems * sizeof(double)) != hipSuccess) throw OomError("diag_gemm: split-K scratch");
      d.ws = ws;
    }
    gemm(d, A, Prec::F64, B, Prec::F64, C, Prec::F64, (Prec)prec, s);
    PNK_HIP(hipStreamSynchronize(s));
  } catch (const ArgError&) {
    st = CC_ERR_ARG;
  } catch (const OomError&) {
    (void)hipGetLastError();
    st = CC_ERR_OOM;
  } catch (const std::exception&) {
    st = CC_ERR_HIP;
  }
  if (cast) (void)hipFree(cast);
  if (ws) (void)hipFree(ws);
  return st;
}

}  // extern "C"
