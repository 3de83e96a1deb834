// CCSD residual / Jacobian-vector product / Fock operator as a sequence of
// matrix-core contractions (see ccsd.hpp).
//
// Index names follow the paper: i,j,k,l occupied; a,b,c,d virtual. Layouts:
// t1[i][a], t2[i][j][a][b], DF blocks X[P][p][q] with P < naux and an extra
// slice P = naux holding the one-electron operator h, dressed like L.
//
// Working equations (T1-dressed closed-shell CCSD; the CCD part is the
// paper's Appendix A with the g_c^a and K signs read as in its
// random-gauge form):
//   r_i^a   = F~_ai + sum_kcd (ac|kd)~ u_ik^cd - sum_klc (ki|lc)~ u_kl^ac
//             + sum_kc F~_kc u_ik^ac
//   r_ij^ab = (ai|bj)~ + sum_cd (ac|bd)~ t_ij^cd + sum_kl W_klij t_kl^ab
//             + P_ij^ab [ sum_c Gv_bc t_ij^ac - sum_k Go_kj t_ik^ab
//                         + sum_kc J_ai,kc u_jk^bc - sum_kc K_ki,ac t_kj^cb
//                         - sum_kc K_ki,bc t_kj^ac ]
// with u = 2 t_ij^ab - t_ij^ba, W_klij = (ki|lj)~ + sum_cd (kc|ld) t_ij^cd,
// Gv_bc = F~_bc - sum (kc|ld) u_kl^bd, Go_kj = F~_kj + sum (kc|ld) u_jl^cd,
// J_ai,kc = (ai|kc)~ + 1/2 sum (kc|ld) u_il^ad - 1/2 sum (kd|lc) t_il^ad,
// K_ki,ac = (ki|ac)~ - 1/2 sum (kd|lc) t_il^da, P_ij^ab Z = Z_ij^ab + Z_ji^ba.
// The dressed ladder splits as sum_cd (ac|bd) t_ij^cd (precomputed
// W_vvvv) + P_ij^ab[-sum_k t_k^a Z'_ij,kb], Z' = Z - 1/2 Y t1 with
// Z_ij,kb = sum_cd (kc|bd) t_ij^cd and Y_ij,kl = sum_cd (kc|ld) t_ij^cd.

#include "ccsd.hpp"
#include "fock_op.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>

#include "cc_kernels.hpp"
#include "gemm.hpp"
#include "tensor_ops.hpp"

namespace pnk {

// ------------------------------------------------------------- arena ----

namespace {
void release(void* p, hipStream_t s, bool async) {
  if (!p) return;
  if (async) (void)hipFreeAsync(p, s);
  else (void)hipFree(p);
}
}  // namespace

Arena::~Arena() { release(base_, stream_, async_); }

void Arena::reserve(size_t bytes, hipStream_t stream, bool stream_ordered) {
  release(base_, stream_, async_);
  base_ = nullptr;
  cap_ = used_ = 0;
  stream_ = stream;
  async_ = stream_ordered;
  if (bytes == 0) return;
  hipError_t e = stream_ordered ? hipMallocAsync((void**)&base_, bytes, stream) : hipMalloc(&base_, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    base_ = nullptr;
    throw OomError("device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  cap_ = bytes;
}

void* Arena::take_bytes(size_t bytes) {
  const size_t a = (used_ + 255) & ~size_t(255);
  if (a + bytes > cap_) throw OomError("engine arena exhausted");
  used_ = a + bytes;
  return base_ + a;
}

// ------------------------------------------------------------ timers ----

Timers::~Timers() {
  reset();
  for (auto& p : pool_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
}

void Timers::begin(int slot, hipStream_t s) {
  Pair p;
  if (pool_.empty()) {
    PNK_HIP(hipEventCreate(&p.a));
    PNK_HIP(hipEventCreate(&p.b));
  } else {
    p = pool_.back();
    pool_.pop_back();
  }
  p.slot = slot;
  PNK_HIP(hipEventRecord(p.a, s));
  used_.push_back(p);
  is_open_[slot] = true;
}

void Timers::end(int slot, hipStream_t s) {
  for (auto it = used_.rbegin(); it != used_.rend(); ++it)
    if (it->slot == slot) {
      PNK_HIP(hipEventRecord(it->b, s));
      break;
    }
  is_open_[slot] = false;
}

void Timers::read(int slot, int* count, double* total_ms) {
  for (auto& p : used_) {
    PNK_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    PNK_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    count_[p.slot] += 1;
    total_[p.slot] += ms;
    pool_.push_back(p);
  }
  used_.clear();
  *count = count_[slot];
  *total_ms = total_[slot];
}

void Timers::reset() {
  for (auto& p : used_) {
    (void)hipEventSynchronize(p.b);
    pool_.push_back(p);
  }
  used_.clear();
  for (int k = 0; k < kTimerSlots; ++k) { count_[k] = 0; total_[k] = 0.0; is_open_[k] = false; }
}

// ----------------------------------------------------------- sizing -----

namespace {

// n rounded up to a multiple of m
int64_t pad_to(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

struct Sizes {
  int64_t o, v, naux, np, n, ov, n2, p2, p2m, o2, wna;
  explicit Sizes(int o_, int v_, int naux_)
      : o(o_), v(v_), naux(naux_), np(naux_ + 1), n(o_ + v_), ov((int64_t)o_ * v_), n2(ov * ov),
        p2((int64_t)v_ * (v_ + 1) / 2), p2m((int64_t)v_ * (v_ - 1) / 2), o2((int64_t)o_ * (o_ + 1) / 2) {
    // (ac|bd) is built for blocks of `wna` values of a at a time
    const int64_t v3 = v * v * v;
    wna = std::max<int64_t>(1, std::min<int64_t>(v, (32ll << 20) / v3));
  }
};

// Split-K scratch. Products with few output tiles, or with a long
// contraction, split it; the chunk count is also capped by this size
// (splits * M * N * batch must fit). 16 times the largest o^2 v^2-class
// tensor, at most 16 M elements (128 MB): room for the four chunks of the
// o v x o v products at o = 10, v = 90, the twelve of their 300 x 900 x 900
// ones, and the three to seven chunks of the ladder products at o = 20,
// v = 180.
int64_t splitk_elems(const Sizes& z) {
  const int64_t big = std::max<int64_t>({z.o * z.o * z.v * z.v, z.ov * z.ov, (int64_t)z.o * z.o * z.o * z.o});
  return std::min<int64_t>(std::max<int64_t>(16 * big, 1 << 16), 16 * 1024 * 1024);
}

// Rounded copies of FP64 operands for the FP32/BF16 products of J v: room
// for both operands of the largest dual product (the ring term, 2ov x 2ov),
// with rows padded to 16 bytes.
int64_t cast_bytes(const Sizes& z, const EngineOptions& opt) {
  if (!opt.lowp_f32 && !opt.lowp_bf16) return 0;
  // (rows of the packed copies are padded along k, to 64 elements in BF16)
  return (opt.lowp_f32 ? 4 : 2) * (4 * z.n2 + 160 * z.ov) + (1 << 20);
}

// Calls `f(count_doubles)` for every FP64 buffer in allocation order, and
// `g(count_bytes)` for the low-precision copies.
template <class F, class G>
void for_each_buffer(const Sizes& z, const EngineOptions& opt, F f, G g) {
  const int64_t o = z.o, v = z.v, naux = z.naux, np = z.np, n = z.n, ov = z.ov, n2 = z.n2;
  // constants
  f(o * o); f(ov); f(v * v); f(n * n); f(n * n); f(naux); f(naux * o * n);
  f(np * o * o); f(np * ov); f(np * ov); f(np * v * v);
  const int64_t p2 = z.p2, p2m = z.p2m, o2 = z.o2;
  f(p2 * p2); f(p2m * p2m); f(z.wna * v * v * v); g(4 * (2 * p2 + 2 * p2m));
  f(o * v * v * v); f(n2); f(n2); f(n2); f(n2); f(n2);
  if (opt.lowp_f32) {
    g(4 * p2 * pad_to(p2, 4)); g(4 * p2m * pad_to(p2m, 4));
    g(4 * o * v * v * v); g(4 * n2); g(4 * n2); g(4 * n2); g(4 * n2);
  }
  if (opt.lowp_bf16) {
    g(2 * p2 * pad_to(p2, 64)); g(2 * p2m * pad_to(p2m, 64));
    g(2 * ov * pad_to(v * v, 64)); g(2 * n2); g(2 * ov * pad_to(ov, 64)); g(2 * ov * pad_to(ov, 64)); g(2 * n2);
  }
  g(cast_bytes(z, opt));
  // intermediates, value and tangent
  for (int rep = 0; rep < 2; ++rep) {
    f(np * o * o); f(np * ov); f(np * v * v); f(naux); f(naux * o * o); f(naux * ov);
    f(o * o); f(ov); f(ov); f(v * v);
    for (int k = 0; k < 7; ++k) f(n2);  // U, Tail, Tsail, Uail, Ukdic, Uklca, Uiakc
    f(n2); f(n2);                       // Tmp, X
    f(v * v); f(o * o); f(o * o * o * o); f(o * o * o * o); f(o * o * o * o); f(o * o * ov);
    f(n2); f(n2);                       // J, Kp
    f(naux * ov); f(naux * ov); f(naux * v * v); f(o * o * ov); f(o * o * ov);
    f(o2 * p2); f(o2 * p2m); f(o2 * p2); f(o2 * p2m);  // Tp, Tm, Rp, Rm
  }
  f(reduce_partials_size(64));
  f(ov + n2);  // zeros
  f(splitk_elems(z));
  f(ov + n2); f(ov + n2);  // graph tangent in / out
}

}  // namespace

size_t engine_bytes(int o, int v, int naux, const EngineOptions& opt) {
  Sizes z(o, v, naux);
  size_t total = 0;
  auto add = [&](int64_t bytes) { total += ((size_t)bytes + 255) & ~size_t(255); };
  for_each_buffer(z, opt, [&](int64_t nd) { add(nd * 8); }, [&](int64_t nb) { add(nb); });
  return total + 4096;
}

// ----------------------------------------------------------- engine -----

Engine::Engine(int o, int v, int naux, const EngineOptions& opt)
    : o_(o), v_(v), naux_(naux), np_(naux + 1), ov_((int64_t)o * v), n2_((int64_t)o * v * o * v), opt_(opt) {
  PNK_REQUIRE(o > 0 && v > 0 && naux > 0, "nocc, nvir and naux must be positive");
  Sizes z(o, v, naux);
  arena_.reserve(engine_bytes(o, v, naux, opt), opt.alloc_stream, opt.stream_ordered);
  const int64_t O = o, V = v, NA = naux, NP = np_, N = o + v, OV = ov_, N2 = n2_;
  auto take = [&](int64_t n) { return arena_.take<double>((size_t)n); };
  f_oo_ = take(O * O); f_ov_ = take(OV); f_vv_ = take(V * V); fock_ = take(N * N); h_ = take(N * N); dtr_ = take(NA);
  Lo_ = take(NA * O * N);
  Loo0.v = take(NP * O * O); Lov0.v = take(NP * OV); Lvo0.v = take(NP * OV); Lvv0.v = take(NP * V * V);
  p2_ = z.p2; p2m_ = z.p2m; o2_ = z.o2; wblk_na_ = (int)z.wna;
  S.v = take(z.p2 * z.p2); Am.v = take(z.p2m * z.p2m); wblk_ = take(z.wna * V * V * V);
  pair_a_ = arena_.take<int>(z.p2); pair_b_ = arena_.take<int>(z.p2);
  mpair_a_ = arena_.take<int>(z.p2m); mpair_b_ = arena_.take<int>(z.p2m);
  Wov.v = take(O * V * V * V);
  Ioovv.v = take(N2); Iovov.v = take(N2); Ix.v = take(N2); Ikldc.v = take(N2); Itil.v = take(N2);
  // the low-precision ladder tensors keep rows of a 16-byte multiple (the
  // pair counts v(v+1)/2, v(v-1)/2 need not be), for vector loads
  ld32_ = pad_to(z.p2, 4); ld32m_ = pad_to(z.p2m, 4);
  ld16_ = pad_to(z.p2, 64); ld16m_ = pad_to(z.p2m, 64);  // whole 64-deep panels, zero-padded
  if (opt.lowp_f32) {
    S.lp32 = arena_.take<float>(z.p2 * ld32_); Am.lp32 = arena_.take<float>(z.p2m * ld32m_);
    Wov.lp32 = arena_.take<float>(O * V * V * V);
    Ioovv.lp32 = arena_.take<float>(N2); Iovov.lp32 = arena_.take<float>(N2);
    Ix.lp32 = arena_.take<float>(N2); Ikldc.lp32 = arena_.take<float>(N2);
  }
  if (opt.lowp_bf16) {
    S.lp16 = arena_.take<uint16_t>(z.p2 * ld16_); Am.lp16 = arena_.take<uint16_t>(z.p2m * ld16m_);
    ldw16_ = pad_to(V * V, 64);  // rows along k, zero-padded to whole panels
    Wov.lp16 = arena_.take<uint16_t>(OV * ldw16_);
    // the ring integrals in BF16 are read along k (the matrix-core operand
    // layout), rows zero-padded to whole 64-deep panels: Iovov as is (it is
    // symmetric), Ix transposed
    ldov16_ = pad_to(OV, 64);
    Ioovv.lp16 = arena_.take<uint16_t>(N2); Iovov.lp16 = arena_.take<uint16_t>(OV * ldov16_);
    Ix.lp16 = arena_.take<uint16_t>(OV * ldov16_); Ikldc.lp16 = arena_.take<uint16_t>(N2);
  }
  cast_bytes_ = cast_bytes(z, opt);
  if (cast_bytes_) cast_ws_ = arena_.take<char>((size_t)cast_bytes_);
  Ten* inter[] = {&Loo, &Lvo, &Lvv, &this->D, &LooT, &LvoT, &Foo, &Fov, &Fvo, &Fvv,
                  &U, &Tail, &Tsail, &Uail, &Ukdic, &Uklca, &Uiakc, &Tmp, &X,
                  &Gv, &Go, &Kilj, &Wkl, &Y, &Z, &J, &Kp, &Q, &QT, &LvvT, &Kilc, &KilcT,
                  &Tp, &Tm, &Rp, &Rm};
  const int64_t isz[] = {NP * O * O, NP * OV, NP * V * V, NA, NA * O * O, NA * OV, O * O, OV, OV, V * V,
                         N2, N2, N2, N2, N2, N2, N2, N2, N2,
                         V * V, O * O, O * O * O * O, O * O * O * O, O * O * O * O, O * O * OV, N2, N2,
                         NA * OV, NA * OV, NA * V * V, O * O * OV, O * O * OV,
                         z.o2 * z.p2, z.o2 * z.p2m, z.o2 * z.p2, z.o2 * z.p2m};
  static_assert(sizeof(inter) / sizeof(inter[0]) == sizeof(isz) / sizeof(isz[0]), "buffer table");
  for (int rep = 0; rep < 2; ++rep)
    for (size_t k = 0; k < sizeof(isz) / sizeof(isz[0]); ++k) {
      if (rep == 0) inter[k]->v = take(isz[k]);
      else inter[k]->d = take(isz[k]);
      inter[k]->var = true;
    }
  partials_ = take(reduce_partials_size(64));
  zeros_ = take(OV + N2);
  ws_elems_ = splitk_elems(z);
  ws_ = take(ws_elems_);
  tin_ = take(OV + N2);
  tout_ = take(OV + N2);
  T1.var = T2.var = R1.var = R2.var = true;
  fop_.o = o;
  fop_.v = v;
  fop_.f_oo = f_oo_;
  fop_.f_vv = f_vv_;
  fop_ok_ = fock_op_plan(fop_);
  (void)z;
}

Engine::~Engine() {
  for (GraphSlot* g : {&res_slot_, &jvp_slot_[0], &jvp_slot_[1], &jvp_slot_[2]})
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (cap_) (void)hipStreamDestroy(cap_);
}

// Record run(m) on a private stream (stream capture does not execute) and
// instantiate it. Returns false (and leaves the slot empty) if the runtime
// refuses; the caller then runs eagerly.
bool Engine::capture(Mode m, GraphSlot* slot) {
  if (!cap_ && hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    cap_ = nullptr;
    return false;
  }
  hipStream_t saved = s_;
  Timers* tm = timers_;
  timers_ = nullptr;
  s_ = cap_;
  hipGraph_t g = nullptr;
  bool ok = false;
  if (hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    // a failure while recording must not leave a partial graph behind
    bool threw = false;
    try {
      run(m);
    } catch (const std::exception& e) {
      threw = true;
      if (std::getenv("PNK_DEBUG")) std::fprintf(stderr, "pnk: graph capture failed: %s\n", e.what());
    }
    if (hipStreamEndCapture(cap_, &g) == hipSuccess && g && !threw &&
        hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0) == hipSuccess)
      ok = true;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (!ok) slot->exec = nullptr;
  s_ = saved;
  timers_ = tm;
  mode_ = Mode::Value;
  return ok;
}

// True when slot holds a graph for these buffers. A graph is recorded on the
// second consecutive call with the same key (so one-off evaluations, such as
// the residual at t = 0, stay eager).
bool Engine::graph_ready(GraphSlot* slot, const void* k0, const void* k1, const void* k2, const void* k3, Mode m) {
  if (!use_graphs_) return false;
  const bool same = slot->key[0] == k0 && slot->key[1] == k1 && slot->key[2] == k2 && slot->key[3] == k3;
  if (same && slot->exec) return true;
  if (!same) {
    if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
    slot->exec = nullptr;
    slot->key[0] = k0; slot->key[1] = k1; slot->key[2] = k2; slot->key[3] = k3;
    slot->hits = 1;
    return false;
  }
  if (++slot->hits < 2) return false;
  return capture(m, slot);
}

// ---------------------------------------------------- op primitives -----

namespace {
GemmDesc gd(int M, int N, int K, int64_t am, int64_t ak, int64_t bk, int64_t bn, int64_t cm, int64_t cn,
            double alpha = 1.0, double beta = 0.0) {
  GemmDesc d;
  d.M = M; d.N = N; d.K = K;
  d.a_m = am; d.a_k = ak; d.b_k = bk; d.b_n = bn; d.c_m = cm; d.c_n = cn;
  d.alpha = alpha; d.beta = beta;
  return d;
}
GemmDesc batch0(GemmDesc d, int nb, int64_t ab, int64_t bb, int64_t cb) {
  d.nb0 = nb; d.a_b0 = ab; d.b_b0 = bb; d.c_b0 = cb;
  return d;
}
}  // namespace

void Engine::operand(const Ten& t, bool tangent, const void** p, Prec* prec) const {
  if (tangent) { *p = t.d; *prec = Prec::F64; return; }
  if (mode_ == Mode::Tangent && !t.var) {
    if (jprec_ == Prec::BF16 && t.lp16) { *p = t.lp16; *prec = Prec::BF16; return; }
    if (jprec_ == Prec::F32 && t.lp32) { *p = t.lp32; *prec = Prec::F32; return; }
  }
  *p = t.v;
  *prec = Prec::F64;
}

// C = alpha A B + beta C, or its tangent dC = alpha (dA B + A dB) + beta dC
void Engine::mm(const GemmDesc& d, const Ten& A, const Ten& B, const Ten& C) {
  const double f = 2.0 * d.M * d.N * d.K * (double)d.nb0 * d.nb1;
  if (mode_ == Mode::Value) {
    mm_flops_ += f;
    gemm64(with_ws(d), A.v, B.v, C.v, s_);
    return;
  }
  if (!C.var) return;
  // the tangent of a product with one varying operand is one product, with
  // two varying operands two
  mm_flops_ += (A.var && B.var) ? 2.0 * f : f;
  PNK_REQUIRE(A.var || B.var, "internal: variable output of a constant product");
  const void *pa, *pb;
  Prec qa, qb;
  GemmDesc e = with_ws(d);
  if (A.var && B.var) {
    // dA B + A dB as one launch when the operand precisions agree
    const void *pa2, *pb2;
    Prec qa2, qb2;
    operand(A, true, &pa, &qa);
    operand(B, false, &pb, &qb);
    operand(A, false, &pa2, &qa2);
    operand(B, true, &pb2, &qb2);
    if (qa == qa2 && qb == qb2) {
      gemm_sum(e, pa, pb, pa2, pb2, qa, qb, C.d, Prec::F64, jprec_, s_);
      return;
    }
  }
  bool first = true;
  if (A.var) {
    operand(A, true, &pa, &qa);
    operand(B, false, &pb, &qb);
    gemm(e, pa, qa, pb, qb, C.d, Prec::F64, jprec_, s_);
    first = false;
  }
  if (B.var) {
    if (!first) e.beta = 1.0;
    operand(A, false, &pa, &qa);
    operand(B, true, &pb, &qb);
    gemm(e, pa, qa, pb, qb, C.d, Prec::F64, jprec_, s_);
  }
}

void Engine::perm(const Ten& in, const Ten& out, int d0, int d1, int d2, int d3, int p0, int p1, int p2, int p3,
                  double alpha, double beta) {
  const int dims[4] = {d0, d1, d2, d3};
  const int pm[4] = {p0, p1, p2, p3};
  if (mode_ == Mode::Value) {
    permute4(in.v, out.v, dims, pm, alpha, beta, s_);
    return;
  }
  if (!out.var) return;
  if (in.var) permute4(in.d, out.d, dims, pm, alpha, beta, s_);
  else if (beta == 0.0) fill((int64_t)d0 * d1 * d2 * d3, 0.0, out.d, s_);
}

void Engine::lin_copy(const Ten& in, int64_t in_off, const Ten& out, int64_t n) {
  if (mode_ == Mode::Value) {
    copy(n, in.v + in_off, out.v, s_);
    return;
  }
  if (!out.var) return;
  if (in.var) copy(n, in.d + in_off, out.d, s_);
  else fill(n, 0.0, out.d, s_);
}

void Engine::lin_axpby(int64_t n, double a, const Ten& x, double b, const Ten& y) {
  if (mode_ == Mode::Value) {
    axpby(n, a, x.v, b, y.v, s_);
    return;
  }
  if (!y.var) return;
  if (x.var) axpby(n, a, x.d, b, y.d, s_);
  else if (b == 0.0) fill(n, 0.0, y.d, s_);
  else if (b != 1.0) axpby(n, 0.0, y.d, b, y.d, s_);
}

void Engine::lin_trace(const Ten& in, int nslices, const Ten& out) {
  if (mode_ == Mode::Value) trace_slices(nslices, o_, in.v, out.v, s_);
  else trace_slices(nslices, o_, in.d, out.d, s_);
}

void Engine::lin_pairsym(const Ten& Xs, const Ten& R) {
  if (mode_ == Mode::Value) pair_symmetrize_add(o_, v_, Xs.v, 1.0, R.v, s_);
  else pair_symmetrize_add(o_, v_, Xs.d, 1.0, R.d, s_);
}

void Engine::lin_ppl_pack(const Ten& t2, const Ten& tp, const Ten& tm) {
  if (mode_ == Mode::Value) ppl_pack_t(o_, v_, t2.v, pair_a_, pair_b_, mpair_a_, mpair_b_, tp.v, tm.v, s_);
  else ppl_pack_t(o_, v_, t2.d, pair_a_, pair_b_, mpair_a_, mpair_b_, tp.d, tm.d, s_);
}

void Engine::lin_ppl_unpack(const Ten& rp, const Ten& rm, const Ten& R) {
  if (mode_ == Mode::Value) ppl_unpack_add(o_, v_, rp.v, rm.v, R.v, s_);
  else ppl_unpack_add(o_, v_, rp.d, rm.d, R.d, s_);
}

// ------------------------------------------------------------ prepare ---

void Engine::prepare(const ProblemView& p, hipStream_t s) {
  PNK_REQUIRE(p.o == o_ && p.v == v_ && p.naux == naux_, "prepare: dimensions differ from the engine's");
  s_ = s;
  mode_ = Mode::Value;
  const int o = o_, v = v_, naux = naux_, n = o + v;
  const int64_t ov = ov_, vv = (int64_t)v * v;
  PNK_HIP(hipMemcpyAsync(f_oo_, p.f_oo, sizeof(double) * o * o, hipMemcpyDeviceToDevice, s));
  PNK_HIP(hipMemcpyAsync(f_ov_, p.f_ov, sizeof(double) * ov, hipMemcpyDeviceToDevice, s));
  PNK_HIP(hipMemcpyAsync(f_vv_, p.f_vv, sizeof(double) * vv, hipMemcpyDeviceToDevice, s));
  // h = f - G[L], G[L]_pq = sum_P 2 L_pq d_P - sum_Pk L_pk L_kq
  assemble_fock(o, v, f_oo_, f_ov_, f_vv_, fock_, s);
  copy((int64_t)n * n, fock_, h_, s);
  trace_occ(naux, o, n, p.L, dtr_, s);
  gemm64(with_ws(gd(1, n * n, naux, 0, 1, (int64_t)n * n, 1, 0, 1, -2.0, 1.0)), dtr_, p.L, h_, s);
  extract_occ_rows(naux, o, n, p.L, Lo_, s);
  gemm64(with_ws(gd(n, n, naux * o, 1, n, n, 1, n, 1, 1.0, 1.0)), Lo_, Lo_, h_, s);
  extract_blocks(naux, o, v, p.L, h_, Loo0.v, Lov0.v, Lvo0.v, Lvv0.v, s);
  // symmetry-adapted (ac|bd): pair tables, then blocks of a at a time:
  // Wblk[a - a0][b][c][d] = sum_P L_ac L_bd (batch b0 = b, b1 = a - a0),
  // packed into S (a <= b, c <= d) and A (a < b, c < d)
  {
    std::vector<int> pa(p2_), pb(p2_), ma(std::max<int64_t>(p2m_, 1)), mb(std::max<int64_t>(p2m_, 1));
    int64_t k = 0, km = 0;
    for (int a = 0; a < v; ++a)
      for (int b = a; b < v; ++b) {
        pa[k] = a; pb[k] = b; ++k;
        if (b > a) { ma[km] = a; mb[km] = b; ++km; }
      }
    PNK_HIP(hipMemcpyAsync(pair_a_, pa.data(), p2_ * sizeof(int), hipMemcpyHostToDevice, s));
    PNK_HIP(hipMemcpyAsync(pair_b_, pb.data(), p2_ * sizeof(int), hipMemcpyHostToDevice, s));
    if (p2m_ > 0) {
      PNK_HIP(hipMemcpyAsync(mpair_a_, ma.data(), p2m_ * sizeof(int), hipMemcpyHostToDevice, s));
      PNK_HIP(hipMemcpyAsync(mpair_b_, mb.data(), p2m_ * sizeof(int), hipMemcpyHostToDevice, s));
    }
    PNK_HIP(hipStreamSynchronize(s));  // host tables go out of scope
    for (int a0 = 0; a0 < v; a0 += wblk_na_) {
      const int na = std::min(wblk_na_, v - a0);
      GemmDesc d = gd(v, v, naux, 1, vv, vv, 1, v, 1);
      d.nb0 = v; d.nb1 = na;
      d.a_b0 = 0; d.a_b1 = v;
      d.b_b0 = v; d.b_b1 = 0;
      d.c_b0 = vv; d.c_b1 = vv * v;
      gemm64(with_ws(d), Lvv0.v + (int64_t)a0 * v, Lvv0.v, wblk_, s);
      ppl_pack_w(v, a0, na, wblk_, pair_a_, pair_b_, mpair_a_, mpair_b_, S.v, Am.v, s);
    }
  }
  // Wov[k][b][c][d] = (kc|bd)
  {
    GemmDesc d = gd(v, v, naux, 1, ov, vv, 1, v, 1);
    d.nb0 = v; d.nb1 = o;
    d.a_b0 = 0; d.a_b1 = v;
    d.b_b0 = v; d.b_b1 = 0;
    d.c_b0 = vv; d.c_b1 = vv * v;
    gemm64(with_ws(d), Lov0.v, Lvv0.v, Wov.v, s);
  }
  // Ioovv[k][l][c][d] = (kc|ld)
  {
    GemmDesc d = gd(v, v, naux, 1, ov, ov, 1, v, 1);
    d.nb0 = o; d.nb1 = o;
    d.a_b0 = 0; d.a_b1 = v;
    d.b_b0 = v; d.b_b1 = 0;
    d.c_b0 = vv; d.c_b1 = vv * o;
    gemm64(with_ws(d), Lov0.v, Lov0.v, Ioovv.v, s);
  }
  // Iovov[(k,c)][(l,d)] = (kc|ld); Ix[l][d][k][c] = (kd|lc)
  gemm64(with_ws(gd((int)ov, (int)ov, naux, 1, ov, ov, 1, ov, 1)), Lov0.v, Lov0.v, Iovov.v, s);
  {
    const int dims[4] = {o, v, o, v};
    const int pm[4] = {2, 1, 0, 3};
    permute4(Iovov.v, Ix.v, dims, pm, 1.0, 0.0, s);
    const int dims2[4] = {o, o, v, v};
    const int pm2[4] = {0, 1, 3, 2};
    permute4(Ioovv.v, Ikldc.v, dims2, pm2, 1.0, 0.0, s);
    permute4(Ioovv.v, Itil.v, dims2, pm2, -1.0, 0.0, s);
    axpby(n2_, 2.0, Ioovv.v, 1.0, Itil.v, s);
  }
  // the ladder tensors with padded rows, the others flat
  if (S.lp32) cast_f64_to_f32_rows(p2_, p2_, ld32_, S.v, (float*)S.lp32, s);
  if (S.lp16) cast_f64_to_bf16_rows(p2_, p2_, ld16_, S.v, (uint16_t*)S.lp16, s);
  if (Am.lp32) cast_f64_to_f32_rows(p2m_, p2m_, ld32m_, Am.v, (float*)Am.lp32, s);
  if (Am.lp16) cast_f64_to_bf16_rows(p2m_, p2m_, ld16m_, Am.v, (uint16_t*)Am.lp16, s);
  Ten* lows[] = {&Wov, &Ioovv, &Iovov, &Ix, &Ikldc};
  const int64_t lsz[] = {(int64_t)o * v * vv, n2_, n2_, n2_, n2_};
  for (int k = 0; k < 5; ++k) {
    if (lows[k]->lp32) cast_f64_to_f32(lsz[k], lows[k]->v, (float*)lows[k]->lp32, s);
    if (lows[k]->lp16 && lows[k] != &Iovov && lows[k] != &Ix && lows[k] != &Wov)
      cast_f64_to_bf16(lsz[k], lows[k]->v, (uint16_t*)lows[k]->lp16, s);
  }
  if (Wov.lp16) cast_f64_to_bf16_rows(ov, (int64_t)v * v, ldw16_, Wov.v, (uint16_t*)Wov.lp16, s);
  if (Iovov.lp16) {
    cast_f64_to_bf16_rows(ov, ov, ldov16_, Iovov.v, (uint16_t*)Iovov.lp16, s);
    // Ix^T[(k,c)][(l,d)] = Ix[(l,d)][(k,c)] = (kd|lc), staged in Tmp
    const int dims[4] = {o, v, o, v};
    const int pm[4] = {0, 3, 2, 1};
    permute4(Iovov.v, Tmp.v, dims, pm, 1.0, 0.0, s);
    cast_f64_to_bf16_rows(ov, ov, ldov16_, Tmp.v, (uint16_t*)Ix.lp16, s);
  }
  fill(ov_ + n2_, 0.0, zeros_, s);
  // f_ov == 0 lets A_F skip its singles-doubles coupling
  nrm_inf(ov, f_ov_, partials_ + reduce_partials_size(64) - 1, partials_, s);
  double fmax = 0.0;
  PNK_HIP(hipMemcpyAsync(&fmax, partials_ + reduce_partials_size(64) - 1, sizeof(double), hipMemcpyDeviceToHost, s));
  PNK_HIP(hipStreamSynchronize(s));
  fov_zero_ = (fmax == 0.0);
}

// --------------------------------------------------------- the program --

void Engine::run(Mode m) {
  mode_ = m;
  const int o = o_, v = v_, naux = naux_, np = np_;
  const int64_t O = o, V = v, ov = ov_, vv = V * V, oo = O * O, n2 = n2_;
  const int OV = (int)ov, OO = (int)oo, VV = (int)vv;

  // ---- T1 dressing: L~ = (1 - tau) L (1 + tau), slice naux is h ----
  lin_copy(Loo0, 0, Loo, np * oo);
  mm(gd(np * o, o, v, v, 1, 1, v, o, 1, 1.0, 1.0), Lov0, T1, Loo);            // + L_kc t_i^c
  lin_copy(Lvo0, 0, Lvo, np * ov);
  mm(gd(np * v, o, v, v, 1, 1, v, o, 1, 1.0, 1.0), Lvv0, T1, Lvo);            // + L_ab t_i^b
  mm(batch0(gd(v, o, o, 1, v, o, 1, o, 1, -1.0, 1.0), np, 0, oo, ov), T1, Loo, Lvo);  // - t_k^a L~_ki
  lin_copy(Lvv0, 0, Lvv, np * vv);
  mm(batch0(gd(v, v, o, 1, v, v, 1, v, 1, -1.0, 1.0), np, 0, ov, vv), T1, Lov0, Lvv); // - t_k^a L_kc

  // ---- dressed Fock F~ = h~ + sum_P [2 L~ D - L~_{:,o} L~_{o,:}] ----
  lin_trace(Loo, naux, D);
  perm(Loo, LooT, 1, naux, o, o, 0, 2, 1, 3, 1.0, 0.0);
  perm(Lvo, LvoT, 1, naux, v, o, 0, 2, 1, 3, 1.0, 0.0);
  lin_copy(Loo, naux * oo, Foo, oo);
  mm(gd(1, OO, naux, 0, 1, oo, 1, 0, 1, 2.0, 1.0), D, Loo, Foo);
  mm(gd(o, o, naux * o, naux * O, 1, o, 1, o, 1, -1.0, 1.0), LooT, Loo, Foo);
  lin_copy(Lov0, naux * ov, Fov, ov);
  mm(gd(1, OV, naux, 0, 1, ov, 1, 0, 1, 2.0, 1.0), D, Lov0, Fov);
  mm(gd(o, v, naux * o, naux * O, 1, v, 1, v, 1, -1.0, 1.0), LooT, Lov0, Fov);
  lin_copy(Lvo, naux * ov, Fvo, ov);
  mm(gd(1, OV, naux, 0, 1, ov, 1, 0, 1, 2.0, 1.0), D, Lvo, Fvo);
  mm(gd(v, o, naux * o, naux * O, 1, o, 1, o, 1, -1.0, 1.0), LvoT, Loo, Fvo);
  lin_copy(Lvv, naux * vv, Fvv, vv);
  mm(gd(1, VV, naux, 0, 1, vv, 1, 0, 1, 2.0, 1.0), D, Lvv, Fvv);
  mm(gd(v, v, naux * o, naux * O, 1, v, 1, v, 1, -1.0, 1.0), LvoT, Lov0, Fvv);

  // ---- amplitude layouts ----
  perm(T2, U, o, o, v, v, 0, 1, 3, 2, -1.0, 0.0);
  lin_axpby(n2, 2.0, T2, 1.0, U);                                  // u = 2t - t_swap
  perm(T2, Tail, o, o, v, v, 2, 0, 1, 3, 1.0, 0.0);                // [a][i][l][d] = t_il^ad
  perm(T2, Tsail, o, o, v, v, 3, 0, 1, 2, 1.0, 0.0);               // [a][i][l][d] = t_il^da
  perm(U, Uail, o, o, v, v, 2, 0, 1, 3, 1.0, 0.0);                 // [a][i][l][d] = u_il^ad
  perm(U, Ukdic, o, o, v, v, 1, 3, 0, 2, 1.0, 0.0);                // [k][d][i][c] = u_ik^cd
  perm(U, Uklca, o, o, v, v, 0, 1, 3, 2, 1.0, 0.0);                // [k][l][c][a] = u_kl^ac
  perm(U, Uiakc, o, o, v, v, 0, 2, 1, 3, 1.0, 0.0);                // [i][a][k][c] = u_ik^ac

  // ---- r2 = (ai|bj)~ ----
  mm(gd(OV, OV, naux, 1, ov, ov, 1, ov, 1), Lvo, Lvo, Tmp);        // [(a,i)][(b,j)]
  perm(Tmp, R2, v, o, v, o, 1, 3, 0, 2, 1.0, 0.0);
  // ---- particle-particle ladder, symmetry-adapted: for i <= j and the
  // (anti)symmetric combinations of c,d, R+ = T+ S, R- = T- A ----
  lin_ppl_pack(T2, Tp, Tm);
  {
    // S and A are symmetric matrices: read them along the contiguous index
    // the compute type stages best (n for FP64/FP32, k for BF16)
    const bool kc = mode_ == Mode::Tangent && jprec_ == Prec::BF16;
    const int P2 = (int)p2_, P2m = (int)p2m_, O2 = (int)o2_, O2m = o_ * (o_ - 1) / 2;
    // row length of the copy the product reads (padded in FP32 / BF16)
    const bool t32 = mode_ == Mode::Tangent && jprec_ == Prec::F32;
    const int64_t ls = kc && S.lp16 ? ld16_ : (t32 && S.lp32 ? ld32_ : p2_);
    const int64_t lm = kc && Am.lp16 ? ld16m_ : (t32 && Am.lp32 ? ld32m_ : p2m_);
    if (timers_) timers_->begin(kTimerPPL, s_);
    // (the BF16 copies' rows are zero from P2 to their length: the packed
    // amplitudes may run the contraction over whole panels)
    GemmDesc gs = gd(O2, P2, P2, p2_, 1, kc ? 1 : ls, kc ? ls : 1, p2_, 1);
    if (kc && S.lp16) gs.b_kzero = ld16_;
    mm(gs, Tp, S, Rp);
    // the antisymmetric pairs over i < j only (t_ii^cd = t_ii^dc)
    if (P2m > 0 && O2m > 0) {
      GemmDesc ga = gd(O2m, P2m, P2m, p2m_, 1, kc ? 1 : lm, kc ? lm : 1, p2m_, 1);
      if (kc && Am.lp16) ga.b_kzero = ld16m_;
      mm(ga, Tm, Am, Rm);
    }
    if (timers_) timers_->end(kTimerPPL, s_);
  }
  lin_ppl_unpack(Rp, Rm, R2);
  // ---- hole-hole ladder ----
  mm(gd(OO, OO, naux, 1, oo, oo, 1, oo, 1), Loo, Loo, Kilj);       // [(k,i)][(l,j)]
  perm(Kilj, Wkl, o, o, o, o, 0, 2, 1, 3, 1.0, 0.0);               // [(k,l)][(i,j)]
  mm(gd(OO, OO, VV, vv, 1, 1, vv, oo, 1), Ioovv, T2, Y);           // Y[(k,l)][(i,j)]
  lin_axpby(oo * oo, 1.0, Y, 1.0, Wkl);
  mm(gd(OO, VV, OO, 1, oo, vv, 1, vv, 1, 1.0, 1.0), Wkl, T2, R2);

  // ---- Fock-type intermediates ----
  lin_copy(Fvv, 0, Gv, vv);
  mm(gd(v, v, (int)(oo * v), oo * V, 1, v, 1, v, 1, -1.0, 1.0), Uail, Ikldc, Gv);
  lin_copy(Foo, 0, Go, oo);
  mm(gd(o, o, (int)(O * vv), O * vv, 1, 1, O * vv, o, 1, 1.0, 1.0), Ioovv, U, Go);
  mm(gd((int)(oo * v), v, v, v, 1, 1, v, v, 1), T2, Gv, X);        // X = sum_c Gv_bc t_ij^ac
  mm(batch0(gd(o, VV, o, 1, o, vv, 1, vv, 1, -1.0, 1.0), o, 0, O * vv, O * vv), Go, T2, X);

  // ---- T1 part of the dressed ladder ----
  {
    // Z[(i,j)][(k,b)]; BF16 tangents read the padded BF16 copy of Wov
    const bool kcw = mode_ == Mode::Tangent && jprec_ == Prec::BF16 && Wov.lp16;
    GemmDesc gz = gd(OO, OV, VV, vv, 1, 1, kcw ? ldw16_ : vv, ov, 1);
    if (kcw) gz.b_kzero = ldw16_;
    mm(gz, T2, Wov, Z);
  }
  mm(batch0(gd(OO, v, o, 1, oo, v, 1, ov, 1, -0.5, 1.0), o, O * oo, 0, v), Y, T1, Z);
  mm(batch0(gd(v, v, o, 1, v, v, 1, v, 1, -1.0, 1.0), OO, 0, ov, vv), T1, Z, X);

  // ---- ring terms ----
  mm(gd(OV, OV, naux, 1, ov, ov, 1, ov, 1), Lvo, Lov0, J);         // (ai|kc)~
  // (BF16 tangents read the ring integrals along k: Iovov is symmetric, and
  // the BF16 copy of Ix holds its transpose)
  const bool kc16 = mode_ == Mode::Tangent && jprec_ == Prec::BF16 && Iovov.lp16;
  auto ring = [&](double alpha) {
    GemmDesc g = gd(OV, OV, OV, ov, 1, kc16 ? 1 : ov, kc16 ? ldov16_ : 1, ov, 1, alpha, 1.0);
    if (kc16) g.b_kzero = ldov16_;
    return g;
  };
  mm(ring(0.5), Uail, Iovov, J);
  mm(ring(-0.5), Tail, Ix, J);
  mm(gd(OO, VV, naux, 1, oo, vv, 1, vv, 1), Loo, Lvv, Tmp);        // (ki|ac)~ as [(k,i)][(a,c)]
  perm(Tmp, Kp, o, o, v, v, 2, 1, 0, 3, 1.0, 0.0);                 // K'[(a,i)][(k,c)]
  mm(ring(-0.5), Tsail, Ix, Kp);
  mm(gd(OV, OV, OV, ov, 1, 1, ov, ov, 1), J, Uail, Tmp);           // J u_jk^bc
  mm(gd(OV, OV, OV, ov, 1, 1, ov, ov, 1, -1.0, 1.0), Kp, Tail, Tmp);  // - K t_kj^cb
  perm(Tmp, X, v, o, v, o, 1, 3, 0, 2, 1.0, 1.0);
  mm(gd(OV, OV, OV, ov, 1, 1, ov, ov, 1), Kp, Tsail, Tmp);         // K_ki,bc t_kj^ac as [(b,i)][(a,j)]
  perm(Tmp, X, v, o, v, o, 1, 3, 2, 0, -1.0, 1.0);

  // ---- r2 += P_ij^ab X ----
  lin_pairsym(X, R2);

  // ---- singles ----
  perm(Fvo, R1, 1, 1, v, o, 0, 1, 3, 2, 1.0, 0.0);                 // F~_ai
  mm(gd(naux, OV, OV, ov, 1, ov, 1, ov, 1), Lov0, Ukdic, Q);       // Q[P][(i,c)]
  perm(Q, QT, 1, naux, o, v, 0, 2, 1, 3, 1.0, 0.0);
  perm(Lvv, LvvT, 1, naux, v, v, 0, 1, 3, 2, 1.0, 0.0);
  mm(gd(o, v, naux * v, naux * V, 1, v, 1, v, 1, 1.0, 1.0), QT, LvvT, R1);
  mm(gd(OO, OV, naux, 1, oo, ov, 1, ov, 1), Loo, Lov0, Kilc);      // (ki|lc)~ as [(k,i)][(l,c)]
  perm(Kilc, KilcT, o, o, o, v, 1, 0, 2, 3, 1.0, 0.0);
  mm(gd(o, v, (int)(oo * v), oo * V, 1, v, 1, v, 1, -1.0, 1.0), KilcT, Uklca, R1);
  mm(gd(OV, 1, OV, ov, 1, 1, 1, 1, 1, 1.0, 1.0), Uiakc, Fov, R1);
}

void Engine::residual(const double* t1, const double* t2, double* r1, double* r2, hipStream_t s) {
  s_ = s;
  T1.v = const_cast<double*>(t1);
  T2.v = const_cast<double*>(t2);
  R1.v = r1;
  R2.v = r2;
  if (timers_) timers_->begin(kTimerResidual, s);
  if (graph_ready(&res_slot_, t1, t2, r1, r2, Mode::Value)) PNK_HIP(hipGraphLaunch(res_slot_.exec, s));
  else run(Mode::Value);
  if (timers_) timers_->end(kTimerResidual, s);
}

void Engine::jvp(const double* x1, const double* x2, double* y1, double* y2, Prec prec, hipStream_t s) {
  PNK_REQUIRE(T1.v && T2.v, "jvp before any residual evaluation");
  s_ = s;
  jprec_ = prec;
  if (timers_) timers_->begin(kTimerJvp, s);
  // graphs run on fixed tangent buffers: copy in, replay, copy out
  T1.d = tin_;
  T2.d = tin_ + ov_;
  R1.d = tout_;
  R2.d = tout_ + ov_;
  GraphSlot* slot = &jvp_slot_[(int)prec];
  if (graph_ready(slot, T1.v, T2.v, nullptr, nullptr, Mode::Tangent)) {
    jprec_ = prec;
    // (one copy each way when the caller's singles and doubles are adjacent)
    if (x2 == x1 + ov_) {
      PNK_HIP(hipMemcpyAsync(tin_, x1, (ov_ + n2_) * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      PNK_HIP(hipMemcpyAsync(tin_, x1, ov_ * sizeof(double), hipMemcpyDeviceToDevice, s));
      PNK_HIP(hipMemcpyAsync(tin_ + ov_, x2, n2_ * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    PNK_HIP(hipGraphLaunch(slot->exec, s));
    if (y2 == y1 + ov_) {
      PNK_HIP(hipMemcpyAsync(y1, tout_, (ov_ + n2_) * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      PNK_HIP(hipMemcpyAsync(y1, tout_, ov_ * sizeof(double), hipMemcpyDeviceToDevice, s));
      PNK_HIP(hipMemcpyAsync(y2, tout_ + ov_, n2_ * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  } else {
    T1.d = const_cast<double*>(x1);
    T2.d = const_cast<double*>(x2);
    R1.d = y1;
    R2.d = y2;
    run(Mode::Tangent);
  }
  if (timers_) timers_->end(kTimerJvp, s);
  mode_ = Mode::Value;
  jprec_ = Prec::F64;
}

void Engine::energy(const double* t1, const double* t2, double* e_dev, hipStream_t s) {
  pnk::energy(o_, v_, f_ov_, Itil.v, t1, t2, e_dev, partials_, s);
}

// (A_F x)_ij^ab = sum_c (f_ac x_ij^cb + f_bc x_ij^ac) - sum_k (f_ki x_kj^ab + f_kj x_ik^ab)
// (A_F x)_i^a   = sum_c f_ac x_i^c - sum_k f_ki x_k^a + sum_kc f_kc (2 x_ik^ac - x_ik^ca)
void Engine::fock_apply(const double* x1, const double* x2, double* y1, double* y2, hipStream_t s) {
  const int o = o_, v = v_;
  const int64_t O = o, V = v, vv = V * V, oo = O * O, ov = ov_;
  if (timers_) timers_->begin(kTimerFock, s);
  if (fop_ok_ && x1 != y1 && x2 != y2) {
    // virtual and occupied contractions and singles in one launch
    fock_op_apply(fop_, x1, x2, y1, y2, s);
  } else {
    // a index: batched over ij, y_ij = f_vv x_ij
    gemm64(with_ws(batch0(gd(v, v, v, v, 1, v, 1, v, 1), (int)oo, 0, vv, vv)), f_vv_, x2, y2, s);
    // b index: y[(ija)][b] += sum_c x[(ija)][c] f_bc
    gemm64(with_ws(gd((int)(oo * v), v, v, v, 1, 1, v, v, 1, 1.0, 1.0)), x2, f_vv_, y2, s);
    // i index: y[i][(jab)] -= sum_k f_ki x[k][(jab)]
    gemm64(with_ws(gd(o, (int)(O * vv), o, 1, o, O * vv, 1, O * vv, 1, -1.0, 1.0)), f_oo_, x2, y2, s);
    // j index: batched over i, y_i[j][(ab)] -= sum_k f_kj x_i[k][(ab)]
    gemm64(with_ws(batch0(gd(o, (int)vv, o, 1, o, vv, 1, vv, 1, -1.0, 1.0), o, 0, O * vv, O * vv)), f_oo_, x2, y2, s);
    // singles
    gemm64(with_ws(gd(o, v, v, v, 1, 1, v, v, 1)), x1, f_vv_, y1, s);
    gemm64(with_ws(gd(o, v, o, 1, o, v, 1, v, 1, -1.0, 1.0)), f_oo_, x1, y1, s);
  }
  if (!fov_zero_) {
    // u_x[i][a][k][c] = 2 x_ik^ac - x_ik^ca, then y1 += u_x f_ov
    const int dims[4] = {o, o, v, v};
    const int p1[4] = {0, 2, 1, 3};  // x_ik^ac at [i][a][k][c]
    const int p2[4] = {0, 3, 1, 2};  // x_ik^ca at [i][a][k][c]
    permute4(x2, Tmp.v, dims, p1, 2.0, 0.0, s);
    permute4(x2, Tmp.v, dims, p2, -1.0, 1.0, s);
    gemm64(with_ws(gd((int)ov, 1, (int)ov, ov, 1, 1, 1, 1, 1, 1.0, 1.0)), Tmp.v, f_ov_, y1, s);
  }
  if (timers_) timers_->end(kTimerFock, s);
}

}  // namespace pnk
