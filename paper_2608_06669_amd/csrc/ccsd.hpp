// Closed-shell CCSD residual, its Jacobian-vector product and the Fock
// preconditioner A_F on one GPU.
//
// The residual is evaluated from T1-dressed density-fitted integrals: the
// singles amplitudes are folded into the DF factors, L~ = (1 - tau) L
// (1 + tau), after which the doubles keep the CCD form of the paper's
// working equations (Appendix A, MO representation), built from dressed
// quantities. Every contraction is a strided matrix-core product; index
// permutations between them are bandwidth-bound LDS-tiled transposes.
//
// The Jacobian-vector product is the exact directional derivative of the
// same sequence of operations (forward-mode tangents; the analytic product
// of Appendix B generalised to every term). The operations that do not
// depend on the direction (all dressed quantities at the expansion point)
// are kept from the residual evaluation, so a product costs only the
// tangent contractions, in FP64, FP32 or BF16 with FP32 accumulation.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"
#include "fock_op.hpp"
#include "gemm.hpp"

namespace pnk {

struct ProblemView {
  int o = 0, v = 0, naux = 0;
  const double* f_oo = nullptr;  // device [o][o]
  const double* f_ov = nullptr;  // device [o][v]
  const double* f_vv = nullptr;  // device [v][v]
  const double* L = nullptr;     // device [naux][n][n]
};

// Device memory owned by one engine; sized once from (o, v, naux).
class Arena {
 public:
  Arena() = default;
  ~Arena();
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  // Allocate `bytes`. With a stream, the allocation and the later release are
  // stream-ordered (hipMallocAsync / hipFreeAsync) and never synchronise
  // the device, so concurrent solves on other streams keep running.
  void reserve(size_t bytes, hipStream_t stream = nullptr, bool stream_ordered = false);
  template <typename T> T* take(size_t n) { return reinterpret_cast<T*>(take_bytes(n * sizeof(T))); }
  size_t capacity() const { return cap_; }

 private:
  void* take_bytes(size_t bytes);
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  hipStream_t stream_ = nullptr;
  bool async_ = false;
};

struct EngineOptions {
  bool lowp_f32 = false;   // keep FP32 copies of the constant integral tensors
  bool lowp_bf16 = false;  // keep BF16 copies
  hipStream_t alloc_stream = nullptr;  // stream for stream-ordered allocation
  bool stream_ordered = false;
};

// Device-side timing of tagged launches with HIP events recorded on the
// launching stream (diagnostics; off unless enabled).
enum TimerSlot { kTimerPPL = 0, kTimerResidual, kTimerJvp, kTimerFock, kTimerPrecond, kTimerSlots };
class Timers {
 public:
  ~Timers();
  void begin(int slot, hipStream_t s);
  void end(int slot, hipStream_t s);
  // Synchronises the recorded events and returns (count, total ms).
  void read(int slot, int* count, double* total_ms);
  // Adds durations measured elsewhere (event nodes inside a graph).
  void add(int slot, int count, double ms) { count_[slot] += count; total_[slot] += ms; }
  void reset();

 private:
  struct Pair { hipEvent_t a, b; int slot; };
  std::vector<Pair> used_;
  std::vector<Pair> pool_;
  bool is_open_[kTimerSlots] = {};
  int count_[kTimerSlots] = {};
  double total_[kTimerSlots] = {};
};

// Bytes the engine allocates for these dimensions (used for admission).
size_t engine_bytes(int o, int v, int naux, const EngineOptions& opt);

class Engine {
 public:
  Engine(int o, int v, int naux, const EngineOptions& opt);
  ~Engine();
  int o() const { return o_; }
  int v() const { return v_; }
  int naux() const { return naux_; }
  int64_t nvec() const { return ov_ + n2_; }  // packed [t1 | t2] length
  const EngineOptions& options() const { return opt_; }

  // Integral tensors of a problem (h, dressed-block sources, W_vvvv, ...).
  void prepare(const ProblemView& p, hipStream_t s);
  // Residual r(t) into r1, r2; keeps every intermediate so jvp() can
  // linearise at t. t1/t2 must stay unchanged until the next residual().
  void residual(const double* t1, const double* t2, double* r1, double* r2, hipStream_t s);
  // J(t) x at the t of the last residual(); compute precision `prec`.
  void jvp(const double* x1, const double* x2, double* y1, double* y2, Prec prec, hipStream_t s);
  // Correlation energy at (t1, t2), written to a device double.
  void energy(const double* t1, const double* t2, double* e_dev, hipStream_t s);
  // y = A_F x (Fock operator of equation Preconditioner)
  void fock_apply(const double* x1, const double* x2, double* y1, double* y2, hipStream_t s);

  const double* f_oo() const { return f_oo_; }
  const double* f_vv() const { return f_vv_; }
  bool fov_zero() const { return fov_zero_; }
  // Fused A_F kernel plan (null when the general path must be used).
  const FockOp* fock_op() const { return fop_ok_ ? &fop_ : nullptr; }
  double* scratch_partials() { return partials_; }
  const double* zeros() const { return zeros_; }
  void set_timers(Timers* t) { timers_ = t; }
  // Replay recorded HIP graphs for repeated residual / J v evaluations with
  // the same buffers (default on).
  void set_graphs(bool on) { use_graphs_ = on; }
  Timers* timers() const { return timers_; }
  // Matrix-core flops launched by the host side of the evaluations since
  // the last reset: 2 M N K per product and batch entry at the products'
  // own sizes (tiles' padding not counted). Graph replays launch nothing
  // from the host, so count on an eager evaluation (set_graphs(false)).
  double contraction_flops() const { return mm_flops_; }
  void reset_contraction_flops() { mm_flops_ = 0.0; }

 private:
  struct Ten {
    double* v = nullptr;        // value (FP64)
    double* d = nullptr;        // tangent (FP64)
    bool var = false;           // depends on the amplitudes
    const void* lp32 = nullptr; // FP32 copy of a constant
    const void* lp16 = nullptr; // BF16 copy of a constant
  };
  enum class Mode { Value, Tangent };

  void run(Mode m);
  void mm(const GemmDesc& d, const Ten& A, const Ten& B, const Ten& C);
  void perm(const Ten& in, const Ten& out, int d0, int d1, int d2, int d3, int p0, int p1, int p2, int p3,
            double alpha, double beta);
  void lin_copy(const Ten& in, int64_t in_off, const Ten& out, int64_t n);
  void lin_axpby(int64_t n, double a, const Ten& x, double b, const Ten& y);
  void lin_trace(const Ten& in, int nslices, const Ten& out);
  void lin_pairsym(const Ten& X, const Ten& R);
  void lin_ppl_pack(const Ten& t2, const Ten& Tp, const Ten& Tm);
  void lin_ppl_unpack(const Ten& Rp, const Ten& Rm, const Ten& R);
  void operand(const Ten& t, bool tangent, const void** p, Prec* prec) const;

  int o_, v_, naux_, np_;
  int64_t ov_, n2_;
  EngineOptions opt_;
  Arena arena_;
  Mode mode_ = Mode::Value;
  Prec jprec_ = Prec::F64;
  hipStream_t s_ = nullptr;

  // problem constants
  double *f_oo_, *f_ov_, *f_vv_, *fock_, *h_, *dtr_, *Lo_;
  bool fov_zero_ = true;
  FockOp fop_;
  bool fop_ok_ = false;
  Ten Loo0, Lov0, Lvo0, Lvv0, S, Am, Wov, Ioovv, Iovov, Ix, Ikldc, Itil;
  // symmetry-adapted ladder: pair tables and the (ac|bd) block staging area
  int *pair_a_, *pair_b_, *mpair_a_, *mpair_b_;
  double* wblk_;
  int wblk_na_;
  int64_t p2_, p2m_, o2_;
  int64_t ld32_ = 0, ld32m_ = 0, ld16_ = 0, ld16m_ = 0;  // row lengths of the low-precision ladder copies
  int64_t ldov16_ = 0;  // row length of the BF16 ring integrals (read along k)
  int64_t ldw16_ = 0;   // row length of the BF16 copy of Wov
  // amplitudes and outputs
  Ten T1, T2, R1, R2;
  // intermediates
  Ten Loo, Lvo, Lvv, D, LooT, LvoT, Foo, Fov, Fvo, Fvv;
  Ten U, Tail, Tsail, Uail, Ukdic, Uklca, Uiakc;
  Ten Tmp, X, Gv, Go, Kilj, Wkl, Y, Z, J, Kp, Q, QT, LvvT, Kilc, KilcT;
  Ten Tp, Tm, Rp, Rm;
  double* partials_;
  double* zeros_;  // zero t-vector for the residual at t = 0
  Timers* timers_ = nullptr;
  double mm_flops_ = 0.0;
  // recorded graphs of the residual (value) and J v (tangent, per precision)
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    int hits = 0;
  };
  GraphSlot res_slot_, jvp_slot_[3];
  bool use_graphs_ = true;
  hipStream_t cap_ = nullptr;
  double *tin_ = nullptr, *tout_ = nullptr;  // fixed tangent input / output
  bool capture(Mode m, GraphSlot* slot);
  bool graph_ready(GraphSlot* slot, const void* k0, const void* k1, const void* k2, const void* k3, Mode m);
  double* ws_ = nullptr;  // split-K partial sums
  int64_t ws_elems_ = 0;
  void* cast_ws_ = nullptr;  // rounded operand copies for FP32/BF16 products
  int64_t cast_bytes_ = 0;
  GemmDesc with_ws(GemmDesc d) const {
    d.ws = ws_;
    d.ws_elems = ws_elems_;
    d.cast_ws = cast_ws_;
    d.cast_ws_bytes = cast_bytes_;
    return d;
  }
};

}  // namespace pnk
