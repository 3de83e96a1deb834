// PNK (preconditioned Newton-Krylov) and FP+DIIS solvers over an Engine.
#pragma once

#include <string>
#include <cstdlib>
#include <vector>

#include "ccsd.hpp"
#include "gauge.hpp"

namespace pnk {

struct PnkOptions {
  double tol_inf = 1e-8;
  int max_newton = 100;
  int m_max = 20;
  double gamma = 0.9, alpha = 1.5, eta0 = 0.5, eta_max = 0.9;
  double inner_rtol = 1e-12;
  int inner_maxit = 200;
  int inner_restart = 30;
  Prec jvp_prec = Prec::F64;
  bool use_fd_jvp = false;
  bool init_mp2 = true;
  // outer protocol (the method table): PNK; NK (Newton-GMRES without
  // preconditioner); INK (t <- t - A_F^-1 r(t), the Newton update with A_F
  // in place of the Jacobian)
  enum Protocol { kPNK = 0, kNK = 1, kINK = 2 };
  int protocol = kPNK;
  bool ccd = false;  // CCD level: t1 held at zero, singles equations dropped
  // stagnation stop (0: off): end once stall_window Newton steps pass
  // without ||r||_inf falling below stall_factor times its value at the
  // last step where it did
  int stall_window = 0;
  double stall_factor = 0.5;
  // tolerance of the inner solves applied to J q inside the Krylov loop
  // (0: inner_rtol); the solve of the Newton right-hand side keeps inner_rtol
  double inner_rtol_jv = 0.0;
};

struct FpOptions {
  double tol_inf = 1e-8;
  int max_iter = 500;
  int diis_size = 8;
  int diis_start = 2;
  double level_shift = 0.0;
  bool init_mp2 = true;
  double inner_rtol = 1e-12;
  bool ccd = false;  // CCD level: t1 held at zero, singles equations dropped
};

struct SolveStats {
  double e_corr = 0.0, res_inf = 0.0, res_2 = 0.0;
  int converged = 0, newton_iters = 0, n_residual = 0, n_jvp = 0, n_afmv = 0, n_inner_iters = 0;
  double seconds = 0.0;
  int diverged = 0;  // nonfinite residual norm
  int stalled = 0;   // ended by the stagnation stop
};

// Krylov and history buffers for one problem size (device), plus pinned
// host scalars. Sized once; reused across solves of the same dimensions.
class Solver {
 public:
  // outer_cap: length the outer Krylov, residual and DIIS vectors are
  // sized for (0: the engine's vector length; a redundant gauge needs its
  // own, longer one)
  Solver(Engine& eng, int m_max, int inner_restart, int diis_size, hipStream_t alloc_stream = nullptr,
         bool stream_ordered = false, int64_t outer_cap = 0);
  ~Solver();
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  static size_t bytes(int64_t nvec, int m_max, int inner_restart, int diis_size, int64_t outer_cap = 0);
  int64_t outer_capacity() const { return cap_; }

  // A_F x = b by restarted GMRES to ||b - A_F x|| <= rtol ||b||; packed
  // [t1 | t2] vectors of length nvec. Returns the number of A_F products.
  // pair_symmetric: b2[j][i] = b2[i][j]^T, as for every closed-shell
  // amplitude vector; the symmetric solve may then work on pairs i <= j
  // (it solves for the pair-symmetric part of b).
  int precond_solve(const double* b, double* x, double rtol, int maxit, int restart, hipStream_t s,
                    bool* converged = nullptr, bool pair_symmetric = false);
  // Spectral radius of the Jacobian of the (S)FP map, G = I - diag(D +
  // shift)^-1 J(t), on pair-symmetric vectors: m Arnoldi steps from q0
  // (device, packed, pair-symmetric, nonzero) with the Jacobian linearised
  // at t (device, packed); m <= the basis allocated for PNK. Returns the
  // largest Ritz modulus and the Ritz values (host).
  double fp_spectral_radius(const double* t, const double* q0, double shift, int m, hipStream_t s,
                            std::vector<double>* ritz_re, std::vector<double>* ritz_im);
  // Symmetric A_F (f_ov = 0): device-resident Lanczos form of GMRES, on
  // the full or the packed pair layout.
  int precond_solve_sym(const double* b, double* x, double rtol, int maxit, hipStream_t s, bool* converged,
                        bool packed);
  // Use the short-recurrence form when A_F is symmetric (default on).
  void set_symmetric_inner(bool on) { sym_inner_ = on; }
  // Replay recorded HIP graphs for the inner iterations (default on).
  void set_graphs(bool on) { use_graphs_ = on; }
  static constexpr int kLanczosBlock = 6;  // steps per recorded block (full layout)
  static constexpr int kPackedBlock = 4;   // steps per recorded block (packed layout, fused update)
  // (the packed three-launch form uses kLanczosBlock)
  void solve_pnk(double* x, const PnkOptions& opt, SolveStats* st, hipStream_t s);
  void solve_fp_diis(double* x, const FpOptions& opt, SolveStats* st, hipStream_t s);
  // Solve for the amplitudes of a non-orthogonal or redundant gauge
  // (nullptr: the orbital basis, the default). solve_pnk and solve_fp_diis
  // then iterate on gauge vectors (length g->nvec(), at most the outer
  // capacity): x, the residual, the stopping test and the FP denominators
  // (diagonals of the gauge's Fock blocks) are the gauge's, while the
  // engine works in the orbital basis between the transforms. The gauge's
  // buffers must outlive the solves that use it.
  void set_gauge(const Gauge* g);

  // Residual history (norm-2, norm-inf) per outer residual evaluation.
  const std::vector<double>& history() const { return hist_; }

 private:
  void read_scalars(double* host, const double* dev, int n, hipStream_t s);
  void upload(double* dev, const double* src, int n, hipStream_t s);
  // CGS2 of w (length n) against Q[0..m-1] (stride ldq), returns h (m
  // entries) and ||w|| on the host; w is left orthogonalised, not normalised.
  double orthogonalise(int64_t n, double* Q, int64_t ldq, int m, double* w, std::vector<double>& h, hipStream_t s);
  void norms(int64_t n, const double* r, double* ninf, double* n2, hipStream_t s);

  Engine& eng_;
  int64_t n_;       // orbital vector length (the inner solves)
  int64_t cap_;     // capacity of the outer vectors
  int64_t nv_;      // current outer vector length: n_, or the gauge's
  int vo_, vv_;     // occupied / virtual dimensions of the outer vectors
  int m_max_, restart_, diis_;
  double* Qo_;     // outer Krylov basis (m_max + 1) x cap
  double* Qi_;     // inner Krylov basis (restart + 1) x n
  double* r_;      // residual (cap)
  double* ri_;     // inner GMRES residual (n)
  double* w_;      // work vectors (cap)
  double* w2_;
  double* hx_;     // DIIS amplitudes, diis x cap
  double* he_;     // DIIS error vectors, diis x cap
  double* dsc_;    // device scalars
  double* partials_;
  double* host_;   // pinned host scalars
  hipStream_t alloc_stream_;
  bool async_;
  bool sym_inner_ = true;
  // one line per outer iteration on stderr when PNK_VERBOSE is set
  bool verbose_ = std::getenv("PNK_VERBOSE") != nullptr;
  bool use_graphs_ = true;
  // recorded runs of nb blocks, nb = 1 .. kMaxBatchBlocks
  static constexpr int kMaxBatchBlocks = 16;
  // form of the current symmetric solve: full layout; packed pairs, three
  // launches per step; packed pairs, two launches (fused update)
  enum { kLzFull = 0, kLzPacked3 = 1, kLzFused = 2, kLzModes = 3 };
  hipGraphExec_t lz_graphs_[kLzModes][2][kMaxBatchBlocks + 1] = {};  // [mode][timed][nb]
  bool lz_graph_failed_[kLzModes][2][kMaxBatchBlocks + 1] = {};
  int lz_mode_ = kLzFull;
  std::vector<hipEvent_t> lz_ev_;  // event pairs around the A_F launches of a timed run
  int lz_steps_hint_ = 0;          // steps the last symmetric solve ran
  // With timing on, one symmetric solve in kTimedEvery replays the graphs
  // with event nodes (they cost several microseconds per bracketed launch)
  static constexpr int kTimedEvery = 8;
  int64_t lz_solves_ = 0;
  void lanczos_step(double* vprev, double* v, double* p, double* w1, double* w2, double* x, double* st,
                    double* stn, hipStream_t s);
  // state slots of the Lanczos recurrence (device scalars)
  double* lanczos_state() const;
  void lanczos_block(hipStream_t s);
  int lz_block_len() const;
  bool ensure_lanczos_graph(bool timed, int nb);
  std::vector<double> hist_;
  const Gauge* gauge_ = nullptr;
  // the maps the solvers iterate on, in the gauge when one is set
  void g_residual(const double* x, double* r, hipStream_t s);
  int g_precond(const double* b, double* x, double rtol, int maxit, int restart, hipStream_t s, bool* conv);
  void g_energy(const double* x, double* e_dev, hipStream_t s);
  // a zero outer vector (the engine's, or w2_ cleared to the gauge's length)
  const double* g_zeros(hipStream_t s);
};

}  // namespace pnk
