/*
 * pnkcc: preconditioned Newton-Krylov solver for closed-shell CCSD
 * amplitude equations on AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2608.06669, "A robust and efficient solver for coupled
 * cluster equations". Section "Theory" defines the amplitude equations
 * r(t) = <Phi_mu| e^{-T} H e^{T} |Phi_0> = 0 (equation CC_ampl), the energy
 * (equation CC_energy), the Newton system J delta = -r (equation
 * LinSyst_4_Newton) and the gauge-invariant Fock preconditioner
 * [A_F]_{mu,nu} = <Phi_mu|[F, X_nu]|Phi_0> (equation Preconditioner, working
 * equations in Appendix C). Appendix F gives the PNK algorithm and its
 * Eisenstat-Walker forcing term. The paper works at the CCD level; this
 * library solves CCSD (singles through the T1-similarity-transformed
 * Hamiltonian) with density-fitted integrals.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers to float64, row-major, owned by
 *   the caller (for example torch tensors' data_ptr()). The library keeps no
 *   pointer after a call returns. Host pointers are marked "host".
 * - Indices: i,j,k,l occupied (0..nocc-1), a,b,c,d virtual (0..nvir-1),
 *   n = nocc + nvir, P auxiliary (0..naux-1).
 * - Amplitudes and residuals: t1[i][a] (nocc*nvir) and t2[i][j][a][b]
 *   (nocc^2*nvir^2) with t2[i][j][a][b] == t2[j][i][b][a] (a precondition
 *   of every entry point, not checked: the particle-particle ladder skips
 *   what vanishes under it). Residual
 *   components are the projections onto a+_{a,alpha} a_{i,alpha}|Phi_0> and
 *   a+_{a,alpha} a_{i,alpha} a+_{b,beta} a_{j,beta}|Phi_0> of
 *   e^{-T} H e^{T}|Phi_0>, with T = sum t1 E_ai + 1/2 sum t2 E_ai E_bj.
 * - `stream` is a hipStream_t (NULL: the default stream). All device work of
 *   a call is ordered on it. Calls that return host scalars (energies,
 *   iteration counts, solver info) synchronise the stream before returning;
 *   cc_jvp and cc_fock_apply do not synchronise.
 * - Errors: a status code; no exception crosses the boundary.
 *   cc_last_error() describes the last failure on the handle. On an error no
 *   output is guaranteed to be written.
 * - A handle holds device workspace sized for the last problem shape and
 *   caches the integral tensors derived from the last problem, keyed on its
 *   pointers, sizes and a 64-bit hash of its contents (recomputed on every
 *   call, so changing the data in place is safe). A handle must not be used
 *   by two threads at once; use one handle per thread or stream.
 */
#ifndef PNKCC_H
#define PNKCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CC_OK = 0,
  CC_NOT_CONVERGED = 1,  /* solver stopped at its iteration cap; outputs hold the last iterate */
  CC_ERR_ARG = -1,       /* invalid argument (sizes, null pointers, options) */
  CC_ERR_OOM = -2,       /* device allocation failed or workspace limit exceeded */
  CC_ERR_HIP = -3,       /* HIP runtime error */
  CC_ERR_NAN = -4,       /* non-finite residual norm */
  CC_ERR_REJECTED = -5,  /* serving: request can never fit the memory budget */
  CC_ERR_INTERNAL = -6
} cc_status;

/* Internal compute precision of Jacobian-vector products; inputs and
 * outputs stay float64. FP32 and BF16 products use float accumulation. */
typedef enum { CC_FP64 = 0, CC_FP32 = 1, CC_BF16 = 2 } cc_precision;

typedef struct cc_handle cc_handle;

/* Create a handle on HIP device `device`. workspace_limit_bytes caps the
 * device memory the handle may hold (0: no cap). */
cc_status cc_create(cc_handle** h, int device, size_t workspace_limit_bytes);
void cc_destroy(cc_handle* h);
/* Text of the last error on this handle (valid until the next call). */
const char* cc_last_error(const cc_handle* h);

/* A closed-shell problem (Section "Theory"; gauge transformation f -> U f U^T
 * of Appendix A): Fock blocks and density-fitting factors with
 * (pq|rs) = sum_P L[P][p][q] L[P][r][s]. f must be symmetric
 * (f_vo = f_ov^T); L[P] must be symmetric. Any orthogonal gauge within the
 * occupied and within the virtual block is allowed (f_oo, f_vv need not be
 * diagonal; f_ov may be nonzero). */
typedef struct {
  int32_t nocc, nvir, naux;
  const double* f_oo; /* device [nocc][nocc] */
  const double* f_ov; /* device [nocc][nvir] */
  const double* f_vv; /* device [nvir][nvir] */
  const double* L;    /* device [naux][n][n] */
} cc_problem;

/* Bytes of device workspace a handle needs for this shape: the integral
 * tensors (including the (ac|bd) block, nvir^4 doubles), the intermediates
 * of the residual and its linearisation, and Krylov bases of m_max + 1 and
 * inner_restart + 1 vectors plus diis_size history pairs.
 * lowp_flags: bit 0 keeps FP32 copies, bit 1 BF16 copies of the constant
 * integral tensors for mixed-precision products. */
size_t cc_workspace_bytes(int32_t nocc, int32_t nvir, int32_t naux, int lowp_flags, int m_max, int inner_restart,
                          int diis_size);

/* CCSD residual r(t) (equation CC_ampl) into r1, r2. If e_corr_host is not
 * NULL the correlation energy E(t) - E_ref (equation CC_energy) is written
 * there (host) and the stream is synchronised. */
cc_status cc_residual(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, double* r1, double* r2,
                      double* e_corr_host, void* stream);

/* Correlation energy at (t1, t2), host output; synchronises. */
cc_status cc_energy(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, double* e_corr_host,
                    void* stream);

/* Jacobian-vector product J(t) v (the directional derivative of r at t
 * along v = (v1, v2); the analytic product of Appendix B carried through
 * every term) into jv1, jv2. `prec` is the compute precision of the
 * contractions of the product. Also evaluates r(t) to linearise. */
cc_status cc_jvp(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, const double* v1,
                 const double* v2, double* jv1, double* jv2, cc_precision prec, void* stream);

/* y = A_F x, the Fock operator of equation Preconditioner (Appendix C
 * working equations, extended to singles: (A_F x)_i^a = sum_c f_ac x_i^c -
 * sum_k f_ki x_k^a + sum_kc f_kc (2 x_ik^ac - x_ik^ca)). The paper's
 * normalisation factor 4 is absent (it cancels in preconditioning). */
cc_status cc_fock_apply(cc_handle* h, const cc_problem* p, const double* x1, const double* x2, double* y1,
                        double* y2, void* stream);

/* Solve A_F x = b (the preconditioner of equation Preconditioner, inverted
 * by GMRES as in Algorithm 1) to ||b - A_F x||_2 <= rtol ||b||_2 or maxit
 * A_F products; the product count goes to iters_out (host, may be NULL).
 * When f_ov = 0, A_F is symmetric and GMRES takes its Lanczos (MINRES)
 * form, run on D^1/2 A_F D^1/2 with D = 2 on the singles and 1 on the
 * doubles (same solution; the scaled residual bounds the true one).
 * Otherwise restarted GMRES (restart 30). Returns CC_NOT_CONVERGED when
 * maxit is reached first. Synchronises. */
cc_status cc_precond_solve(cc_handle* h, const cc_problem* p, const double* b1, const double* b2, double* x1,
                           double* x2, double rtol, int maxit, int* iters_out, void* stream);

/* cc_precond_solve for a pair-symmetric right-hand side, b2[j][i][b][a] =
 * b2[i][j][a][b], as every closed-shell amplitude vector is (the residual,
 * J v and their preconditioned images). When f_ov = 0 the Lanczos vectors
 * then hold only the pairs i <= j, which halves their memory traffic and
 * the virtual contractions. What is solved is the pair-symmetric part of b
 * ((b2[i][j] + b2[j][i]^T) / 2); x is pair-symmetric. Same arguments and
 * errors as cc_precond_solve. */
cc_status cc_precond_solve_pairsym(cc_handle* h, const cc_problem* p, const double* b1, const double* b2, double* x1,
                                   double* x2, double rtol, int maxit, int* iters_out, void* stream);

/* PNK options (Appendix F; Section "Adaptive Forcing").
 * tol_inf:   stop when ||r||_inf < tol_inf
 * max_newton: Newton steps cap
 * m_max:     GMRES iteration cap per Newton step (Krylov basis size)
 * gamma, alpha: Eisenstat-Walker eta_k = gamma (||r_k||/||r_{k-1}||)^alpha
 * eta0, eta_max: first forcing term and cap
 * inner_rtol, inner_maxit, inner_restart: GMRES for A_F^{-1}
 * jvp_prec:  compute precision of J v (outer quantities stay FP64)
 * use_fd_jvp: 1 = forward-difference product of equation
 *            jacobian_vector_product_via_finite_difference instead of the
 *            analytic one (FP64 only)
 * init_mp2:  1 = start from theta = -A_F^{-1} r(0); 0 = start from t1/t2
 * protocol:  outer solver of the method table: CC_PNK (Newton-GMRES
 *            preconditioned by A_F, Algorithm 1); CC_NK (the same without
 *            preconditioner; like every protocol it starts from the MP2
 *            amplitudes when init_mp2); CC_INK (t <- t + dt with
 *            A_F dt = -r(t), equation inexact_newton_update: one residual
 *            and one inner solve per step, max_newton of them; m_max and
 *            the forcing terms are unused)
 * ccd:       1 = the paper's CCD level: t1 is held at zero and the singles
 *            equations are dropped (t1 in and out is zero)
 * stall_window, stall_factor: stagnation stop (not in the paper; 0 = off):
 *            the solve ends as CC_NOT_CONVERGED, with info->stalled = 1,
 *            once stall_window Newton steps have passed without ||r||_inf
 *            falling below stall_factor times its value at the last step
 *            where it did (the first step counts as such)
 * inner_rtol_jv: tolerance of the inner solves of A_F^-1 (J q) inside the
 *            Krylov loop (0: inner_rtol). The right-hand side solve
 *            A_F^-1 r of each Newton step keeps inner_rtol. With J v in FP32
 *            or BF16 the products carry relative errors of about 1e-6 or
 *            1e-3, which bounds what a tighter inner solve can add */
typedef enum { CC_PNK = 0, CC_NK = 1, CC_INK = 2 } cc_protocol;

typedef struct {
  double tol_inf;
  int max_newton;
  int m_max;
  double gamma, alpha, eta0, eta_max;
  double inner_rtol;
  int inner_maxit;
  int inner_restart;
  cc_precision jvp_prec;
  int use_fd_jvp;
  int init_mp2;
  cc_protocol protocol;
  int ccd;
  int stall_window;
  double stall_factor;
  double inner_rtol_jv;
} cc_pnk_opts;

/* FP (+ level shift, + DIIS) options: t <- t - r/(D + level_shift) with D
 * from the diagonal of f in the given gauge (equation Commutator_MO;
 * Appendix D), DIIS over the last diis_size (amplitude, step) pairs from
 * iteration diis_start on (diis_size 0: plain FP); ccd as for PNK. */
typedef struct {
  double tol_inf;
  int max_iter;
  int diis_size;
  int diis_start;
  double level_shift;
  int init_mp2;
  int ccd;
} cc_fp_opts;

/* Solve statistics (host). n_residual and n_jvp count residual evaluations
 * and Jacobian products (the paper's cost measure); n_afmv counts A_F
 * products of the inner solves; stalled = 1 when the stagnation stop of
 * cc_pnk_opts ended the solve. */
typedef struct {
  double e_corr, res_inf, res_2;
  int converged, newton_iters, n_residual, n_jvp, n_afmv, n_inner_iters;
  double seconds;
  int stalled;
} cc_info;

/* Defaults: tol 1e-8, 100 Newton steps, m_max 20, gamma 0.9, alpha 1.5,
 * eta0 0.5, eta_max 0.9, inner rtol 1e-12, inner maxit 200, restart 30,
 * FP64 products, analytic J v, MP2 start, PNK, CCSD, no stagnation stop
 * (stall_window 0, stall_factor 0.5), inner_rtol_jv 0 (= inner_rtol). */
void cc_pnk_opts_default(cc_pnk_opts* o);
/* Defaults: tol 1e-8, 500 iterations, DIIS 8 from iteration 2, no shift,
 * MP2 start, CCSD. */
void cc_fp_opts_default(cc_fp_opts* o);

/* PNK solve. t1/t2: in = initial guess when !init_mp2, out = solution (or
 * last iterate). info (host) may be NULL. Returns CC_OK, CC_NOT_CONVERGED or
 * CC_ERR_NAN (non-finite residual; outputs hold the last iterate).
 * Synchronises. */
cc_status cc_solve_pnk(cc_handle* h, const cc_problem* p, const cc_pnk_opts* opts, double* t1, double* t2,
                       cc_info* info, void* stream);

/* FP/SFP(+DIIS) solve; same contract as cc_solve_pnk. A residual norm above
 * 1e6 ends the iteration as CC_NOT_CONVERGED (divergence). */
cc_status cc_solve_fp_diis(cc_handle* h, const cc_problem* p, const cc_fp_opts* opts, double* t1, double* t2,
                           cc_info* info, void* stream);

/* Spectral radius of the Jacobian of the (S)FP map t -> t - r(t) / (D +
 * shift), G = I - diag(D + shift)^-1 J(t), with D the Jacobi denominators of
 * the diagonal of f in the given gauge (Section "Regularization": FP
 * converges locally when this radius is below one; the shift is the Ridge
 * term of Appendix D). J is linearised at (t1, t2) (device). G acts on
 * pair-symmetric vectors: m Arnoldi steps (CGS2) from the start vector (q1,
 * q2) (device, nonzero, pair-symmetric), the projection (x2[i][j] +
 * x2[j][i]^T) / 2 after every product. rho_out (host) receives the largest
 * modulus of the Ritz values; ritz_re / ritz_im (host, m entries each, may
 * be NULL) the Ritz values, n_ritz (may be NULL) their number (less than m
 * when the Krylov space became invariant). CC_ERR_ARG for a zero start or
 * m outside 1..200. Synchronises. */
cc_status cc_fp_spectral_radius(cc_handle* h, const cc_problem* p, const double* t1, const double* t2, const double* q1,
                                const double* q2, double shift, int m, double* rho_out, double* ritz_re,
                                double* ritz_im, int* n_ritz, void* stream);

/* ---------------------------------------------------------------------
 * Non-orthogonal and redundant orbital gauges (Appendix A, random gauge
 * representation).
 *
 * Per orbital block, m gauge functions chi = phi W that span the block's
 * orbitals but need be neither orthonormal nor independent: w_oo
 * [nocc][m_occ] and w_vv [nvir][m_vir] (DEVICE, FP64, row-major,
 * caller-owned, full row rank, m >= the block size; m_occ = 0 or m_vir = 0
 * means the square case m = nocc or nvir), column mu holding gauge function
 * mu expanded in the orthonormal orbitals of the problem (the orbitals f
 * and L are given in). The gauge functions overlap as S = W^T W, singular
 * when m exceeds the block size (a redundant gauge, as projected atomic
 * orbitals are). The orbital coefficients in them are C = W^+ =
 * W^T (W W^T)^-1 (W^-1 for square W). The gauge amplitudes are the
 * covariant components (the appendix's theta = U-bar^(x4) t with
 * U-bar = S U = W^T), of shapes th1 [m_occ][m_vir] and th2
 * [m_occ][m_occ][m_vir][m_vir]:
 *   th1[mu][lam]          = sum_ia W_o[i][mu] W_v[a][lam] t1[i][a]
 *   th2[mu][nu][lam][sig] = sum W_o[i][mu] W_o[j][nu] W_v[a][lam] W_v[b][sig] t2[i][j][a][b]
 * and the gauge residual is r(theta) = U-bar^(x4) r(t(theta)) with
 * t(theta) = C^(x4) theta. Amplitudes and residuals lie in the range of
 * U-bar^(x4); for a redundant gauge the components of theta outside it
 * change neither t(theta) nor r(theta), the Jacobian is singular there and
 * the solves below return amplitudes in the range. The gauge's Fock blocks
 * W^T f C^T make its A_F non-symmetric; its inverse on the range is
 * applied as U-bar^(x4) A_F^-1 C^(x4) with the orbital-basis inner solve.
 * The FP denominators are the diagonals of those blocks (the appendix's FP
 * update). Each call copies W to the host and inverts W (square) or W W^T
 * (Gauss-Jordan, partial pivoting): CC_ERR_ARG for a W that is not finite
 * or not of full row rank, or m below the block size. The handle keeps
 * 3 N + N_g + 2 (m_occ m_vir)^2 doubles of gauge buffers (N = o v +
 * o^2 v^2, N_g = m_occ m_vir + (m_occ m_vir)^2) once a gauge call has run,
 * and a gauge solve sizes its outer Krylov and DIIS vectors for N_g. All
 * calls synchronise.
 * --------------------------------------------------------------------- */
typedef struct {
  const double* w_oo;
  const double* w_vv;
  int m_occ; /* gauge functions of the occupied block (0: nocc) */
  int m_vir; /* gauge functions of the virtual block (0: nvir) */
} cc_gauge;

/* y = U-bar^(x4) x (to_gauge != 0: orbital amplitudes or residuals
 * (x1 [o][v], x2 [o][o][v][v]) to the gauge's (y1 [m_occ][m_vir], y2
 * [m_occ][m_occ][m_vir][m_vir])) or y = C^(x4) x (to_gauge == 0: gauge
 * components to orbital ones, the inverse of the first on its range), all
 * device; y must not overlap x. */
cc_status cc_gauge_transform(cc_handle* h, const cc_problem* p, const cc_gauge* g, int to_gauge, const double* x1,
                             const double* x2, double* y1, double* y2, void* stream);

/* Gauge residual (r1, r2) at gauge amplitudes (th1, th2), all device, and
 * optionally the correlation energy (gauge invariant) to e_corr_host. */
cc_status cc_residual_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const double* th1,
                            const double* th2, double* r1, double* r2, double* e_corr_host, void* stream);

/* J v of the gauge residual at (th1, th2) in direction (v1, v2): the
 * orbital-basis product of cc_jvp (precision prec) between the transforms. */
cc_status cc_jvp_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const double* th1, const double* th2,
                       const double* v1, const double* v2, double* jv1, double* jv2, cc_precision prec,
                       void* stream);

/* PNK / FP(+DIIS) solves on the gauge amplitudes: the contracts of
 * cc_solve_pnk / cc_solve_fp_diis with (th1, th2) gauge amplitudes in and
 * out, the stopping test on the gauge residual's ||r||_inf. */
cc_status cc_solve_pnk_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const cc_pnk_opts* opts,
                             double* th1, double* th2, cc_info* info, void* stream);
cc_status cc_solve_fp_diis_gauge(cc_handle* h, const cc_problem* p, const cc_gauge* g, const cc_fp_opts* opts,
                                 double* th1, double* th2, cc_info* info, void* stream);

/* Residual history of the last solve on the handle: pairs (||r||_2,
 * ||r||_inf) per outer residual evaluation, up to max_pairs written to
 * `pairs` (host, 2 * max_pairs doubles); returns the number available. */
int cc_last_history(const cc_handle* h, double* pairs, int max_pairs);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of PNK solves on one GPU.
 *
 * Requests carry HOST problem arrays that are copied at submission and
 * dropped once the solve has consumed them. A scheduler admits queued
 * requests while a slot is free and the request's device footprint
 * (cc_workspace_bytes of its shape and options plus its problem arrays)
 * fits in the unused part of mem_budget: the first one in arrival order
 * that fits, except that a request passed over 2 * max_slots times by later
 * ones blocks those behind it until it runs. Admitted requests run
 * concurrently, each on its own stream, so their kernels overlap on the
 * device. A finished request frees its problem arrays and slot and leaves
 * its handle (integral workspace, recorded graphs, Krylov bases) in a cache
 * keyed by (nocc, nvir, naux, precision) for a later request of the same
 * key; cached handles count against mem_budget and the least recently used
 * are freed when a queued request needs the room. A request whose footprint
 * exceeds the whole budget is rejected at submission (CC_ERR_REJECTED).
 * Each result depends only on its own request: the same kernels and launch
 * shapes run whatever else is in flight, on a fresh or a cached handle.
 * --------------------------------------------------------------------- */
typedef struct cc_server cc_server;

/* max_slots: solves in flight at once; mem_budget: device bytes for all of
 * them (0: 90% of the free device memory). */
cc_status cc_server_create(cc_server** s, int device, size_t mem_budget, int max_slots);
/* Copy the host problem (f_oo, f_ov, f_vv, L are HOST pointers here) and
 * queue a PNK solve; *req_id receives its id. opts may be NULL (defaults). */
cc_status cc_server_submit(cc_server* s, const cc_problem* p_host, const cc_pnk_opts* opts, uint64_t* req_id);
/* Non-blocking: *done = 1 when finished, then info (may be NULL) and the
 * solution (t1_host [o][v], t2_host [o][o][v][v], may be NULL) are copied
 * out and the request is released (only its times are kept; a later poll of
 * the same id is CC_ERR_ARG). Returns the solve's own status once done. */
cc_status cc_server_poll(cc_server* s, uint64_t req_id, int* done, cc_info* info, double* t1_host, double* t2_host);
/* Wait until every submitted request has finished. */
cc_status cc_server_drain(cc_server* s);
/* Admission/latency figures (host): queued, running, finished counts, peak
 * bytes admitted at once (cached handles included), the host memory still
 * held for requests, and the handle cache; cc_server_request_times gives
 * one request's submit/admit/finish times in seconds since server creation
 * (also after it was collected). */
typedef struct {
  uint64_t queued, running, finished, rejected;
  size_t bytes_in_use, peak_bytes, budget;
  int max_slots, peak_running;
  size_t host_bytes_held;   /* host copies of inputs and results not yet collected */
  uint64_t requests_held;   /* requests submitted and not yet collected by a done poll */
  size_t cached_bytes;      /* device bytes of cached idle handles (part of bytes_in_use) */
  uint64_t cached_handles, handle_reuses;
} cc_server_stats;
cc_status cc_server_get_stats(cc_server* s, cc_server_stats* st);
cc_status cc_server_request_times(cc_server* s, uint64_t req_id, double* t_submit, double* t_admit,
                                  double* t_finish);
void cc_server_destroy(cc_server* s);

/* ---------------------------------------------------------------------
 * Diagnostics (for kernel tests; not part of the solver path)
 * --------------------------------------------------------------------- */
/* Device timing of tagged work on the handle, with HIP events recorded on
 * the stream each launch runs on. Slots: 0 the particle-particle ladder
 * contraction (one launch per residual or J v), 1 whole residual
 * evaluations, 2 whole J v products, 3 A_F products, 4 inner A_F solves.
 * cc_diag_timing(h, 1) enables and resets; cc_diag_timing_read synchronises
 * the recorded events and returns the launch count and total milliseconds
 * of one slot. */
cc_status cc_diag_timing(cc_handle* h, int enable);
cc_status cc_diag_timing_read(cc_handle* h, int slot, int* count, double* total_ms);

/* Matrix-core flops of one residual evaluation (equations CC_ampl and
 * CC_energy as implemented: T1-dressed terms, symmetry-adapted ladder) and
 * of one J v product in precision prec, counted as 2 M N K per contraction
 * at the contractions' own sizes (the tiles' padding is not counted): the
 * algorithmic flop count of the roofline figures. Runs one eager residual
 * and J v at t = 0 on the handle (problem device arrays as for
 * cc_residual) and writes the two counts to the host doubles. Synchronises. */
cc_status cc_diag_contraction_flops(cc_handle* h, const cc_problem* p, cc_precision prec, double* residual_flops,
                                    double* jvp_flops, void* stream);

/* Eigenvalues of an m x m real upper Hessenberg matrix H (host, row-major;
 * entries below the subdiagonal ignored) into re[m], im[m] (host), by the
 * shifted QR iteration the spectral-radius call uses (host code, no GPU).
 * CC_NOT_CONVERGED if the iteration stalls. */
cc_status cc_diag_hessenberg_eigenvalues(int m, const double* H, double* re, double* im);

/* The position sets of the occupied A_F kernel on the packed pair layout
 * (the o x o contractions of the A_F product, Appendix A.7, for each
 * virtual pair (a, b)): every workgroup takes 64 positions closed under
 * (a, b) -> (b, a). For nvir virtuals, writes for set u and lane l the
 * position a[64 u + l], b[64 u + l] (entries >= nvir mark padding lanes)
 * and lane_t[64 u + l], the lane of the same set holding (b, a); *nsets
 * receives the set count. Host arrays of cap elements each; host code, no
 * GPU. CC_ERR_ARG for null pointers, nvir < 1 or cap < 64 * nsets. */
cc_status cc_diag_occ_sets(int nvir, int* a, int* b, int* lane_t, int64_t cap, int* nsets);

/* C = alpha * A * B + beta * C with element strides (A[m*a_m + k*a_k],
 * B[k*b_k + n*b_n], C[m*c_m + n*c_n]), all float64 device arrays, computed
 * on the matrix cores in precision `prec` (FP32/BF16: float accumulation).
 * This is the contraction kernel every residual term runs on. */
cc_status cc_diag_gemm(int M, int N, int K, const double* A, int64_t a_m, int64_t a_k, const double* B,
                       int64_t b_k, int64_t b_n, double* C, int64_t c_m, int64_t c_n, double alpha, double beta,
                       cc_precision prec, void* stream);

/* Batched cc_diag_gemm: C[b] = alpha A[b] B[b] + beta C[b] for b < nbatch,
 * with batch strides a_b, b_b, c_b (elements) added to the three base
 * pointers. flags bit 0: round FP64 operands of an FP32/BF16 product once
 * into a scratch copy (rows contiguous along k) before the product, as the
 * residual and J v do for their large products; bit 1: allow split-K (the
 * contraction cut into chunks whose partial sums are added in a fixed
 * order) when the output tiles cannot fill the GPU. The scratch memory is
 * allocated and freed inside the call (diagnostics only). Synchronises. */
cc_status cc_diag_gemm_batched(int M, int N, int K, int nbatch, const double* A, int64_t a_m, int64_t a_k,
                               int64_t a_b, const double* B, int64_t b_k, int64_t b_n, int64_t b_b, double* C,
                               int64_t c_m, int64_t c_n, int64_t c_b, double alpha, double beta, cc_precision prec,
                               int flags, void* stream);

/* ---------------------------------------------------------------------
 * Allocation-free product (for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).
 *
 * cc_gemm_noalloc takes the arguments of cc_diag_gemm_batched and computes
 * the same product with the same kernels and the same split-K chunks (its
 * results are bitwise those of cc_diag_gemm_batched), but allocates
 * nothing: its scratch (split-K partial sums, at most 4 Mi doubles, and the
 * operand copies of flags bit 0, at most 32 MiB) is a fixed 64 MiB array
 * that the library holds on each device it runs on until the process ends.
 * A product whose rounded operand copies (2 bytes per element for BF16, 4
 * for FP32, nbatch * (M + N) * K' elements, K' = K rounded up to a multiple
 * of 8 for BF16 and of 4 for FP32) exceed 32 MiB is refused with
 * CC_ERR_OOM before any work is queued; split-K uses at most the 4 Mi
 * doubles (fewer chunks when a product would need more). All calls on one
 * device share its array: calls that overlap in time on one device race
 * and must be ordered by the caller (one stream, or events). Does not
 * synchronise; device pointers as for cc_diag_gemm_batched.
 * --------------------------------------------------------------------- */
cc_status cc_gemm_noalloc(int M, int N, int K, int nbatch, const double* A, int64_t a_m, int64_t a_k, int64_t a_b,
                          const double* B, int64_t b_k, int64_t b_n, int64_t b_b, double* C, int64_t c_m,
                          int64_t c_n, int64_t c_b, double alpha, double beta, cc_precision prec, int flags,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PNKCC_H */
