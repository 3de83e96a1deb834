// Fock operator y = A_F x (equation Preconditioner, Appendix C working
// equations extended to singles), f_ov-free part, in two launches:
//
//   y_ij^ab = sum_c f_ac x_ij^cb + sum_c x_ij^ac f_cb      (virtual kernel)
//             - sum_k f_ki x_kj^ab - sum_k f_kj x_ik^ab     (occupied kernel)
//   y_i^a   = sum_c f_ac x_i^c - sum_k f_ki x_k^a          (occupied kernel)
//
// f_oo and f_vv are symmetric (any orthogonal gauge). Vectors are packed as
// [x1 (o*v) | x2 (o*o*v*v)], x1[i][a], x2[i][j][a][b].
//
// The occupied launch can also carry the first Lanczos update of the inner
// solve: p = A_F v_k - beta_k v_{k-1} (singles rows optionally scaled) and
// per-workgroup partial sums of <v_k, p>, <p, p> and <v_k, v_k>.
#pragma once

#include "common.hpp"

namespace pnk {

constexpr int kFockOpMaxOcc = 31;  // the occupied kernel stages o^2 slices in LDS

struct FockOp {
  int o = 0, v = 0;
  const double* f_oo = nullptr;
  const double* f_vv = nullptr;
  // set by fock_op_plan
  int bm = 0, tiles = 0;    // virtual kernel: bm x bm blocks, tiles per pair
  int ch = 0, nchunks = 0;  // occupied kernel: ch (ab) elements per workgroup
  int nsingles = 0;         // ... plus workgroups of 16 singles each
  // occupied kernel on the packed pair layout: pt x pt tiles (and their
  // mirrors), pntile tiles per side, pnchunks = pntile (pntile + 1) / 2
  // psplit workgroups share a tile, each taking every psplit-th pair;
  // pdwg = pnchunks * psplit rounded up to a multiple of 8 (XCD grouping)
  int npair = 0, pt = 0, pntile = 0, pnchunks = 0, psplit = 1, pdwg = 0;
  // register-blocked form (used when its staging fits a workgroup's LDS):
  // psets = 1, sets of 64 positions over pnb = ceil(v / 8) blocks per side
  // (pnb^2 sets), each split over pbsplit workgroups by its pnblk 4 x 4
  // blocks of the upper triangle of the o x o output; pdwg counts these
  // workgroups instead
  int psets = 0, pnb = 0, pbsplit = 1, pnblk = 0, pnw = 4;  // pnw: waves per workgroup
  int64_t nparts() const { return (int64_t)nchunks + nsingles; }
  int psingles = 0;  // singles workgroups of the packed form
  int64_t nparts_packed() const { return (int64_t)pdwg + psingles; }
};

// Picks the launch shapes; false when these kernels do not apply (o too
// large) and the caller must use the general path.
bool fock_op_plan(FockOp& op);

// Host copy of the occupied kernel's position sets for v virtuals: for set
// u and lane l, a[64 u + l], b[64 u + l] is the lane's (a, b) (past v: a
// padding lane) and lt[64 u + l] the lane holding (b, a). Returns the set
// count, or -1 when v < 1 or cap (elements per array) is too small.
int fock_op_set_positions(int v, int* a, int* b, int* lt, int64_t cap);

// y = A_F x (y must not alias x)
void fock_op_apply(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, hipStream_t s);

// The same two launches on packed vectors with the first Lanczos update:
// fock_op_lanczos_vir writes the virtual part of A_F v into p; then
// fock_op_lanczos_occ completes p = S A_F v - (*beta) vprev and writes, for
// each workgroup b, its shares of v . p, p . p and v . v in partials[b],
// partials[nparts + b] and partials[2 nparts + b] (nparts = op.nparts(),
// each share summed in a fixed order). beta is a device scalar; S
// multiplies the singles rows by singles_scale and leaves the doubles rows
// alone. done is a device flag: when it is nonzero as a launch starts, the
// launch writes nothing (a converged solve can leave queued steps behind).
void fock_op_lanczos_vir(const FockOp& op, const double* v, double* p, const double* done, hipStream_t s);
void fock_op_lanczos_occ(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                         double* partials, double singles_scale, const double* done, hipStream_t s);

// The same Lanczos step on the packed pair layout of pair-symmetric vectors
// (x2[j][i] = x2[i][j]^T): [x1 (o*v) | x2 for pairs i <= j, pair P(i, j) =
// i o - i (i - 1) / 2 + j - i, each v*v]. The three partial sums are those
// of the full vectors (the blocks of pairs i < j count twice); partials has
// 3 op.nparts_packed() entries. The virtual part comes from
// fock_op_lanczos_vir_packed (three-launch step: then a separate update) or
// fock_op_lanczos_vir_fused below (two-launch step).
void fock_op_lanczos_vir_packed(const FockOp& op, const double* v, double* p, const double* done, hipStream_t s);
void fock_op_lanczos_occ_packed(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                                double* partials, double singles_scale, const double* done, hipStream_t s);

// State of the symmetric inner solve (device scalars, kLzStateStride
// doubles per slot; slot j holds the state after step j's update): [0]
// beta_j, [1] alpha, [2] beta_{j+1}, [3..6] c_{j-1}, s_{j-1}, c_j, s_j, [7]
// phibar, [8] rho1, [9] delta, [10] eps, [11] phi, [12] |phibar| (the
// residual estimate), [13] 1/beta, [14] done (the stopping test held), [15]
// first (the next step only normalises the start vector). A third slot,
// `fin`, holds what the host reads: steps run, the last residual estimate
// and beta, the absolute tolerance, ||b|| and the start vector's norm.
constexpr int kLzStateStride = 16;
enum { kLzBeta = 0, kLzAlpha, kLzBetaN, kLzC2, kLzS2, kLzC1, kLzS1, kLzPhiBar, kLzRho1, kLzDelta, kLzEps, kLzPhi,
       kLzRes, kLzInvB, kLzDone, kLzFirst, kLzNState };
enum { kLzFinSteps = 0, kLzFinRes, kLzFinBeta, kLzFinTol, kLzFinBNorm, kLzFinBHat, kLzFinCount };
static_assert(kLzNState <= kLzStateStride && kLzFinCount <= kLzStateStride, "Lanczos state slot too small");

// Step k of the packed symmetric solve, first launch: the update of step
// k-1 fused with the virtual part of step k. From the shares of <v,p>,
// <p,p>, <v,v> of the last occupied launch (partials, nparts each) it
// takes alpha_{k-1}, beta_k, the Givens rotation and the stopping test
// (state st -> stn, fin), writes v_k = (P - alpha V) / beta_k to Vn, the
// MINRES updates w2 = (V - delta w1 - eps w2) / rho and x += phi w2, and
// the virtual part of A_F v_k to the doubles of Y. P, V, Vn, Y, w1, w2, x
// are packed vectors; Vn and Y must differ from P, V and each other. With
// the first flag set in st it only normalises (P = start vector, V = 0,
// shares (0, ||P||^2, 0)). When st is done it passes the flag on.
void fock_op_lanczos_vir_fused(const FockOp& op, const double* P, const double* V, double* Vn, double* Y, double* w1,
                               double* w2, double* x, const double* partials, int nparts, const double* st,
                               double* stn, double* fin, hipStream_t s);

// Whether the packed symmetric solve takes two launches per step (the
// update fused into fock_op_lanczos_vir_fused): for 32-wide blocks, where
// a workgroup's update is one batch of four elements per thread. Wider
// blocks would stream several batches ahead of their matrix-core product,
// so they keep the separate update launch (three launches per step).
bool fock_op_fused_step(const FockOp& op);

// True for the launch of a Lanczos step that is timed in a recorded graph:
// the fused first launch in the two-launch form (fused), else the occupied
// launch.
bool fock_op_is_timed_lanczos_kernel(const void* func, bool fused);

}  // namespace pnk
