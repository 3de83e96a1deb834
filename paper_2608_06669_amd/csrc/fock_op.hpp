// Fused Fock operator y = A_F x (equation Preconditioner, Appendix C working
// equations extended to singles) for f_ov = 0, in one kernel launch:
//
//   y_ij^ab = sum_c f_ac x_ij^cb + sum_c x_ij^ac f_cb
//             - sum_k f_ki x_kj^ab - sum_k f_kj x_ik^ab
//   y_i^a   = sum_c f_ac x_i^c - sum_k f_ki x_k^a
//
// f_oo and f_vv are symmetric (any orthogonal gauge). Vectors are packed as
// [x1 (o*v) | x2 (o*o*v*v)], x1[i][a], x2[i][j][a][b].
//
// The same launch can also carry the first Lanczos update of the inner
// solve: p = A_F v_k - beta_k v_{k-1} together with per-workgroup partial
// sums of <v_k, p>, so the operator's output is never re-read for it.
#pragma once

#include "common.hpp"

namespace pnk {

struct FockOp {
  int o = 0, v = 0;
  const double* f_oo = nullptr;
  const double* f_vv = nullptr;
  // set by fock_op_plan
  int bm = 0, tiles = 0, gx = 0, gy = 0;
  int64_t nparts() const { return (int64_t)gx * gy; }
};

// Picks the tile shape; returns false when the fused kernel does not apply
// (o > kFockOpMaxOcc) and the caller must use the general path.
constexpr int kFockOpMaxOcc = 256;
bool fock_op_plan(FockOp& op);

// y = A_F x (the f_ov-free part; y must not alias x)
void fock_op_apply(const FockOp& op, const double* x1, const double* x2, double* y1, double* y2, hipStream_t s);

// Packed vectors: p = A_F v - (*beta) vprev and partials[b] = sum over
// workgroup b of v . p (op.nparts() entries, each summed in a fixed order).
// beta is a device scalar.
void fock_op_lanczos(const FockOp& op, const double* v, const double* vprev, const double* beta, double* p,
                     double* partials, hipStream_t s);

// True for the kernel function that fock_op_lanczos launches (used to find
// its nodes in a recorded graph).
bool fock_op_is_lanczos_kernel(const void* func);

}  // namespace pnk
