// Amplitudes in a non-orthogonal, possibly redundant orbital gauge
// (Appendix A, random gauge representation).
//
// Per orbital block the gauge functions are chi = phi W with W of full row
// rank (W_o: o x m_o, W_v: v x m_v, m >= the block size; column mu holds
// gauge function mu in the orthonormal orbitals of its block), overlapping
// as S = W^T W. The orbital coefficients in the gauge functions are
// C = W^+ = W^T (W W^T)^-1 (W^-1 when W is square). The gauge amplitudes are
// the covariant components theta = (W^T)^(x4) t, and the residual
// transforms the same way: r(theta) = (W^T)^(x4) r(t(theta)),
// t = (C^T)^(x4) theta. The one-body part of the residual acts on a gauge
// index through F = W^T f C^T (per block, m x m), so A_F of the gauge is
// (W^T)^(x4) A_F (C^T)^(x4). On the range of (W^T)^(x4) (where amplitudes
// and residuals lie) it is invertible, with inverse the orbital-basis
// inverse between the two transforms; with m > n it is singular on the
// complement of that range, which neither t(theta) nor r(theta) sees.
#pragma once

#include "common.hpp"

namespace pnk {

struct Gauge {
  int o = 0, v = 0;    // orbital block sizes
  int mo = 0, mv = 0;  // gauge functions per block
  // row-major: fwd_o = W_o^T [mo][o], bwd_o = C_o^T [o][mo], Fo = W_o^T f_oo C_o^T [mo][mo];
  // likewise for the virtual block
  double *fwd_o = nullptr, *fwd_v = nullptr, *bwd_o = nullptr, *bwd_v = nullptr;
  double *Fo = nullptr, *Fv = nullptr;
  // orbital-length work vectors: t holds the orbital-basis amplitudes of the
  // last residual (the point J v is linearised at); w1, w2 scratch
  double *t = nullptr, *w1 = nullptr, *w2 = nullptr;
  // gauge-length packed vector (the iterate of a gauge solve) and the
  // intermediates of the four-index transforms (mo^2 mv^2 each)
  double *xg = nullptr, *ta = nullptr, *tb = nullptr;
  int64_t nvec() const { return (int64_t)mo * mv + (int64_t)mo * mo * mv * mv; }
};

// Doubles of the matrices and vectors a Gauge holds.
int64_t gauge_matrix_elems(int o, int v, int mo, int mv);
int64_t gauge_vector_elems(int o, int v, int mo, int mv);

// y = (A_o (x) A_o (x) A_v (x) A_v) x with A_o [po][qo], A_v [pv][qv]
// row-major [out][in], on x1 [qo][qv], x2 [qo][qo][qv][qv] into
// y1 [po][pv], y2 [po][po][pv][pv]:
//   y1[mu][lam] = sum A_o[mu][i] A_v[lam][a] x1[i][a],
//   y2[mu][nu][lam][sig] = sum A_o[mu][i] A_o[nu][j] A_v[lam][a] A_v[sig][b] x2[i][j][a][b]
// as six matrix-core products through ta, tb, which must hold
// max(qo^2 qv pv, qo po pv^2) and qo^2 pv^2 doubles. The x, y, ta, tb
// arrays must not overlap.
void gauge_apply(int qo, int qv, int po, int pv, const double* Ao, const double* Av, const double* x1,
                 const double* x2, double* y1, double* y2, double* ta, double* tb, hipStream_t s);

// Gauss-Jordan inverse with partial pivoting (host, row-major n x n).
// Returns false when a pivot falls below 1e-13 of the largest entry.
bool invert_matrix(int n, const double* A, double* Ainv);

// Fills the matrices of g (its pointers and sizes set) from W_o [o][mo],
// W_v [v][mv], f_oo and f_vv (device, row-major). Synchronises s. Throws
// ArgError when a W is not of full row rank or not finite.
void gauge_setup(Gauge& g, const double* w_oo, const double* w_vv, const double* f_oo, const double* f_vv,
                 hipStream_t s);

}  // namespace pnk
