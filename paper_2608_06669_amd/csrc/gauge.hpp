// Amplitudes in a non-orthogonal orbital gauge (Appendix A, random gauge
// representation).
//
// Per orbital block the gauge functions are chi = phi W with W invertible
// (W_o: o x o, W_v: v x v; column mu holds gauge function mu in the
// orthonormal orbitals of its block), overlapping as S = W^T W. The gauge
// amplitudes are the covariant components theta = (W^T)^(x4) t, and the
// residual transforms the same way: r(theta) = (W^T)^(x4) r(t(theta)),
// t = (W^-T)^(x4) theta. The one-body part of the residual acts on a gauge
// index through F = W^T f W^-T (per block), so A_F of the gauge is the
// similarity transform (W^T)^(x4) A_F (W^-T)^(x4): not symmetric, but its
// inverse is the orbital-basis inverse between the two transforms.
#pragma once

#include "common.hpp"

namespace pnk {

struct Gauge {
  int o = 0, v = 0;
  // row-major [o][o] / [v][v]: fwd = W^T, bwd = W^-T, Fo/Fv = W^T f W^-T
  double *fwd_o = nullptr, *fwd_v = nullptr, *bwd_o = nullptr, *bwd_v = nullptr;
  double *Fo = nullptr, *Fv = nullptr;
  // work vectors: t holds the orbital-basis amplitudes of the last residual
  // (the point J v is linearised at); w1, w2 packed vectors; ta, tb
  // o*o*v*v intermediates of the four-index transform
  double *t = nullptr, *w1 = nullptr, *w2 = nullptr, *ta = nullptr, *tb = nullptr;
};

// Doubles of the packed matrices and vectors a Gauge holds for (o, v).
int64_t gauge_matrix_elems(int o, int v);
int64_t gauge_vector_elems(int o, int v);

// y = (A_o (x) A_o (x) A_v (x) A_v) x on packed vectors [x1 (o*v) | x2
// (o*o*v*v)], A row-major [out][in]:
//   y1[mu][lam] = sum A_o[mu][i] A_v[lam][a] x1[i][a],
//   y2[mu][nu][lam][sig] = sum A_o[mu][i] A_o[nu][j] A_v[lam][a] A_v[sig][b] x2[i][j][a][b]
// as six matrix-core products through ta, tb (o*o*v*v each). x, y, ta, tb
// must not overlap.
void gauge_apply(int o, int v, const double* Ao, const double* Av, const double* x, double* y, double* ta,
                 double* tb, hipStream_t s);

// Gauss-Jordan inverse with partial pivoting (host, row-major n x n).
// Returns false when a pivot falls below 1e-13 of the largest entry.
bool invert_matrix(int n, const double* A, double* Ainv);

// Fills the matrices of g (its pointers set, o and v set) from W_o, W_v,
// f_oo and f_vv (device, row-major). Synchronises s. Throws ArgError when
// a W is singular or not finite.
void gauge_setup(Gauge& g, const double* w_oo, const double* w_vv, const double* f_oo, const double* f_vv,
                 hipStream_t s);

}  // namespace pnk
