// Small problem-specific kernels of the CCSD path (bandwidth or latency
// bound): integral block extraction, Fock assembly, traces, the energy
// reduction and the Jacobi update.
#pragma once

#include "common.hpp"

namespace pnk {

// f[n][n] from f_oo [o][o], f_ov [o][v], f_vv [v][v] (f_vo = f_ov^T)
void assemble_fock(int o, int v, const double* f_oo, const double* f_ov, const double* f_vv, double* f,
                   hipStream_t s);
// Lo[P][k][q] = L[P][k][q] for k < o (rows of the occupied orbitals)
void extract_occ_rows(int naux, int o, int n, const double* L, double* Lo, hipStream_t s);
// Blocks of the np = naux + 1 slices [L[0..naux-1]; h]: oo [np][o][o],
// ov [np][o][v], vo [np][v][o], vv [np][v][v]
void extract_blocks(int naux, int o, int v, const double* L, const double* h, double* Loo, double* Lov,
                    double* Lvo, double* Lvv, hipStream_t s);
// D[P] = sum_k X[P][k][k] for P < nslices, X of shape [.][o][o]
void trace_slices(int nslices, int o, const double* X, double* D, hipStream_t s);
// d[P] = sum_{k<o} L[P][k][k], L of shape [naux][n][n]
void trace_occ(int naux, int o, int n, const double* L, double* d, hipStream_t s);
// E = 2 sum f_ov t1 + sum_ijab Itil (t2 + t1_ia t1_jb) -> out (device), deterministic
void energy(int o, int v, const double* f_ov, const double* Itil, const double* t1, const double* t2, double* out,
            double* partials, hipStream_t s);
// t <- t - r / (D + shift) with Jacobi denominators from diag(f_oo), diag(f_vv);
// e = -r / (D + shift) is written to `step` when it is not null
void jacobi_update(int o, int v, const double* f_oo, const double* f_vv, double shift, const double* r, double* t,
                   double* step, hipStream_t s);
// Symmetry-adapted particle-particle ladder. Pairs a <= b are numbered
// row-major over the upper triangle (p), pairs a < b likewise (p'), and
// occupied pairs i <= j likewise; pair_a/pair_b map a packed index back.
// S[p][q] = W_ab,cd + W_ab,dc and A[p'][q'] = W_ab,cd - W_ab,dc for the
// rows whose a lies in [a0, a0 + na); Wblk[a - a0][b][c][d] = (ac|bd).
void ppl_pack_w(int v, int a0, int na, const double* Wblk, const int* pair_a, const int* pair_b,
                const int* mpair_a, const int* mpair_b, double* S, double* A, hipStream_t s);
// Tp[ij][q] = (t_ij^cd + t_ij^dc)/2 (c < d) or t_ij^cc / 2 (c = d);
// Tm[ij][q'] = (t_ij^cd - t_ij^dc)/2, for i <= j.
void ppl_pack_t(int o, int v, const double* t2, const int* pair_a, const int* pair_b, const int* mpair_a,
                const int* mpair_b, double* Tp, double* Tm, hipStream_t s);
// R[i][j][a][b] += sum_cd (ac|bd) t_ij^cd rebuilt from Rp = Tp S, Rm = Tm A.
void ppl_unpack_add(int o, int v, const double* Rp, const double* Rm, double* R, hipStream_t s);

// y = x / *s_dev (the divisor stays on the device; y = 0 when it is 0)
void scale_by_inverse(int64_t n, const double* x, const double* s_dev, double* y, hipStream_t s);

}  // namespace pnk
