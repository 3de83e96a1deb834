// Eigenvalues of a small real upper Hessenberg matrix on the host (the
// Ritz values of an Arnoldi process).
#pragma once

namespace pnk {

// H: m x m, row-major, upper Hessenberg (entries below the subdiagonal are
// ignored). Writes the m eigenvalues to re[], im[] (no particular order).
// Returns false if the iteration did not converge.
bool hessenberg_eigenvalues(const double* H, int m, double* re, double* im);

}  // namespace pnk
