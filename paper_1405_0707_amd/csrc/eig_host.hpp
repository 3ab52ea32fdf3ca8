// Host eigensolvers for the small projected matrix of the restart step.
#pragma once

#include <vector>

namespace expmv {

// A (n x n, row-major) symmetric part -> eigenvalues w (n) and orthonormal
// eigenvectors in the columns of Q (n x n row-major): A = Q diag(w) Q^T.
// Returns false if the QR iteration did not deflate every off-diagonal
// entry within 60 n sweeps, or if the input or the result is not finite (w
// and Q then hold the unconverged iterate).
bool sym_eig(int n, const double* A, double* w, double* Q);

// General real A (n x n row-major) -> eigenvalues wr + i wi and eigenvectors
// (column i of Vr + i Vi, unit 2-norm).  Complex eigenvalues come as exact
// conjugate pairs.  Returns false if the QR iteration did not converge or
// an eigenvalue is not finite.
bool general_eig(int n, const double* A, double* wr, double* wi, double* Vr, double* Vi);

// Upper Hessenberg form H = Q^T A Q of a general A (both n x n row-major),
// handed from the first half of general_eig to the second.
struct HessForm {
  int n = 0;
  std::vector<double> H, Q;
};

// The two halves of general_eig: eigenvalues (exact conjugate pairs), then
// eigenvectors only for the indices with want[i] != 0 (want NULL: all; the
// other columns are zero).  With hf, general_eigvals leaves the Hessenberg
// form there and general_eigvecs starts from it; without, general_eigvecs
// reduces A again.
bool general_eigvals(int n, const double* A, double* wr, double* wi, HessForm* hf = nullptr);
void general_eigvecs(int n, const double* A, const double* wr, const double* wi,
                     const char* want, double* Vr, double* Vi, const HessForm* hf = nullptr);

}  // namespace expmv
