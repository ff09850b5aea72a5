// Band-matrix eigensolver of the block recurrence (see bandeig.hip).
#pragma once

#include "common.h"

namespace bbl {

struct BandEigLayout {
  size_t gersh, shifts_a, shifts_b, counts, brk, Lscr, Dscr, X, TX, flag, bytes;
};

// Workspace layout for N x N band matrices of half-bandwidth kd, k pairs.
BandEigLayout band_eig_layout(int N, int kd, int k);

// Lowest k eigenpairs of the band matrix (band[i*(kd+1)+d] = T[i][i-d]).
//   S   device N x k eigenvectors (row-major)
//   res device: res[0..k) eigenvalues ascending, res[k..2k) residual
//       estimates ||Bj S[N-b:N, c]|| (0 if Bj == nullptr), res[2k] = max(|theta_0|, |lambda_max|),
//       res[2k+1] = lambda_max
void band_eigensolve(const double *band, int N, int kd, int k, void *ws, const BandEigLayout &L,
                     const double *Bj, int b, double *S, double *res, hipStream_t s);

}  // namespace bbl
