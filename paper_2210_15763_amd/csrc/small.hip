// Small dense FP64 kernels of the block recurrence (one workgroup each):
//  * spectral factorisation of the overlap O = W'^T W' = U Lambda U^T with
//    deflation of near-singular directions (Methods: B_n = Lambda^{1/2} U^T,
//    V_{n+1} = W' U Lambda^{-1/2}), followed by a Householder QR of the b x b
//    factor so the coupling block kept in the band matrix is upper triangular;
//  * the Cholesky polish of the second pass (CholQR) and the final B_n;
//  * assembly of A_n (symmetrised) and B_n into the band matrix;
//  * column norms / sign normalisation of Ritz vectors.
#include "common.h"
#include "small.h"

namespace bbl {

namespace {

// Overlap factorisation with deflation.  Writes, all row-major b x b:
//   C0   : matrix taking W' to the next block's pre-image (see below)
//   QB,RB: QR of the spectral factor Bsv = Lambda^{1/2} U^T (deflated rows 0)
//   mask : 1 for a deflated column (to be replaced by a random direction)
//   flag : 1 if any column was deflated
// Without deflation C0 = U Lambda^{-1/2} QB, so Y = W' C0 satisfies W' = Y RB.
// With deflation C0 = U_keep Lambda_keep^{-1/2} (zero deflated columns); the
// caller fills those columns randomly, orthogonalises them, and applies QB.
__global__ __launch_bounds__(256) void k_svqb_prepare(const double *__restrict__ O, int b,
                                                      double tau, const double *hnorm_ptr,
                                                      const double *hn2_ptr, double *C0,
                                                      double *QB, double *RB, int *mask,
                                                      int *flag, int *ndefl_total,
                                                      const int *when) {
  if (when && *when == 0) return;
  __shared__ double A[kMaxBlock * kMaxBlock], U[kMaxBlock * kMaxBlock];
  __shared__ double Bs[kMaxBlock * kMaxBlock], Q[kMaxBlock * kMaxBlock];
  __shared__ double lam[kMaxBlock], sig[kMaxBlock], v[kMaxBlock], sc[4];
  __shared__ int keep[kMaxBlock];
  const int t = threadIdx.x;
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    A[i] = 0.5 * (O[r * b + c] + O[c * b + r]);
  }
  __syncthreads();
  wg_jacobi_eig(A, U, lam, b, sc);
  if (t == 0) {
    double smax = 0.0;
    for (int i = 0; i < b; ++i) {
      sig[i] = sqrt(fmax(lam[i], 0.0));
      smax = fmax(smax, sig[i]);
    }
    const double hn = fmax(hnorm_ptr ? *hnorm_ptr : 0.0, hn2_ptr ? *hn2_ptr : 0.0);
    const double thr = tau * fmax(smax, hn);
    int nd = 0;
    for (int i = 0; i < b; ++i) {
      keep[i] = sig[i] > thr ? 1 : 0;
      nd += 1 - keep[i];
    }
    sc[3] = (double)nd;
  }
  __syncthreads();
  const int nd = (int)sc[3];
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    Bs[i] = keep[r] ? sig[r] * U[c * b + r] : 0.0;       // row r = sigma_r u_r^T
    A[i] = keep[c] ? U[r * b + c] / sig[c] : 0.0;        // column c = u_c / sigma_c
  }
  __syncthreads();
  wg_householder_qr(Bs, Q, b, v, sc);
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    double cv;
    if (nd == 0) {
      cv = 0.0;
      for (int m = 0; m < b; ++m) cv += A[r * b + m] * Q[m * b + c];
    } else {
      cv = A[i];
    }
    C0[i] = cv;
    QB[i] = Q[i];
    RB[i] = Bs[i];
  }
  if (t < b) mask[t] = keep[t] ? 0 : 1;
  if (t == 0) {
    *flag = nd > 0 ? 1 : 0;
    if (ndefl_total) *ndefl_total += nd;
  }
}

// Single-thread Cholesky O = R^T R (R upper, row-major) and R^{-1}.  Returns
// the smallest pivot (before the square root); a non-positive pivot is
// replaced by 1 so the factors stay finite.
__device__ double chol_upper(const double *O, int b, double *R, double *Ri) {
  double pmin = 1e308;
  for (int i = 0; i < b * b; ++i) R[i] = 0.0;
  for (int j = 0; j < b; ++j) {
    double s = O[j * b + j];
    for (int k = 0; k < j; ++k) s -= R[k * b + j] * R[k * b + j];
    pmin = fmin(pmin, s);
    if (!(s > 0.0)) s = 1.0;
    const double rjj = sqrt(s);
    R[j * b + j] = rjj;
    for (int c = j + 1; c < b; ++c) {
      double x = 0.5 * (O[j * b + c] + O[c * b + j]);
      for (int k = 0; k < j; ++k) x -= R[k * b + j] * R[k * b + c];
      R[j * b + c] = x / rjj;
    }
  }
  for (int i = 0; i < b * b; ++i) Ri[i] = 0.0;
  for (int c = 0; c < b; ++c) {
    Ri[c * b + c] = 1.0 / R[c * b + c];
    for (int r = c - 1; r >= 0; --r) {
      double x = 0.0;
      for (int m = r + 1; m <= c; ++m) x += R[r * b + m] * Ri[m * b + c];
      Ri[r * b + c] = -x / R[r * b + r];
    }
  }
  return pmin;
}

// The same factorisation in registers for a compile-time B (one thread):
// R[a][c] (a <= c) at trR(c, a), R^{-1} likewise.  thr: a pivot that is not
// above it is replaced by 1 and counted in nbad.  Returns the smallest pivot.
__host__ __device__ constexpr int trR(int c, int a) { return c * (c + 1) / 2 + a; }

template <int B>
__device__ __forceinline__ double chol_reg(const double *O, double thr, double (&R)[B * (B + 1) / 2],
                                           double (&Ri)[B * (B + 1) / 2], int &nbad) {
  double pmin = 1e308;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    double sj = O[j * B + j];
#pragma unroll
    for (int m = 0; m < j; ++m) sj = fma(-R[trR(j, m)], R[trR(j, m)], sj);
    pmin = fmin(pmin, sj);
    if (!(sj > thr)) {
      ++nbad;
      sj = 1.0;
    }
    const double rjj = sqrt(sj);
    R[trR(j, j)] = rjj;
#pragma unroll
    for (int c = j + 1; c < B; ++c) {
      double x = 0.5 * (O[j * B + c] + O[c * B + j]);
#pragma unroll
      for (int m = 0; m < j; ++m) x = fma(-R[trR(j, m)], R[trR(c, m)], x);
      R[trR(c, j)] = x / rjj;
    }
  }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    Ri[trR(c, c)] = 1.0 / R[trR(c, c)];
#pragma unroll
    for (int aa = 0; aa < c; ++aa) {
      const int r = c - 1 - aa;
      double x = 0.0;
#pragma unroll
      for (int m = r + 1; m <= c; ++m) x = fma(R[trR(m, r)], Ri[trR(c, m)], x);
      Ri[trR(c, r)] = -x / R[trR(r, r)];
    }
  }
  return pmin;
}

// Unpacks the register triangles into row-major LDS matrices (zero below).
template <int B>
__device__ __forceinline__ void unpack_upper(const double (&T)[B * (B + 1) / 2], double *M) {
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) M[r * B + c] = c >= r ? T[trR(c, r)] : 0.0;
}

// First factorisation of the overlap by Cholesky (CholQR).  Accepted when the
// overlap is safely positive definite: every pivot above 1e-14 * max O_ii
// (condition number of W' below ~1e7, where the Cholesky polish pass restores
// full orthogonality) and above (tau * max(||W'||, ||H||_est))^2 (no column
// is negligible -- the deflation test of the spectral factorisation).  On
// success C0 = R^{-1}, RB = R, QB = I, no deflation; otherwise fail = 1 and the
// spectral factorisation (k_svqb_prepare, gated by fail) takes over.
// BC > 0: compile-time block width (b == BC), factorised in registers.
template <int BC>
__global__ __launch_bounds__(64) void k_chol_try(const double *__restrict__ O, int b, double tau,
                                                 const double *hnorm_ptr, const double *hn2_ptr,
                                                 double *C0, double *QB, double *RB, int *mask,
                                                 int *flag, int *fail) {
  __shared__ double R[kMaxBlock * kMaxBlock], Ri[kMaxBlock * kMaxBlock], Os[kMaxBlock * kMaxBlock];
  __shared__ int ok;
  const int t = threadIdx.x;
  // the serial factorisation reads its input from LDS, not global memory
  for (int i = t; i < b * b; i += blockDim.x) Os[i] = O[i];
  __syncthreads();
  if (t == 0) {
    double dmax = 0.0;
    for (int i = 0; i < b; ++i) dmax = fmax(dmax, Os[i * b + i]);
    double pmin;
    if constexpr (BC > 0) {
      double Rr[BC * (BC + 1) / 2], Rir[BC * (BC + 1) / 2];
      int nbad = 0;
      pmin = chol_reg<BC>(Os, 0.0, Rr, Rir, nbad);
      unpack_upper<BC>(Rr, R);
      unpack_upper<BC>(Rir, Ri);
    } else {
      pmin = chol_upper(Os, b, R, Ri);
    }
    const double hn = fmax(hnorm_ptr ? *hnorm_ptr : 0.0, hn2_ptr ? *hn2_ptr : 0.0);
    const double scale = tau * fmax(sqrt(fmax(dmax, 0.0)), hn);
    ok = (dmax > 0.0 && pmin > 1e-14 * dmax && pmin > scale * scale) ? 1 : 0;
    *fail = 1 - ok;
    if (ok) *flag = 0;
  }
  __syncthreads();
  if (!ok) return;
  for (int i = t; i < b * b; i += blockDim.x) {
    C0[i] = Ri[i];
    RB[i] = R[i];
    QB[i] = (i / b == i % b) ? 1.0 : 0.0;
  }
  if (t < b) mask[t] = 0;
}

// Second pass: O2 = Y^T Y = R2^T R2.  Writes R2^{-1} (upper, row-major) and
// Bout = R2 RB (upper triangular).  breakdown is set to 1 (and never cleared)
// if O2 is not positive definite to working precision.
template <int BC>
__global__ __launch_bounds__(64) void k_chol_finish(const double *__restrict__ O2, int b,
                                                    const double *__restrict__ RB, double *Rinv,
                                                    double *Bout, int *breakdown) {
  __shared__ double R[kMaxBlock * kMaxBlock], Ri[kMaxBlock * kMaxBlock], Os[kMaxBlock * kMaxBlock];
  const int t = threadIdx.x;
  // the serial factorisation reads its input from LDS, not global memory
  for (int i = t; i < b * b; i += blockDim.x) Os[i] = O2[i];
  __syncthreads();
  const double *O2l = Os;
  if (BC > 0 && t == 0) {
    double dmax = 0.0;
    for (int i = 0; i < b; ++i) dmax = fmax(dmax, O2l[i * b + i]);
    double Rr[(BC > 0 ? BC : 1) * ((BC > 0 ? BC : 1) + 1) / 2];
    double Rir[(BC > 0 ? BC : 1) * ((BC > 0 ? BC : 1) + 1) / 2];
    int nbad = 0;
    if constexpr (BC > 0) {
      chol_reg<BC>(O2l, 1e-28 * dmax, Rr, Rir, nbad);
      unpack_upper<BC>(Rr, R);
      unpack_upper<BC>(Rir, Ri);
    }
    if (nbad || !(dmax > 0.0)) *breakdown = 1;  // sticky until the solve ends
  } else if (BC == 0 && t == 0) {
    int bad = 0;
    double dmax = 0.0;
    for (int i = 0; i < b; ++i) dmax = fmax(dmax, O2l[i * b + i]);
    for (int i = 0; i < b * b; ++i) R[i] = 0.0;
    for (int j = 0; j < b; ++j) {
      double s = 0.5 * (O2l[j * b + j] + O2l[j * b + j]);
      for (int k = 0; k < j; ++k) s -= R[k * b + j] * R[k * b + j];
      if (!(s > 1e-28 * dmax) || !(dmax > 0.0)) {
        bad = 1;
        s = 1.0;
      }
      const double rjj = sqrt(s);
      R[j * b + j] = rjj;
      for (int c = j + 1; c < b; ++c) {
        double x = 0.5 * (O2l[j * b + c] + O2l[c * b + j]);
        for (int k = 0; k < j; ++k) x -= R[k * b + j] * R[k * b + c];
        R[j * b + c] = x / rjj;
      }
    }
    // inverse of the upper-triangular R, column by column
    for (int i = 0; i < b * b; ++i) Ri[i] = 0.0;
    for (int c = 0; c < b; ++c) {
      Ri[c * b + c] = 1.0 / R[c * b + c];
      for (int r = c - 1; r >= 0; --r) {
        double x = 0.0;
        for (int m = r + 1; m <= c; ++m) x += R[r * b + m] * Ri[m * b + c];
        Ri[r * b + c] = -x / R[r * b + r];
      }
    }
    if (bad) *breakdown = 1;  // sticky until the solve ends
  }
  __syncthreads();
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    Rinv[i] = Ri[i];
    double x = 0.0;
    for (int m = r; m <= c; ++m) x += R[r * b + m] * RB[m * b + c];
    Bout[i] = (c >= r) ? x : 0.0;
  }
}

// A_J = (Araw + Araw^T)/2 into the band (rows J*b..), and the stacked
// three-term matrix C3 = [B_{J-1}^T ; A_J] (or just A_J when J == 0).
__global__ void k_set_A(const double *__restrict__ Araw, int b, int J, double *band, int kd,
                        const double *__restrict__ Bprev, double *C3, double *hn2) {
  const int t = threadIdx.x;
  if (t == 0 && hn2) {  // |A_ii| = |v_i^T H v_i| <= ||H||: a lower estimate of the norm
    double m = *hn2;
    for (int i = 0; i < b; ++i) m = fmax(m, fabs(Araw[i * b + i]));
    *hn2 = m;
  }
  const int off = (J > 0) ? b : 0;
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    const double a = 0.5 * (Araw[r * b + c] + Araw[c * b + r]);
    C3[(off + r) * b + c] = a;
    if (J > 0) C3[r * b + c] = Bprev[c * b + r];  // (B_{J-1}^T)[r][c]
    if (c <= r) band[((int64_t)J * b + r) * (kd + 1) + (r - c)] = a;
  }
}

// B_J (upper triangular) into the band: T[(J+1)b + r][J b + c] = B[r][c].
__global__ void k_set_B(const double *__restrict__ B, int b, int J, double *band, int kd,
                        int nrows_max) {
  const int t = threadIdx.x;
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    const int row = (J + 1) * b + r;
    const int d = b + r - c;
    if (row < nrows_max && d >= 1 && d <= kd) band[(int64_t)row * (kd + 1) + d] = B[i];
  }
}

// Column statistics of an n x k row-major block: per workgroup partial sum of
// squares and the first index of the largest |x|.
__global__ __launch_bounds__(256) void k_colstats(int64_t n, int k, const double *__restrict__ X,
                                                  double *sumsq, double *amax, int64_t *aidx) {
  __shared__ double s_sq[256];
  __shared__ double s_am[256];
  __shared__ int64_t s_ix[256];
  for (int c = 0; c < k; ++c) {
    double sq = 0.0, am = -1.0;
    int64_t ix = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double x = X[i * k + c];
      sq = fma(x, x, sq);
      if (fabs(x) > am) {
        am = fabs(x);
        ix = i;
      }
    }
    s_sq[threadIdx.x] = sq;
    s_am[threadIdx.x] = am;
    s_ix[threadIdx.x] = ix;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        s_sq[threadIdx.x] += s_sq[threadIdx.x + w];
        const double a2 = s_am[threadIdx.x + w];
        const int64_t i2 = s_ix[threadIdx.x + w];
        if (a2 > s_am[threadIdx.x] || (a2 == s_am[threadIdx.x] && i2 < s_ix[threadIdx.x])) {
          s_am[threadIdx.x] = a2;
          s_ix[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      sumsq[(int64_t)blockIdx.x * k + c] = s_sq[0];
      amax[(int64_t)blockIdx.x * k + c] = s_am[0];
      aidx[(int64_t)blockIdx.x * k + c] = s_ix[0];
    }
    __syncthreads();
  }
}

// factor[c] = sign(x[argmax|x|, c]) / ||x_c||.  One workgroup: per column,
// the threads stride over the P partials, then a fixed-order tree combines
// them (the largest |x| wins, ties to the lowest row index, as in k_colstats).
__global__ __launch_bounds__(256) void k_colfinish(int P, int k, const double *sumsq,
                                                   const double *amax, const int64_t *aidx,
                                                   const double *__restrict__ X, double *factor) {
  __shared__ double s_sq[256], s_am[256];
  __shared__ int64_t s_ix[256];
  for (int c = 0; c < k; ++c) {
    double sq = 0.0, am = -1.0;
    int64_t ix = 0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
      sq += sumsq[(int64_t)p * k + c];
      const double a2 = amax[(int64_t)p * k + c];
      const int64_t i2 = aidx[(int64_t)p * k + c];
      if (a2 > am || (a2 == am && i2 < ix)) {
        am = a2;
        ix = i2;
      }
    }
    s_sq[threadIdx.x] = sq;
    s_am[threadIdx.x] = am;
    s_ix[threadIdx.x] = ix;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        s_sq[threadIdx.x] += s_sq[threadIdx.x + w];
        const double a2 = s_am[threadIdx.x + w];
        const int64_t i2 = s_ix[threadIdx.x + w];
        if (a2 > s_am[threadIdx.x] || (a2 == s_am[threadIdx.x] && i2 < s_ix[threadIdx.x])) {
          s_am[threadIdx.x] = a2;
          s_ix[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double sgn = X[s_ix[0] * k + c] < 0.0 ? -1.0 : 1.0;
      factor[c] = s_sq[0] > 0.0 ? sgn / sqrt(s_sq[0]) : 1.0;
    }
    __syncthreads();
  }
}

__global__ void k_colscale(int64_t n, int k, double *X, const double *factor) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * k;
       i += (int64_t)gridDim.x * blockDim.x)
    X[i] *= factor[i % k];
}

// Second Gram-Schmidt pass needed?  flag = 1 if any column lost more than
// 1 - eta of its norm in the first pass (||w_after||^2 < eta^2 ||w_before||^2,
// the "twice is enough" test of Daniel, Gragg, Kaufman and Stewart), gated by
// an optional outer predicate.
__global__ void k_reorth_check(const double *G0, const double *G1, int b, double eta2,
                               const int *outer, int *flag, int *counter) {
  if (threadIdx.x != 0) return;
  int need = 0;
  for (int i = 0; i < b; ++i) need |= (G1[i * b + i] < eta2 * G0[i * b + i]) ? 1 : 0;
  if (outer && *outer == 0) need = 0;
  *flag = need;
  if (counter) *counter += need;
}


// Thick restart (Wu & Simon; the restarted method of the paper's introduction
// and base-Lanczos subsection).  The lowest p Ritz vectors Y = V S_p of a
// cycle and the next Lanczos block V_m span a space on which H acts as the
// arrowhead matrix [[Theta, Sigma^T], [Sigma, A]] with Theta = diag(theta),
// Sigma = B_last S_p[last block rows] (b x p).  This kernel rotates Y only,
// Y' = Y Q, so that the matrix becomes a band matrix of bandwidth b again:
// Householder reflectors applied from both sides reduce it column by column
// with the index order reversed (V_m first, so the reflectors never touch
// it).  Outputs: band rows 0..p+b-1 of the new cycle (row-major
// band[i*(b+1)+d] = T[i][i-d]; the V_m diagonal block is left to the next
// A), the b x b blocks B_j = T[(j+1)b.., jb..] (upper triangular) into
// Bstore[0..p/b), and Q (p x p, row-major).  One workgroup; p + b <= 64.
__global__ __launch_bounds__(256) void k_restart_reduce(const double *__restrict__ theta,
                                                        const double *__restrict__ S, int ldS,
                                                        int row0, const double *__restrict__ Blast,
                                                        int p, int b, double *band,
                                                        double *Bstore, double *Qout) {
  constexpr int NM = 2 * kMaxBlock;
  // G: the accumulated reflectors on the kept-vector indices b..N-1 (they
  // are the identity on the first b), G[(a-b)*p + (c-b)]
  __shared__ double M[NM * NM], G[kMaxBlock * kMaxBlock], v[NM], w[NM], pv[NM], sc[4];
  const int t = threadIdx.x;
  const int N = p + b;
  // M in reversed order: index a <-> forward index N-1-a (V_m first)
  for (int i = t; i < N * N; i += blockDim.x) {
    const int a = i / N, c = i % N;
    const int fi = N - 1 - a, fj = N - 1 - c;
    double x = 0.0;
    if (fi < p && fj < p) {
      x = (fi == fj) ? theta[fi] : 0.0;
    } else if (fi >= p && fj < p) {  // Sigma[fi - p][fj]
      for (int q = 0; q < b; ++q) x += Blast[(fi - p) * b + q] * S[(size_t)(row0 + q) * ldS + fj];
    } else if (fi < p && fj >= p) {
      for (int q = 0; q < b; ++q) x += Blast[(fj - p) * b + q] * S[(size_t)(row0 + q) * ldS + fi];
    }
    M[i] = x;
  }
  for (int i = t; i < p * p; i += blockDim.x) G[i] = (i / p == i % p) ? 1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c + b + 1 < N; ++c) {
    const int r0 = c + b;  // the reflector acts on indices r0..N-1
    __syncthreads();       // every lane has read the previous step's sc
    if (t == 0) {
      double tail = 0.0;
      for (int i = r0 + 1; i < N; ++i) tail += M[i * N + c] * M[i * N + c];
      const double x0 = M[r0 * N + c];
      if (tail == 0.0) {
        sc[0] = 0.0;
      } else {
        const double nrm = sqrt(x0 * x0 + tail);
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        sc[0] = 2.0 / (v0 * v0 + tail);
        sc[1] = v0;
      }
    }
    __syncthreads();
    const double tau = sc[0];
    if (tau == 0.0) continue;  // uniform: sc is shared
    for (int i = t; i < N; i += blockDim.x)
      v[i] = (i < r0) ? 0.0 : (i == r0 ? sc[1] : M[i * N + c]);
    __syncthreads();
    for (int i = t; i < N; i += blockDim.x) {  // p = tau M v, (G v)
      double x = 0.0, y = 0.0;
      for (int j = r0; j < N; ++j) {
        x += M[i * N + j] * v[j];
        if (i >= b) y += G[(i - b) * p + (j - b)] * v[j];
      }
      pv[i] = tau * x;
      w[i] = y;
    }
    __syncthreads();
    if (t == 0) {
      double vp = 0.0;
      for (int j = r0; j < N; ++j) vp += v[j] * pv[j];
      sc[2] = 0.5 * tau * vp;
    }
    __syncthreads();
    const double K = sc[2];
    for (int i = t; i < N * N; i += blockDim.x) {  // M -= v q^T + q v^T
      const int a = i / N, e = i % N;
      const double qa = pv[a] - K * v[a], qe = pv[e] - K * v[e];
      M[i] -= v[a] * qe + qa * v[e];
    }
    for (int i = t; i < p * p; i += blockDim.x) {  // G -= tau (G v) v^T
      const int a = i / p + b, e = i % p + b;
      G[i] -= tau * w[a] * v[e];
    }
    __syncthreads();
  }
  // forward order: T[i][j] = M[N-1-i][N-1-j], Q[l][i] = G[N-1-l][N-1-i]
  for (int i = t; i < N * (b + 1); i += blockDim.x) {
    const int r = i / (b + 1), d = i % (b + 1);
    if (r - d >= 0) band[(size_t)r * (b + 1) + d] = M[(N - 1 - r) * N + (N - 1 - (r - d))];
  }
  const int q = p / b;
  for (int i = t; i < q * b * b; i += blockDim.x) {
    const int j = i / (b * b), r = (i / b) % b, c = i % b;
    const int fi = (j + 1) * b + r, fj = j * b + c;
    Bstore[i] = (c >= r) ? M[(N - 1 - fi) * N + (N - 1 - fj)] : 0.0;
  }
  for (int i = t; i < p * p; i += blockDim.x) {  // reversed index N-1-l = b + (p-1-l)
    const int l = i / p, c = i % p;
    Qout[i] = G[(p - 1 - l) * p + (p - 1 - c)];
  }
}

// Sp = S[:, 0:p] Q as p / b column blocks of Nr x b (block j at Sp + j*Nr*b),
// the coefficients of the rotated kept Ritz vectors in the cycle's basis.
__global__ void k_restart_coeffs(const double *__restrict__ S, int ldS, int Nr,
                                 const double *__restrict__ Q, int p, int b, double *Sp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Nr * p) return;
  const int r = (int)(i / p), c = (int)(i % p);
  double x = 0.0;
  for (int l = 0; l < p; ++l) x += S[(size_t)r * ldS + l] * Q[l * p + c];
  Sp[(size_t)(c / b) * Nr * b + (size_t)r * b + (c % b)] = x;
}

}  // namespace

void launch_reorth_check(const double *G0, const double *G1, int b, double eta2, const int *outer,
                         int *flag, int *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_reorth_check, dim3(1), dim3(64), 0, s, G0, G1, b, eta2, outer, flag,
                     counter);
  check_launch("k_reorth_check");
}

void launch_svqb_prepare(const double *O, int b, double tau, const double *hnorm_ptr,
                         const double *hn2_ptr, double *C0, double *QB, double *RB, int *mask,
                         int *flag, int *ndefl_total, const int *when, hipStream_t s) {
  hipLaunchKernelGGL(k_svqb_prepare, dim3(1), dim3(256), 0, s, O, b, tau, hnorm_ptr, hn2_ptr, C0,
                     QB, RB, mask, flag, ndefl_total, when);
  check_launch("k_svqb_prepare");
}

void launch_chol_try(const double *O, int b, double tau, const double *hnorm_ptr,
                     const double *hn2_ptr, double *C0, double *QB, double *RB, int *mask,
                     int *flag, int *fail, hipStream_t s) {
  if (b == 8)
    hipLaunchKernelGGL(k_chol_try<8>, dim3(1), dim3(64), 0, s, O, b, tau, hnorm_ptr, hn2_ptr, C0,
                       QB, RB, mask, flag, fail);
  else if (b == 10)
    hipLaunchKernelGGL(k_chol_try<10>, dim3(1), dim3(64), 0, s, O, b, tau, hnorm_ptr, hn2_ptr, C0,
                       QB, RB, mask, flag, fail);
  else
    hipLaunchKernelGGL(k_chol_try<0>, dim3(1), dim3(64), 0, s, O, b, tau, hnorm_ptr, hn2_ptr, C0,
                       QB, RB, mask, flag, fail);
  check_launch("k_chol_try");
}

void launch_chol_finish(const double *O2, int b, const double *RB, double *Rinv, double *Bout,
                        int *breakdown, hipStream_t s) {
  if (b == 8)
    hipLaunchKernelGGL(k_chol_finish<8>, dim3(1), dim3(64), 0, s, O2, b, RB, Rinv, Bout,
                       breakdown);
  else if (b == 10)
    hipLaunchKernelGGL(k_chol_finish<10>, dim3(1), dim3(64), 0, s, O2, b, RB, Rinv, Bout,
                       breakdown);
  else
    hipLaunchKernelGGL(k_chol_finish<0>, dim3(1), dim3(64), 0, s, O2, b, RB, Rinv, Bout,
                       breakdown);
  check_launch("k_chol_finish");
}

void launch_set_A(const double *Araw, int b, int J, double *band, int kd, const double *Bprev,
                  double *C3, double *hn2, hipStream_t s) {
  hipLaunchKernelGGL(k_set_A, dim3(1), dim3(256), 0, s, Araw, b, J, band, kd, Bprev, C3, hn2);
  check_launch("k_set_A");
}

void launch_set_B(const double *B, int b, int J, double *band, int kd, int nrows_max,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_set_B, dim3(1), dim3(256), 0, s, B, b, J, band, kd, nrows_max);
  check_launch("k_set_B");
}

void launch_restart_reduce(const double *theta, const double *S, int ldS, int row0,
                           const double *Blast, int p, int b, double *band, double *Bstore,
                           double *Q, hipStream_t s) {
  hipLaunchKernelGGL(k_restart_reduce, dim3(1), dim3(256), 0, s, theta, S, ldS, row0, Blast, p, b,
                     band, Bstore, Q);
  check_launch("k_restart_reduce");
}

void launch_restart_coeffs(const double *S, int ldS, int Nr, const double *Q, int p, int b,
                           double *Sp, hipStream_t s) {
  const int64_t tot = (int64_t)Nr * p;
  hipLaunchKernelGGL(k_restart_coeffs, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, S, ldS,
                     Nr, Q, p, b, Sp);
  check_launch("k_restart_coeffs");
}

void launch_normalize_columns(int64_t n, int k, double *X, double *scratch, int max_partials,
                              hipStream_t s) {
  const int P = (int)std::max<int64_t>(1, std::min<int64_t>(max_partials, ceil_div(n, 256)));
  double *sumsq = scratch;
  double *amax = sumsq + (size_t)P * k;
  int64_t *aidx = reinterpret_cast<int64_t *>(amax + (size_t)P * k);
  double *factor = reinterpret_cast<double *>(aidx + (size_t)P * k);
  hipLaunchKernelGGL(k_colstats, dim3(P), dim3(256), 0, s, n, k, X, sumsq, amax, aidx);
  check_launch("k_colstats");
  hipLaunchKernelGGL(k_colfinish, dim3(1), dim3(256), 0, s, P, k, sumsq, amax, aidx, X, factor);
  check_launch("k_colfinish");
  const int64_t grid = std::min<int64_t>(4096, ceil_div(n * k, 256));
  hipLaunchKernelGGL(k_colscale, dim3((unsigned)grid), dim3(256), 0, s, n, k, X, factor);
  check_launch("k_colscale");
}

size_t normalize_scratch_bytes(int k, int max_partials) {
  return (size_t)max_partials * k * (8 + 8 + 8) + (size_t)k * 8 + 256;
}

}  // namespace bbl
