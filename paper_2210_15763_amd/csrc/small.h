// Workgroup-cooperative small dense FP64 routines shared by several kernels.
#pragma once

#include "common.h"

namespace bbl {

// Cyclic Jacobi on a symmetric n x n matrix held in LDS (row-major).  On exit
// lam[0..n) ascending and V's columns the matching orthonormal eigenvectors.
__device__ inline void wg_jacobi_eig(double *A, double *V, double *lam, int n, double *cs) {
  const int t = threadIdx.x;
  for (int i = t; i < n * n; i += blockDim.x) V[i] = (i / n == i % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) {
      double off = 0.0, dia = 0.0;
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
          if (p == q) dia += A[p * n + p] * A[p * n + p];
          else off += A[p * n + q] * A[p * n + q];
        }
      cs[2] = (off <= 1e-32 * dia || off < 1e-300) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (cs[2] != 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        if (t == 0) {
          const double apq = A[p * n + q];
          double c = 1.0, s = 0.0;
          if (fabs(apq) > 1e-300 &&
              fabs(apq) > 1e-18 * sqrt(fabs(A[p * n + p] * A[q * n + q]))) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          if (t < n) {  // columns p, q of A and V
            const double aip = A[t * n + p], aiq = A[t * n + q];
            A[t * n + p] = c * aip - s * aiq;
            A[t * n + q] = s * aip + c * aiq;
            const double vip = V[t * n + p], viq = V[t * n + q];
            V[t * n + p] = c * vip - s * viq;
            V[t * n + q] = s * vip + c * viq;
          }
          __syncthreads();
          if (t < n) {  // rows p, q of A
            const double api = A[p * n + t], aqi = A[q * n + t];
            A[p * n + t] = c * api - s * aqi;
            A[q * n + t] = s * api + c * aqi;
          }
        }
        __syncthreads();
      }
    }
  }
  // sort ascending (selection sort, one thread), permuting V's columns
  if (t == 0) {
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
    for (int i = 0; i < n; ++i) {
      int m = i;
      for (int j = i + 1; j < n; ++j)
        if (lam[j] < lam[m]) m = j;
      if (m != i) {
        const double tl = lam[i];
        lam[i] = lam[m];
        lam[m] = tl;
        for (int r = 0; r < n; ++r) {
          const double tv = V[r * n + i];
          V[r * n + i] = V[r * n + m];
          V[r * n + m] = tv;
        }
      }
    }
  }
  __syncthreads();
}

// Householder QR of an n x n matrix in LDS: A <- R (upper triangular), Q with
// Q R = A_in.
__device__ inline void wg_householder_qr(double *A, double *Q, int n, double *v, double *sc) {
  const int t = threadIdx.x;
  for (int i = t; i < n * n; i += blockDim.x) Q[i] = (i / n == i % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = 0; j < n - 1; ++j) {
    if (t == 0) {
      double nrm2 = 0.0;
      for (int i = j; i < n; ++i) nrm2 += A[i * n + j] * A[i * n + j];
      const double x0 = A[j * n + j];
      const double alpha = (x0 >= 0.0 ? -1.0 : 1.0) * sqrt(nrm2);
      for (int i = 0; i < n; ++i) v[i] = (i < j) ? 0.0 : A[i * n + j];
      v[j] = x0 - alpha;
      double vn2 = 0.0;
      for (int i = j; i < n; ++i) vn2 += v[i] * v[i];
      sc[0] = (vn2 > 1e-300 && nrm2 > 0.0) ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double f = sc[0];
    if (f != 0.0) {
      if (t < n) {  // column t of A: A[:, t] -= f v (v^T A[:, t])
        double d = 0.0;
        for (int i = j; i < n; ++i) d += v[i] * A[i * n + t];
        for (int i = j; i < n; ++i) A[i * n + t] -= f * d * v[i];
      }
      __syncthreads();
      if (t < n) {  // row t of Q: Q[t, :] -= f (Q[t, :] v) v^T
        double d = 0.0;
        for (int i = j; i < n; ++i) d += Q[t * n + i] * v[i];
        for (int i = j; i < n; ++i) Q[t * n + i] -= f * d * v[i];
      }
    }
    __syncthreads();
  }
  // exact zeros below the diagonal
  for (int i = t; i < n * n; i += blockDim.x)
    if (i / n > i % n) A[i] = 0.0;
  __syncthreads();
}


// launchers of small.hip
void launch_svqb_prepare(const double *O, int b, double tau, const double *hnorm_ptr,
                         const double *hn2_ptr, double *C0, double *QB, double *RB, int *mask,
                         int *flag, int *ndefl_total, const int *when, hipStream_t s);
void launch_chol_try(const double *O, int b, double tau, const double *hnorm_ptr,
                     const double *hn2_ptr, double *C0, double *QB, double *RB, int *mask,
                     int *flag, int *fail, hipStream_t s);
void launch_chol_finish(const double *O2, int b, const double *RB, double *Rinv, double *Bout,
                        int *breakdown, hipStream_t s);
void launch_set_A(const double *Araw, int b, int J, double *band, int kd, const double *Bprev,
                  double *C3, double *hn2, hipStream_t s);
void launch_set_B(const double *B, int b, int J, double *band, int kd, int nrows_max,
                  hipStream_t s);
// Thick restart: band rows 0..p+b-1, Bstore[0..p/b) and the rotation Q
// (p x p) of the kept Ritz vectors (theta, S[:, 0:p] with row stride ldS,
// last block rows from row0, B_last), then Sp = S[:, 0:p] Q by column blocks.
void launch_restart_reduce(const double *theta, const double *S, int ldS, int row0,
                           const double *Blast, int p, int b, double *band, double *Bstore,
                           double *Q, hipStream_t s);
void launch_restart_coeffs(const double *S, int ldS, int Nr, const double *Q, int p, int b,
                           double *Sp, hipStream_t s);
void launch_normalize_columns(int64_t n, int k, double *X, double *scratch, int max_partials,
                              hipStream_t s);
size_t normalize_scratch_bytes(int k, int max_partials);
void launch_reorth_check(const double *G0, const double *G1, int b, double eta2, const int *outer,
                         int *flag, int *counter, hipStream_t s);

}  // namespace bbl
