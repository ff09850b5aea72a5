// Pivot-block kernels: the leading principal block H[0:n_t, 0:n_t] as its own
// CSR matrix (the truncated space whose eigenvectors bootstrap the pivot,
// Methods last paragraphs).  Column indices are ascending within a row, so
// the entries with col < n_t are a prefix of each row: a binary search gives
// its length, a scan gives the new row pointers, and the prefixes are copied.
#include <algorithm>

#include "common.h"
#include "pivot.h"
#include "small.h"

namespace bbl {
namespace {

__global__ void k_slice_count(int64_t n_t, const int64_t *__restrict__ rp,
                              const int32_t *__restrict__ col, int64_t *__restrict__ rp_t) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_t;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = rp[i], hi = rp[i + 1];  // first position with col >= n_t
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)col[mid] < n_t) lo = mid + 1;
      else hi = mid;
    }
    rp_t[i + 1] = lo - rp[i];
    if (i == 0) rp_t[0] = 0;
  }
}

// In-place inclusive scan of a[1..m] by one 1024-thread workgroup.
__global__ __launch_bounds__(1024) void k_scan_inplace(int64_t *a, int64_t m) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (m + 1023) / 1024;
  const int64_t b0 = 1 + t * per, b1 = min(m + 1, b0 + per);
  int64_t s = 0;
  for (int64_t i = b0; i < b1; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = (t > 0) ? part[t - 1] : 0;
  for (int64_t i = b0; i < b1; ++i) {
    run += a[i];
    a[i] = run;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_slice_fill(int64_t n_t, const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col,
                                                    const VT *__restrict__ val,
                                                    const int64_t *__restrict__ rp_t,
                                                    int32_t *__restrict__ col_t,
                                                    VT *__restrict__ val_t) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; i < n_t;
       i += (int64_t)gridDim.x * blockDim.x / 64) {
    const int64_t src = rp[i], dst = rp_t[i], len = rp_t[i + 1] - rp_t[i];
    for (int64_t p = lane; p < len; p += 64) {
      col_t[dst + p] = col[src + p];
      val_t[dst + p] = val[src + p];
    }
  }
}

// Overlap of k unit vectors X with span(P): K = M G^+ M^T, M = X^T P (k x b),
// G = P^T P (b x b) and G^+ its pseudo-inverse (eigenvalues at or below
// 1e-12 of the largest dropped).  K's eigenvalues are the squared cosines of
// the principal angles between span(X) and span(P); its diagonal is the
// weight of each x_i inside span(P).  out[0..k): cosines, descending;
// out[k..2k): the weights.  One workgroup.
__global__ __launch_bounds__(256) void k_overlap(const double *__restrict__ M,
                                                 const double *__restrict__ G, int k, int b,
                                                 double *out) {
  __shared__ double A[kMaxBlock * kMaxBlock], U[kMaxBlock * kMaxBlock], lam[kMaxBlock];
  __shared__ double Gp[kMaxBlock * kMaxBlock], K[kMaxBlock * kMaxBlock], cs[4];
  const int t = threadIdx.x;
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    A[i] = 0.5 * (G[r * b + c] + G[c * b + r]);
  }
  __syncthreads();
  wg_jacobi_eig(A, U, lam, b, cs);
  const double lmax = lam[b - 1];
  for (int i = t; i < b * b; i += blockDim.x) {  // G^+ = U diag(1/lam) U^T
    const int r = i / b, c = i % b;
    double x = 0.0;
    for (int q = 0; q < b; ++q)
      if (lam[q] > 1e-12 * lmax && lam[q] > 0.0) x += U[r * b + q] * U[c * b + q] / lam[q];
    Gp[i] = x;
  }
  __syncthreads();
  for (int i = t; i < k * k; i += blockDim.x) {  // K = M G^+ M^T
    const int r = i / k, c = i % k;
    double x = 0.0;
    for (int p = 0; p < b; ++p) {
      double y = 0.0;
      for (int q = 0; q < b; ++q) y += Gp[p * b + q] * M[c * b + q];
      x += M[r * b + p] * y;
    }
    K[i] = x;
  }
  __syncthreads();
  if (t < k) out[k + t] = K[t * k + t];
  for (int i = t; i < k * k; i += blockDim.x) A[i] = 0.5 * (K[i] + K[(i % k) * k + i / k]);
  __syncthreads();
  wg_jacobi_eig(A, U, lam, k, cs);
  if (t < k) out[t] = sqrt(fmax(lam[k - 1 - t], 0.0));
}

}  // namespace

void launch_overlap(const double *M, const double *G, int k, int b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_overlap, dim3(1), dim3(256), 0, s, M, G, k, b, out);
  check_launch("k_overlap");
}

void launch_slice_leading(const bbl_csr &H, int64_t n_t, int64_t *rp_t, int32_t *col_t,
                          void *val_t, hipStream_t s) {
  const int64_t g = std::min<int64_t>(4096, ceil_div(n_t, 256));
  hipLaunchKernelGGL(k_slice_count, dim3((unsigned)g), dim3(256), 0, s, n_t, H.row_ptr, H.col,
                     rp_t);
  check_launch("k_slice_count");
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, rp_t, n_t);
  check_launch("k_scan_inplace");
  const int64_t g2 = std::min<int64_t>(8192, ceil_div(n_t * 64, 256));
  if (H.val_dtype == BBL_F32)
    hipLaunchKernelGGL(k_slice_fill<float>, dim3((unsigned)g2), dim3(256), 0, s, n_t, H.row_ptr,
                       H.col, (const float *)H.val, rp_t, col_t, (float *)val_t);
  else
    hipLaunchKernelGGL(k_slice_fill<double>, dim3((unsigned)g2), dim3(256), 0, s, n_t,
                       H.row_ptr, H.col, (const double *)H.val, rp_t, col_t, (double *)val_t);
  check_launch("k_slice_fill");
}

}  // namespace bbl
