// Lowest eigenpairs of the block-tridiagonal band matrix T_j built from the
// A's and B's (Methods, block Lanczos: the paper hands this small band matrix
// to standard dense LAPACK eigensolvers).  On the GPU it is solved by
//   1. Sturm-count multisection: the number of negative pivots of the band
//      LDL^T factorisation of (T - sigma I) equals the number of eigenvalues
//      below sigma (Sylvester's law of inertia); many shifts are counted at
//      once, one lane per shift with the factorisation window in registers
//      (bandwidths 1, 2, 4, 8, 10) or one 64-lane workgroup per shift;
//   2. inverse iteration on each wanted eigenvalue with the same band LDL^T;
//   3. a Rayleigh-Ritz step on the span of the inverse-iteration vectors, which
//      orthonormalises them and refines the Ritz values.
// Only the k lowest eigenpairs (and the largest eigenvalue, for ||H||_est) are
// computed, in FP64.  Band storage: band[i*(kd+1) + d] = T[i][i-d], d = 0..kd.
#include "bandeig.h"
#include "common.h"
#include "small.h"

namespace bbl {
namespace {

constexpr int kChunk = 64;               // band rows staged in LDS at a time
constexpr int kMaxW = kMaxBlock + 1;     // window width (kd + 1)
constexpr int kMaxPairs = kMaxBlock * (kMaxBlock + 1) / 2;
constexpr int kMaxPPT = (kMaxPairs + 63) / 64;   // pairs per thread

// One band LDL^T sweep of (T - sigma I) by a 64-lane workgroup.  The active
// trailing window (rows/cols k..k+kd) lives in LDS with circular slots
// (absolute index i -> slot i % W).  Returns the number of negative pivots.
// With store = true, the unit-lower multipliers L[k][r-1] = l_{k+r,k} and the
// pivots D[k] are written out.
__device__ int ldl_sweep(const double *__restrict__ Tb, int N, int kd, double sigma,
                         double pivmin, bool store, double *win, double *chunk, double *L,
                         double *D) {
  const int W = kd + 1;
  const int NP = kd * (kd + 1) / 2;
  const int t = threadIdx.x;
  // this thread's (r, c) pairs, 1 <= c <= r <= kd, and their current slots
  int pr[kMaxPPT], rs[kMaxPPT], cs[kMaxPPT];
#pragma unroll
  for (int q = 0; q < kMaxPPT; ++q) {
    const int e = t + 64 * q;
    int r = 1, base = 0;
    while (e < NP && base + r <= e) {
      base += r;
      ++r;
    }
    const int c = (e < NP) ? e - base + 1 : 1;
    pr[q] = (e < NP) ? r : 1 << 20;  // out-of-range pairs never update
    rs[q] = r % W;
    cs[q] = c % W;
  }
  // rows 0..W-1 of the band into the window; then stream chunks
  for (int i = t; i < min(kChunk, N) * W; i += blockDim.x) chunk[i] = Tb[i];
  __syncthreads();
  for (int e = t; e < W * W; e += blockDim.x) {
    const int r = e / W, c = e % W;
    double v = 0.0;
    if (r < N && c <= r) {
      v = chunk[r * W + (r - c)];
      if (r == c) v -= sigma;
    }
    win[e] = v;
  }
  __syncthreads();
  int cnt = 0;
  int ks = 0;
  for (int k = 0; k < N; ++k) {
    double d = win[ks * W + ks];
    if (fabs(d) < pivmin) d = (store && d > 0.0) ? pivmin : -pivmin;
    cnt += (d < 0.0) ? 1 : 0;
    const double inv = 1.0 / d;
    if (store) {
      if (t == 0) D[k] = d;
      if (t < kd) {
        int sl = ks + 1 + t;
        if (sl >= W) sl -= W;
        L[(int64_t)k * kd + t] = (k + 1 + t < N) ? win[sl * W + ks] * inv : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < kMaxPPT; ++q) {
      if (k + pr[q] < N) {
        const double wr = win[rs[q] * W + ks] * inv;  // multiplier l_{r,k}
        const double lc = win[cs[q] * W + ks];
        win[rs[q] * W + cs[q]] = fma(-wr, lc, win[rs[q] * W + cs[q]]);
      }
      rs[q] = (rs[q] + 1 == W) ? 0 : rs[q] + 1;
      cs[q] = (cs[q] + 1 == W) ? 0 : cs[q] + 1;
    }
    __syncthreads();
    const int nr = k + W;  // row entering the window, into slot ks
    if (nr < N) {
      if (nr % kChunk == 0) {
        const int rows = min(kChunk, N - nr);
        for (int i = t; i < rows * W; i += blockDim.x) chunk[i] = Tb[(int64_t)nr * W + i];
        __syncthreads();
      }
      if (t < W) {
        double v = chunk[(nr % kChunk) * W + t];  // T[nr][nr - t]
        if (t == 0) v -= sigma;
        int sl = ks - t;  // slot of column nr - t  (nr = ks mod W)
        if (sl < 0) sl += W;
        win[ks * W + sl] = v;
      }
    }
    ks = (ks + 1 == W) ? 0 : ks + 1;
    __syncthreads();
  }
  return cnt;
}

__global__ __launch_bounds__(64) void k_sturm(const double *__restrict__ Tb, int N, int kd,
                                              const double *__restrict__ shifts,
                                              int *__restrict__ counts, double pivmin) {
  extern __shared__ double smem[];
  double *win = smem;
  double *chunk = smem + (kd + 1) * (kd + 1);
  const int c = ldl_sweep(Tb, N, kd, shifts[blockIdx.x], pivmin, false, win, chunk, nullptr,
                          nullptr);
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// Register-window band LDL^T for a compile-time bandwidth KD: one shift per
// lane.  The (KD+1) x (KD+1) trailing window of the partially factored
// T - sigma I is held as its lower triangle in registers, indexed by circular
// slots; the row loop is unrolled by KD + 1 so that every slot index is a
// compile-time constant.  Band rows are the same for all lanes (uniform
// loads).  Step k: pivot d = R[k][k], multipliers w_i = R[k+i][k] / d, update
// R[k+i][k+j] -= w_i R[k+j][k]; the same arithmetic as ldl_sweep.
constexpr int tri(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

// 1/d from the hardware reciprocal estimate and two Newton steps
// r <- r + r (1 - d r): full double precision for the LDL^T multipliers at a
// third of the dependent instructions of the IEEE division sequence, which
// sits on the critical path of every row.
__device__ __forceinline__ double newton_inv(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Steps M..KD of one unrolled group of W = KD + 1 rows, slot indices static.
// STORE: multipliers l_{k+i,k} to L[(k*KD + i-1) * ls] and 1/d to
// Dinv[k * ls] (a tiny pivot keeps its sign there); otherwise a tiny pivot
// counts as negative.  ls interleaves the factors of ls lanes.
// FULL: every row of the group and every row entering the window lies inside
// the matrix, so the group is straight-line code whose band loads can be
// issued ahead of the pivot's division; otherwise rows are checked and the
// entering row's loads are clamped to the last row (and zeroed after).
template <int KD, int M, bool STORE, bool FULL>
__device__ __forceinline__ void ldl_steps(const double *__restrict__ Tb, int N, int k0,
                                          double sigma, double pivmin,
                                          double (&R)[(KD + 1) * (KD + 2) / 2], int &cnt,
                                          double *__restrict__ L, double *__restrict__ Dinv,
                                          int ls) {
  if constexpr (M <= KD) {
    constexpr int W = KD + 1;
    const int k = k0 + M;
    if (FULL || k < N) {
      // row k + W enters in the slot freed by this step: T[k+W][k+W-t]
      const int nr = k + W;
      const bool nin = FULL || nr < N;
      const double *rowp = Tb + (int64_t)(FULL ? nr : min(nr, N - 1)) * W;
      double nv[W];
#pragma unroll
      for (int t = 0; t <= KD; ++t) nv[t] = rowp[t];
      // relative row i of the window lives in slot (M + i) % W
      double d = R[tri(M, M)];
      if (fabs(d) < pivmin) d = (STORE && d > 0.0) ? pivmin : -pivmin;
      cnt += d < 0.0 ? 1 : 0;
      const double inv = newton_inv(d);
      double w[KD + 1];
#pragma unroll
      for (int i = 1; i <= KD; ++i) w[i] = R[tri((M + i) % W, M)] * inv;
      if constexpr (STORE) {
        Dinv[(int64_t)k * ls] = inv;
#pragma unroll
        for (int i = 1; i <= KD; ++i)
          L[((int64_t)k * KD + i - 1) * ls] = (FULL || k + i < N) ? w[i] : 0.0;
      }
#pragma unroll
      for (int i = 1; i <= KD; ++i) {
        const int si = (M + i) % W;
#pragma unroll
        for (int j = 1; j <= i; ++j) {
          const int sj = (M + j) % W;
          R[tri(si, sj)] = fma(-w[i], R[tri(sj, M)], R[tri(si, sj)]);
        }
      }
#pragma unroll
      for (int t = 0; t <= KD; ++t) {
        const double v = t == 0 ? nv[0] - sigma : nv[t];
        R[tri(M, (M + W - t) % W)] = nin ? v : 0.0;
      }
      ldl_steps<KD, M + 1, STORE, FULL>(Tb, N, k0, sigma, pivmin, R, cnt, L, Dinv, ls);
    }
  }
}

// The whole band LDL^T sweep: full groups first, then the tail.
template <int KD, bool STORE>
__device__ __forceinline__ void ldl_sweep_reg(const double *__restrict__ Tb, int N, double sigma,
                                              double pivmin, double (&R)[(KD + 1) * (KD + 2) / 2],
                                              int &cnt, double *__restrict__ L,
                                              double *__restrict__ Dinv, int ls) {
  constexpr int W = KD + 1;
  int k0 = 0;
  // one group of W rows per trip; unrolling this loop further would only
  // multiply the code (the group is already W steps of straight-line code)
#pragma unroll 1
  for (; k0 + 2 * W <= N; k0 += W)
    ldl_steps<KD, 0, STORE, true>(Tb, N, k0, sigma, pivmin, R, cnt, L, Dinv, ls);
#pragma unroll 1
  for (; k0 < N; k0 += W)
    ldl_steps<KD, 0, STORE, false>(Tb, N, k0, sigma, pivmin, R, cnt, L, Dinv, ls);
}

// Window of rows 0..KD of T - sigma I.
template <int KD>
__device__ __forceinline__ void ldl_window_init(const double *__restrict__ Tb, int N, double sigma,
                                                double (&R)[(KD + 1) * (KD + 2) / 2]) {
  constexpr int W = KD + 1;
#pragma unroll
  for (int r = 0; r < W; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double v = 0.0;
      if (r < N) {
        v = Tb[(int64_t)r * W + (r - c)];
        if (r == c) v -= sigma;
      }
      R[tri(r, c)] = v;
    }
}

// Sturm counts, one shift per lane.
template <int KD>
__global__ __launch_bounds__(64) void k_sturm_reg(const double *__restrict__ Tb, int N,
                                                  const double *__restrict__ shifts, int nshift,
                                                  int *__restrict__ counts, double pivmin) {
  constexpr int W = KD + 1;
  const int id = blockIdx.x * 64 + threadIdx.x;
  const double sigma = id < nshift ? shifts[id] : 0.0;
  double R[W * (W + 1) / 2];
  ldl_window_init<KD>(Tb, N, sigma, R);
  int cnt = 0;
  ldl_sweep_reg<KD, false>(Tb, N, sigma, pivmin, R, cnt, nullptr, nullptr, 0);
  if (id < nshift) counts[id] = cnt;
}

void sturm_counts(const double *Tb, int N, int kd, const double *shifts, int nshift, int *counts,
                  double pivmin, size_t smem_generic, hipStream_t s) {
  const unsigned waves = (unsigned)((nshift + 63) / 64);
  switch (kd) {
    case 1: hipLaunchKernelGGL(k_sturm_reg<1>, dim3(waves), dim3(64), 0, s, Tb, N, shifts, nshift, counts, pivmin); break;
    case 2: hipLaunchKernelGGL(k_sturm_reg<2>, dim3(waves), dim3(64), 0, s, Tb, N, shifts, nshift, counts, pivmin); break;
    case 4: hipLaunchKernelGGL(k_sturm_reg<4>, dim3(waves), dim3(64), 0, s, Tb, N, shifts, nshift, counts, pivmin); break;
    case 8: hipLaunchKernelGGL(k_sturm_reg<8>, dim3(waves), dim3(64), 0, s, Tb, N, shifts, nshift, counts, pivmin); break;
    case 10: hipLaunchKernelGGL(k_sturm_reg<10>, dim3(waves), dim3(64), 0, s, Tb, N, shifts, nshift, counts, pivmin); break;
    default:
      hipLaunchKernelGGL(k_sturm, dim3(nshift), dim3(64), smem_generic, s, Tb, N, kd, shifts,
                         counts, pivmin);
  }
  check_launch("k_sturm");
}

// Gershgorin interval of T: out[0] = lower bound, out[1] = upper bound.
__global__ __launch_bounds__(256) void k_gersh(const double *__restrict__ Tb, int N, int kd,
                                               double *out) {
  __shared__ double slo[256], shi[256];
  const int W = kd + 1;
  double lo = 1e300, hi = -1e300;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double s = 0.0;
    for (int d = 1; d <= kd; ++d) {
      if (i - d >= 0) s += fabs(Tb[(int64_t)i * W + d]);
      if (i + d < N) s += fabs(Tb[(int64_t)(i + d) * W + d]);
    }
    const double a = Tb[(int64_t)i * W];
    lo = fmin(lo, a - s);
    hi = fmax(hi, a + s);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pad = 1e-12 * fmax(fabs(slo[0]), fabs(shi[0])) + 1e-300;
    out[0] = slo[0] - pad;
    out[1] = shi[0] + pad;
  }
}

// Round 1: shared shifts evenly spaced strictly inside [lo, hi].
__global__ void k_bisect_init(const double *gersh, int S, double *shifts, double *brk, int NT) {
  const double lo = gersh[0], hi = gersh[1];
  for (int s = threadIdx.x + blockIdx.x * blockDim.x; s < S; s += blockDim.x * gridDim.x)
    shifts[s] = lo + (hi - lo) * (double)(s + 1) / (double)(S + 1);
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < NT; t += blockDim.x) {
      brk[2 * t] = lo;
      brk[2 * t + 1] = hi;
    }
}

// Narrow one target's bracket (workgroup tg) from the counts of the last
// round, then lay out S_next shifts inside it.  Target t < k is eigenvalue
// index t; target k is index N - 1 (the largest).  count(sigma) = number of
// eigenvalues below sigma, so lambda_idx lies in
// [max{sigma: count <= idx}, min{sigma: count > idx}].  In the shared round
// every target scans all S_per shifts; afterwards target tg owns shifts
// [tg S_per, (tg + 1) S_per).
__global__ __launch_bounds__(256) void k_bisect_update(int shared_round, const double *shifts,
                                                       const int *counts, int S_per, int N,
                                                       int k, double *brk, int S_next,
                                                       double *next_shifts) {
  __shared__ double slo[256], shi[256];
  const int tg = blockIdx.x;
  const int idx = (tg < k) ? tg : N - 1;
  const int s0 = shared_round ? 0 : tg * S_per;
  double lo = brk[2 * tg], hi = brk[2 * tg + 1];
  for (int s = threadIdx.x; s < S_per; s += blockDim.x) {
    const double sg = shifts[s0 + s];
    const int c = counts[s0 + s];
    if (c <= idx) lo = fmax(lo, sg);
    else hi = fmin(hi, sg);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      slo[threadIdx.x] = fmax(slo[threadIdx.x], slo[threadIdx.x + w]);
      shi[threadIdx.x] = fmin(shi[threadIdx.x], shi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  double l = slo[0], h = shi[0];
  if (l > h) {  // rounding made the counts non-monotone: keep the crossing
    const double m = 0.5 * (l + h);
    l = m;
    h = m;
  }
  if (threadIdx.x == 0) {
    brk[2 * tg] = l;
    brk[2 * tg + 1] = h;
  }
  if (next_shifts)
    for (int s = threadIdx.x; s < S_next; s += blockDim.x)
      next_shifts[tg * S_next + s] = l + (h - l) * (double)(s + 1) / (double)(S_next + 1);
}

__device__ __forceinline__ double hash_unit(uint32_t x) {
  // integer hash (Wang-style mixing) to a value in (-1, 1)
  x = (x ^ 61u) ^ (x >> 16);
  x *= 9u;
  x = x ^ (x >> 4);
  x *= 0x27d4eb2du;
  x = x ^ (x >> 15);
  return ((double)x + 0.5) * (2.0 / 4294967296.0) - 1.0;
}

// Inverse iteration for target tg = blockIdx.x < k at the bracket midpoint.
__global__ __launch_bounds__(64) void k_invit(const double *__restrict__ Tb, int N, int kd,
                                              const double *__restrict__ brk, int k,
                                              double pivmin, double *Lscr, double *Dscr,
                                              double *X, int niter) {
  extern __shared__ double smem[];
  double *win = smem;
  double *chunk = win + (kd + 1) * (kd + 1);
  double *x = chunk + kChunk * (kd + 1);
  __shared__ double red[64];
  const int tg = blockIdx.x;
  const int t = threadIdx.x;
  const double theta = 0.5 * (brk[2 * tg] + brk[2 * tg + 1]);
  double *L = Lscr + (int64_t)tg * N * kd;
  double *D = Dscr + (int64_t)tg * N;
  ldl_sweep(Tb, N, kd, theta, pivmin, true, win, chunk, L, D);
  __threadfence();
  __syncthreads();
  for (int i = t; i < N; i += 64) x[i] = hash_unit((uint32_t)(i * 40503u + tg * 2654435761u + 7u));
  __syncthreads();
  for (int it = 0; it < niter; ++it) {
    // forward: unit lower L
    for (int kk = 0; kk < N; ++kk) {
      const double xk = x[kk];
      if (t < kd && kk + 1 + t < N) x[kk + 1 + t] -= L[(int64_t)kk * kd + t] * xk;
      __syncthreads();
    }
    for (int i = t; i < N; i += 64) x[i] /= D[i];
    __syncthreads();
    // backward: L^T
    for (int kk = N - 1; kk >= 0; --kk) {
      double p = (t < kd && kk + 1 + t < N) ? L[(int64_t)kk * kd + t] * x[kk + 1 + t] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off, 64);
      if (t == 0) x[kk] -= p;
      __syncthreads();
    }
    // normalise
    double s = 0.0;
    for (int i = t; i < N; i += 64) s += x[i] * x[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (t == 0) red[0] = s;
    __syncthreads();
    const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 1.0;
    for (int i = t; i < N; i += 64) x[i] *= inv;
    __syncthreads();
  }
  for (int i = t; i < N; i += 64) X[(int64_t)i * k + tg] = x[i];
}

// Forward substitution L y = x (L unit lower, bandwidth KD, multipliers
// L[j*KD + r-1] = l_{j+r,j}), right-looking: once y_j is final it is removed
// from x_{j+1..j+KD}.  q holds x_j..x_{j+KD-1} in circular slots; the slot of
// x_{j0+s} is s % KD for the group of KD rows starting at j0.  All loads of a
// group (its multipliers, inverse pivots and entering x values) are issued
// before its arithmetic, so that one memory latency is exposed per group
// rather than per row.  Stores z_j = y_j / d_j in place of x_j.
// FULL: rows j0 .. j0 + 2 KD - 1 all exist, so no clamping or selects.
template <int KD, bool FULL>
__device__ __forceinline__ void fwd_group(const double *__restrict__ L,
                                          const double *__restrict__ Dinv, int ls, double *X,
                                          int ldx, int N, int j0, double (&q)[KD]) {
  // loads clamped to the last row (and zeroed after) so that they carry no
  // branch and can all be issued at once
  double Lg[KD][KD], dv[KD], xn[KD];
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    const int j = j0 + m;
    const bool in = FULL || j < N, nin = FULL || j + KD < N;
    const int jc = FULL ? j : min(j, N - 1), jnc = FULL ? j + KD : min(j + KD, N - 1);
#pragma unroll
    for (int r = 0; r < KD; ++r) {
      const double v = L[((int64_t)jc * KD + r) * ls];
      Lg[m][r] = in ? v : 0.0;
    }
    const double dvv = Dinv[(int64_t)jc * ls];
    const double xv = X[(int64_t)jnc * ldx];
    dv[m] = in ? dvv : 0.0;
    xn[m] = nin ? xv : 0.0;
  }
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    const double y = q[m];
#pragma unroll
    for (int r = 1; r < KD; ++r) q[(m + r) % KD] = fma(-Lg[m][r - 1], y, q[(m + r) % KD]);
    q[m] = fma(-Lg[m][KD - 1], y, xn[m]);
    if (FULL || j0 + m < N) X[(int64_t)(j0 + m) * ldx] = y * dv[m];
  }
}

// Back substitution L^T x = z, rows i = i0, i0 - 1, ..., i0 - KD + 1:
// x_i = z_i - sum_r l_{i+r,i} x_{i+r}.  wv holds x_{i+1..i+KD}; the slot of
// x_m is (m - i0 - 1) mod KD.  Loads of the group first, as above.
// Accumulates ||x||^2 in row order.
// FULL: rows i0 - KD + 1 .. i0 all exist.
template <int KD, bool FULL>
__device__ __forceinline__ void bwd_group(const double *__restrict__ L, int ls, double *X,
                                          int ldx, int i0, double (&wv)[KD], double &nrm2) {
  double Lg[KD][KD], zg[KD];
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    const int i = i0 - m;
    const bool in = FULL || i >= 0;
    const int ic = FULL ? i : max(i, 0);
#pragma unroll
    for (int r = 0; r < KD; ++r) {
      const double v = L[((int64_t)ic * KD + r) * ls];
      Lg[m][r] = in ? v : 0.0;
    }
    const double zv = X[(int64_t)ic * ldx];
    zg[m] = in ? zv : 0.0;
  }
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    if (!FULL && i0 - m < 0) break;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int r = 1; r <= KD; ++r) {
      const double v = wv[((r - m - 1) % KD + KD) % KD];
      if (r & 1) a0 = fma(Lg[m][r - 1], v, a0);
      else a1 = fma(Lg[m][r - 1], v, a1);
    }
    const double xi = zg[m] - (a0 + a1);
    wv[KD - 1 - m] = xi;
    X[(int64_t)(i0 - m) * ldx] = xi;
    nrm2 = fma(xi, xi, nrm2);
  }
}

// Inverse iteration for a compile-time bandwidth at the bracket midpoint
// theta of target tg < k: factor T - theta I with the register window,
// keeping the multipliers and inverse pivots, then run niter solves
// L D L^T x <- x from a hashed start, normalising after each.  Column tg of
// X (row-major N x k) receives the vector.  Three placements:
//   MODE 0: one lane per target, factors in global scratch (interleaved over
//           the k lanes, so every load and store of the wave is contiguous),
//           vectors in X;
//   MODE 1: as 0 but the vectors in dynamic LDS (N k doubles), copied to X
//           at the end;
//   MODE 2: one workgroup per target (its first lane works): factors and
//           vector in dynamic LDS (N (KD + 2) doubles), so the solves never
//           wait on global memory, whose latency grows under the load of the
//           recurrence running beside a check.
template <int KD, int MODE>
__global__ __launch_bounds__(64) void k_invit_reg(const double *__restrict__ Tb, int N,
                                                  const double *__restrict__ brk, int k,
                                                  double pivmin, double *Lscr, double *Dscr,
                                                  double *X, int niter) {
  constexpr int W = KD + 1;
  extern __shared__ double smem_inv[];
  const int tg = MODE == 2 ? (int)blockIdx.x : (int)(blockIdx.x * 64 + threadIdx.x);
  if (tg >= k || (MODE == 2 && threadIdx.x != 0)) return;
  const double theta = 0.5 * (brk[2 * tg] + brk[2 * tg + 1]);
  // l_{j+r,j} at L[(j*KD + r-1) * ls], 1/d_j at Dinv[j * ls], x_j at x[j * lx]
  double *L, *Dinv, *x;
  int ls, lx;
  if constexpr (MODE == 2) {
    L = smem_inv;
    Dinv = smem_inv + (size_t)N * KD;
    x = Dinv + N;
    ls = 1;
    lx = 1;
  } else {
    L = Lscr + tg;
    Dinv = Dscr + tg;
    x = (MODE == 1 ? smem_inv : X) + tg;
    ls = k;
    lx = k;
  }
  double R[W * (W + 1) / 2];
  ldl_window_init<KD>(Tb, N, theta, R);
  int cnt = 0;
  ldl_sweep_reg<KD, true>(Tb, N, theta, pivmin, R, cnt, L, Dinv, ls);
  for (int i = 0; i < N; ++i)
    x[(int64_t)i * lx] = hash_unit((uint32_t)(i * 40503u + tg * 2654435761u + 7u));
  for (int it = 0; it < niter; ++it) {
    double q[KD];
#pragma unroll
    for (int r = 0; r < KD; ++r) q[r] = r < N ? x[(int64_t)r * lx] : 0.0;
    int j0 = 0;
#pragma unroll 1
    for (; j0 + 2 * KD <= N; j0 += KD) fwd_group<KD, true>(L, Dinv, ls, x, lx, N, j0, q);
#pragma unroll 1
    for (; j0 < N; j0 += KD) fwd_group<KD, false>(L, Dinv, ls, x, lx, N, j0, q);
    double wv[KD];
#pragma unroll
    for (int r = 0; r < KD; ++r) wv[r] = 0.0;
    double nrm2 = 0.0;
    int i0 = N - 1;
#pragma unroll 1
    for (; i0 - KD + 1 >= 0; i0 -= KD) bwd_group<KD, true>(L, ls, x, lx, i0, wv, nrm2);
#pragma unroll 1
    for (; i0 >= 0; i0 -= KD) bwd_group<KD, false>(L, ls, x, lx, i0, wv, nrm2);
    const double sc = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 1.0;
    for (int i = 0; i < N; ++i) x[(int64_t)i * lx] *= sc;
  }
  if (MODE != 0)
    for (int i = 0; i < N; ++i) X[(int64_t)i * k + tg] = x[(int64_t)i * lx];
}

__device__ double wg_sum(double v, double *red) {
  // sum over a 256-thread workgroup (fixed order)
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double band_at(const double *Tb, int kd, int i, int j) {
  const int d = i - j;
  if (d >= 0) return d <= kd ? Tb[(int64_t)i * (kd + 1) + d] : 0.0;
  return -d <= kd ? Tb[(int64_t)j * (kd + 1) - d] : 0.0;
}

// Rayleigh-Ritz on span(X): X <- orthonormal basis (modified Gram-Schmidt,
// twice), K = X^T T X, K = Y diag(theta) Y^T, S = X Y.  Residual estimates
// rho_c = ||Bj S[N-b:N, c]|| (Bj = coupling block to the next Lanczos block).
// res: theta[0..k), rho[k..2k), res[2k] = ||T||_est = max(|theta_0|, |top|),
// res[2k+1] = largest eigenvalue.
// when (optional): run only if *when != 0 (the fallback of k_rr_fast).
__global__ __launch_bounds__(256) void k_rr(const double *__restrict__ Tb, int N, int kd, int k,
                                            double *X, double *TX,
                                            const double *__restrict__ Bj, int b,
                                            const double *__restrict__ brk, double *S,
                                            double *res, const int *__restrict__ when) {
  if (when && *when == 0) return;
  __shared__ double K[kMaxBlock * kMaxBlock], Y[kMaxBlock * kMaxBlock];
  __shared__ double lam[kMaxBlock], cs[4], red[256];
  const int t = threadIdx.x;
  for (int c = 0; c < k; ++c) {
    for (int attempt = 0; attempt < 2; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int a = 0; a < c; ++a) {
          double p = 0.0;
          for (int i = t; i < N; i += blockDim.x) p += X[(int64_t)i * k + a] * X[(int64_t)i * k + c];
          const double dot = wg_sum(p, red);
          for (int i = t; i < N; i += blockDim.x) X[(int64_t)i * k + c] -= dot * X[(int64_t)i * k + a];
          __syncthreads();
        }
      }
      double p = 0.0;
      for (int i = t; i < N; i += blockDim.x) p += X[(int64_t)i * k + c] * X[(int64_t)i * k + c];
      const double nrm = sqrt(wg_sum(p, red));
      if (nrm > 1e-8) {
        for (int i = t; i < N; i += blockDim.x) X[(int64_t)i * k + c] /= nrm;
        __syncthreads();
        break;
      }
      // the vector collapsed onto earlier ones: restart it from a fresh direction
      for (int i = t; i < N; i += blockDim.x)
        X[(int64_t)i * k + c] = hash_unit((uint32_t)(i * 2246822519u + c * 3266489917u + 11u));
      __syncthreads();
    }
  }
  __threadfence();
  __syncthreads();
  for (int64_t e = t; e < (int64_t)N * k; e += blockDim.x) {
    const int i = (int)(e / k), c = (int)(e % k);
    double s = 0.0;
    const int j0 = max(0, i - kd), j1 = min(N - 1, i + kd);
    for (int j = j0; j <= j1; ++j) s += band_at(Tb, kd, i, j) * X[(int64_t)j * k + c];
    TX[e] = s;
  }
  __threadfence();
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int a = e / k, c = e % k;
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += X[(int64_t)i * k + a] * TX[(int64_t)i * k + c];
    K[e] = s;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int a = e / k, c = e % k;
    if (a < c) {
      const double m = 0.5 * (K[a * k + c] + K[c * k + a]);
      K[a * k + c] = m;
      K[c * k + a] = m;
    }
  }
  __syncthreads();
  wg_jacobi_eig(K, Y, lam, k, cs);
  for (int64_t e = t; e < (int64_t)N * k; e += blockDim.x) {
    const int i = (int)(e / k), c = (int)(e % k);
    double s = 0.0;
    for (int a = 0; a < k; ++a) s += X[(int64_t)i * k + a] * Y[a * k + c];
    S[e] = s;
  }
  __threadfence();
  __syncthreads();
  if (t < k) {
    double rho = 0.0;
    if (Bj) {
      for (int r = 0; r < b; ++r) {
        double v = 0.0;
        for (int m = 0; m < b; ++m) v += Bj[r * b + m] * S[(int64_t)(N - b + m) * k + t];
        rho += v * v;
      }
    }
    res[t] = lam[t];
    res[k + t] = sqrt(rho);
  }
  if (t == 0) {
    const double top = 0.5 * (brk[2 * k] + brk[2 * k + 1]);
    res[2 * k] = fmax(fabs(lam[0]), fabs(top));
    res[2 * k + 1] = top;
  }
}

// Wave-wide sum by an xor butterfly; both partners of every step add the
// same two operands, so all 64 lanes end with identical bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Rayleigh-Ritz on one wave for k <= KM (the same step as k_rr):
//   Q = X R^{-1}, twice: Cholesky QR of the inverse-iteration vectors, every
//       lane factoring the wave-summed k x k Gram matrix in registers;
//   K = Q^T T Q (upper triangle, mirrored), K = Y diag(theta) Y^T (Jacobi);
//   S = Q Y and the residual estimates rho_c = ||Bj S[N-b:N, c]||.
// X is left unchanged.  A Cholesky pivot below 1e-12 of its diagonal entry
// (columns nearly dependent) sets *fallback = 1 and ends the kernel, so that
// k_rr redoes the step with Gram-Schmidt and restarts; otherwise *fallback = 0.
// SQ: the final Q is kept in dynamic LDS (N k doubles) for the two passes
// that read it across rows; otherwise it stays in the global scratch Q.
template <int KM, bool SQ>
__global__ __launch_bounds__(64) void k_rr_fast(const double *__restrict__ Tb, int N, int kd,
                                                int k, const double *__restrict__ X, double *Q,
                                                const double *__restrict__ Bj, int b,
                                                const double *__restrict__ brk, double *S,
                                                double *res, int *fallback) {
  constexpr int NP = KM * (KM + 1) / 2;
  extern __shared__ double sQ[];
  __shared__ double K[KM * KM], Y[KM * KM];
  __shared__ double lam[KM], cs[4];
  const int t = threadIdx.x;
  double *Qout = Q;
  for (int pass = 0; pass < 2; ++pass) {
    const double *src = pass == 0 ? X : Q;
    if (SQ && pass == 1) Qout = sQ;
    double g[NP];  // G[a][c] (a <= c) at tri(c, a), then R in place
#pragma unroll
    for (int e = 0; e < NP; ++e) g[e] = 0.0;
    for (int i = t; i < N; i += 64) {
      double x[KM];
#pragma unroll
      for (int c = 0; c < KM; ++c) x[c] = c < k ? src[(int64_t)i * k + c] : 0.0;
#pragma unroll
      for (int c = 0; c < KM; ++c)
#pragma unroll
        for (int a = 0; a <= c; ++a) g[tri(c, a)] = fma(x[a], x[c], g[tri(c, a)]);
    }
#pragma unroll
    for (int e = 0; e < NP; ++e) g[e] = wave_sum(g[e]);
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j >= k) g[tri(j, j)] = 1.0;  // padding columns: R = I there
    bool bad = false;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      const double gjj = g[tri(j, j)];
      double sjj = gjj;
#pragma unroll
      for (int m = 0; m < j; ++m) sjj = fma(-g[tri(j, m)], g[tri(j, m)], sjj);
      if (!(sjj > 1e-12 * gjj)) {
        bad = true;
        sjj = 1.0;
      }
      const double rjj = sqrt(sjj);
      g[tri(j, j)] = rjj;
      const double rinv = 1.0 / rjj;
#pragma unroll
      for (int c = j + 1; c < KM; ++c) {
        double v = g[tri(c, j)];
#pragma unroll
        for (int m = 0; m < j; ++m) v = fma(-g[tri(j, m)], g[tri(c, m)], v);
        g[tri(c, j)] = v * rinv;
      }
    }
    if (bad) {
      if (t == 0) *fallback = 1;
      return;
    }
    // R^{-1} (upper), column by column from the diagonal up
    double ri[NP];
#pragma unroll
    for (int c = 0; c < KM; ++c) {
      ri[tri(c, c)] = 1.0 / g[tri(c, c)];
#pragma unroll
      for (int aa = 0; aa < c; ++aa) {
        const int a = c - 1 - aa;
        double v = 0.0;
#pragma unroll
        for (int m = a + 1; m <= c; ++m) v = fma(g[tri(m, a)], ri[tri(c, m)], v);
        ri[tri(c, a)] = -v * ri[tri(a, a)];  // ri[a][a] = 1 / R[a][a], set in column a
      }
    }
    for (int i = t; i < N; i += 64) {
      double x[KM];
#pragma unroll
      for (int c = 0; c < KM; ++c) x[c] = c < k ? src[(int64_t)i * k + c] : 0.0;
#pragma unroll
      for (int c = 0; c < KM; ++c) {
        double o = 0.0;
#pragma unroll
        for (int a = 0; a <= c; ++a) o = fma(x[a], ri[tri(c, a)], o);
        if (c < k) Qout[(int64_t)i * k + c] = o;
      }
    }
  }
  if (t == 0) *fallback = 0;
  __threadfence();
  __syncthreads();
  const double *Qr = SQ ? sQ : Q;
  // K = Q^T (T Q): each lane forms rows of T Q from the band and Q
  double kk[NP];
#pragma unroll
  for (int e = 0; e < NP; ++e) kk[e] = 0.0;
  for (int i = t; i < N; i += 64) {
    double tq[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) tq[c] = 0.0;
    const int j0 = max(0, i - kd), j1 = min(N - 1, i + kd);
    for (int j = j0; j <= j1; ++j) {
      const double tij = band_at(Tb, kd, i, j);
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if (c < k) tq[c] = fma(tij, Qr[(int64_t)j * k + c], tq[c]);
    }
    double q[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) q[c] = c < k ? Qr[(int64_t)i * k + c] : 0.0;
#pragma unroll
    for (int c = 0; c < KM; ++c)
#pragma unroll
      for (int a = 0; a <= c; ++a) kk[tri(c, a)] = fma(q[a], tq[c], kk[tri(c, a)]);
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) kk[e] = wave_sum(kk[e]);
  if (t == 0) {
#pragma unroll
    for (int c = 0; c < KM; ++c)
#pragma unroll
      for (int a = 0; a <= c; ++a)
        if (c < k) {
          K[a * k + c] = kk[tri(c, a)];
          K[c * k + a] = kk[tri(c, a)];
        }
  }
  __syncthreads();
  wg_jacobi_eig(K, Y, lam, k, cs);
  __syncthreads();
  for (int i = t; i < N; i += 64) {
    double q[KM];
#pragma unroll
    for (int a = 0; a < KM; ++a) q[a] = a < k ? Qr[(int64_t)i * k + a] : 0.0;
    for (int c = 0; c < k; ++c) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < KM; ++a)
        if (a < k) v = fma(q[a], Y[a * k + c], v);
      S[(int64_t)i * k + c] = v;
    }
  }
  __threadfence();
  __syncthreads();
  if (t < k) {
    double rho = 0.0;
    if (Bj) {
      for (int r = 0; r < b; ++r) {
        double v = 0.0;
        for (int m = 0; m < b; ++m) v += Bj[r * b + m] * S[(int64_t)(N - b + m) * k + t];
        rho += v * v;
      }
    }
    res[t] = lam[t];
    res[k + t] = sqrt(rho);
  }
  if (t == 0) {
    const double top = 0.5 * (brk[2 * k] + brk[2 * k + 1]);
    res[2 * k] = fmax(fabs(lam[0]), fabs(top));
    res[2 * k + 1] = top;
  }
}

// Multisection.  Register-window bandwidths: 8192 shifts per round (128
// one-wave workgroups, an eighth of the SIMDs, so that an overlapped check
// leaves most of the chip to the recurrence); other bandwidths (one
// workgroup per shift): 2048.  The first round spreads the shifts over the
// Gershgorin interval, later rounds give each target its own run of
// shifts / (k + 1), rounded down to whole waves.  Rounds continue until every
// bracket has narrowed by at least kNarrow (four rounds for k = 10 on the
// register path: 8193 * 705^3 ~ 2.9e12).  Inverse iteration and Rayleigh-Ritz
// then refine the pairs.
constexpr int kShiftsReg = 8192;
constexpr int kShiftsLds = 2048;
constexpr double kNarrow = 2e12;
constexpr int kInvIters = 2;
// dynamic LDS of the one-wave kernels that stage an N x k block (vectors of
// the inverse iteration, the Rayleigh-Ritz basis)
constexpr size_t kRrLds = 150 * 1024;

bool reg_bandwidth(int kd) { return kd == 1 || kd == 2 || kd == 4 || kd == 8 || kd == 10; }
int shifts_per_target(int nsh, int NT) { return std::max(64, (nsh / NT) / 64 * 64); }

template <int KD, int MODE>
void invit_reg_mode(size_t smem, int grid, const double *band, int N, const double *brk, int k,
                    double *Lscr, double *Dscr, double *X, hipStream_t s) {
  if (smem > 65536) {
    static bool attr = false;  // per process: the kernel's LDS limit
    if (!attr) {
      BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_invit_reg<KD, MODE>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRrLds));
      attr = true;
    }
  }
  hipLaunchKernelGGL((k_invit_reg<KD, MODE>), dim3(grid), dim3(64), smem, s, band, N, brk, k,
                     1e-200, Lscr, Dscr, X, kInvIters);
}

template <int KD>
void invit_reg_launch(const double *band, int N, const double *brk, int k, double *Lscr,
                      double *Dscr, double *X, hipStream_t s) {
  const size_t per_target = (size_t)N * (KD + 2) * sizeof(double);
  const size_t xbytes = (size_t)N * k * sizeof(double);
  if (per_target <= kRrLds)
    invit_reg_mode<KD, 2>(per_target, k, band, N, brk, k, Lscr, Dscr, X, s);
  else if (xbytes <= kRrLds)
    invit_reg_mode<KD, 1>(xbytes, 1, band, N, brk, k, Lscr, Dscr, X, s);
  else
    invit_reg_mode<KD, 0>(0, 1, band, N, brk, k, Lscr, Dscr, X, s);
}

}  // namespace

BandEigLayout band_eig_layout(int N, int kd, int k) {
  BandEigLayout L;
  const int NT = k + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const int nshift = std::max(kShiftsReg, NT * 64);
  L.gersh = take(2 * sizeof(double));
  L.shifts_a = take(nshift * sizeof(double));
  L.shifts_b = take(nshift * sizeof(double));
  L.counts = take(nshift * sizeof(int));
  L.brk = take(2 * NT * sizeof(double));
  L.Lscr = take((size_t)k * N * std::max(kd, 1) * sizeof(double));
  L.Dscr = take((size_t)k * N * sizeof(double));
  L.X = take((size_t)N * k * sizeof(double));
  L.TX = take((size_t)N * k * sizeof(double));
  L.flag = take(64);
  L.bytes = off;
  return L;
}

void band_eigensolve(const double *band, int N, int kd, int k, void *ws, const BandEigLayout &L,
                     const double *Bj, int b, double *S, double *res, hipStream_t s) {
  BBL_REQUIRE(N >= 1 && k >= 1 && k <= N && k <= kMaxBlock && kd >= 0 && kd <= kMaxBlock,
              "band eigensolve: bad sizes");
  char *base = static_cast<char *>(ws);
  double *gersh = reinterpret_cast<double *>(base + L.gersh);
  double *sh_a = reinterpret_cast<double *>(base + L.shifts_a);
  double *sh_b = reinterpret_cast<double *>(base + L.shifts_b);
  int *counts = reinterpret_cast<int *>(base + L.counts);
  double *brk = reinterpret_cast<double *>(base + L.brk);
  double *Lscr = reinterpret_cast<double *>(base + L.Lscr);
  double *Dscr = reinterpret_cast<double *>(base + L.Dscr);
  double *X = reinterpret_cast<double *>(base + L.X);
  double *TX = reinterpret_cast<double *>(base + L.TX);
  const int kdd = std::max(kd, 1);  // kd = 0 (diagonal) handled as bandwidth 1 with zeros
  BBL_REQUIRE(kd >= 1, "band eigensolve: kd must be >= 1");
  const int NT = k + 1;
  const double pivmin = 1e-290;
  hipLaunchKernelGGL(k_gersh, dim3(1), dim3(256), 0, s, band, N, kdd, gersh);
  const bool regk = reg_bandwidth(kdd);
  const int nsh = regk ? kShiftsReg : kShiftsLds;
  const int SP = shifts_per_target(nsh, NT);
  int rounds = 1;
  for (double f = nsh + 1.0; f < kNarrow; f *= SP + 1.0) ++rounds;
  hipLaunchKernelGGL(k_bisect_init, dim3(16), dim3(256), 0, s, gersh, nsh, sh_a, brk, NT);
  check_launch("k_bisect_init");
  const size_t smem_s = (size_t)((kdd + 1) * (kdd + 1) + kChunk * (kdd + 1)) * sizeof(double);
  sturm_counts(band, N, kdd, sh_a, nsh, counts, pivmin, smem_s, s);
  hipLaunchKernelGGL(k_bisect_update, dim3(NT), dim3(256), 0, s, 1, sh_a, counts, nsh, N, k, brk,
                     SP, sh_b);
  check_launch("k_bisect_update");
  for (int r = 1; r < rounds; ++r) {
    sturm_counts(band, N, kdd, sh_b, NT * SP, counts, pivmin, smem_s, s);
    const bool last = (r == rounds - 1);
    hipLaunchKernelGGL(k_bisect_update, dim3(NT), dim3(256), 0, s, 0, sh_b, counts, SP, N, k,
                       brk, SP, last ? nullptr : sh_a);
    check_launch("k_bisect_update");
    std::swap(sh_a, sh_b);
  }
  // inverse iteration: register-window kernel for the common bandwidths,
  // else the LDS-window kernel (x staged in LDS)
  if (regk) {
    switch (kdd) {
      case 1: invit_reg_launch<1>(band, N, brk, k, Lscr, Dscr, X, s); break;
      case 2: invit_reg_launch<2>(band, N, brk, k, Lscr, Dscr, X, s); break;
      case 4: invit_reg_launch<4>(band, N, brk, k, Lscr, Dscr, X, s); break;
      case 8: invit_reg_launch<8>(band, N, brk, k, Lscr, Dscr, X, s); break;
      default: invit_reg_launch<10>(band, N, brk, k, Lscr, Dscr, X, s); break;
    }
    check_launch("k_invit_reg");
  } else {
    const size_t smem = (size_t)((kdd + 1) * (kdd + 1) + kChunk * (kdd + 1) + N) * sizeof(double);
    BBL_REQUIRE(smem <= 150 * 1024, "band eigensolve: band matrix too large for LDS staging");
    if (smem > 64 * 1024)
      BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_invit),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k_invit, dim3(k), dim3(64), smem, s, band, N, kdd, brk, k, 1e-200, Lscr,
                       Dscr, X, kInvIters);
    check_launch("k_invit");
  }
  // Rayleigh-Ritz: one-wave Cholesky QR kernel for k <= 10, with the
  // Gram-Schmidt kernel as its fallback (and for larger k)
  int *fallback = reinterpret_cast<int *>(base + L.flag);
  if (k <= 10) {
    const size_t qbytes = (size_t)N * k * sizeof(double);
    if (qbytes <= kRrLds) {
      static bool attr = false;  // per process: the kernel's LDS limit
      if (!attr) {
        BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rr_fast<10, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRrLds));
        attr = true;
      }
      hipLaunchKernelGGL((k_rr_fast<10, true>), dim3(1), dim3(64), qbytes, s, band, N, kdd, k, X,
                         TX, Bj, b, brk, S, res, fallback);
    } else {
      hipLaunchKernelGGL((k_rr_fast<10, false>), dim3(1), dim3(64), 0, s, band, N, kdd, k, X, TX,
                         Bj, b, brk, S, res, fallback);
    }
    check_launch("k_rr_fast");
    hipLaunchKernelGGL(k_rr, dim3(1), dim3(256), 0, s, band, N, kdd, k, X, TX, Bj, b, brk, S, res,
                       fallback);
  } else {
    hipLaunchKernelGGL(k_rr, dim3(1), dim3(256), 0, s, band, N, kdd, k, X, TX, Bj, b, brk, S, res,
                       nullptr);
  }
  check_launch("k_rr");
}

}  // namespace bbl
