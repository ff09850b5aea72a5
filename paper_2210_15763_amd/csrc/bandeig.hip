// Lowest eigenpairs of the block-tridiagonal band matrix T_j built from the
// A's and B's (Methods: the band matrix "solved using conventional Lapack
// routines").  On the GPU it is solved by
//   1. Sturm-count multisection: the number of negative pivots of the band
//      LDL^T factorisation of (T - sigma I) equals the number of eigenvalues
//      below sigma (Sylvester's law of inertia); many shifts are counted at once,
//      one 64-lane workgroup per shift;
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
        const double lr = win[rs[q] * W + ks];
        const double lc = win[cs[q] * W + ks];
        win[rs[q] * W + cs[q]] -= lr * lc * inv;
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

// Register-window Sturm counts for a compile-time bandwidth KD: one shift per
// lane, 64 shifts per wave.  The (KD+1) x (KD+1) trailing window of the
// partially factored T - sigma I is held as its lower triangle in registers,
// indexed by circular slots; the row loop is unrolled by KD + 1 so that every
// slot index is a compile-time constant.  Band rows are the same for all lanes
// (uniform loads).  Same arithmetic as ldl_sweep, so the counts agree with it.
constexpr int tri(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

// Steps M..KD of one unrolled group of W = KD + 1 rows, slot indices static.
template <int KD, int M>
__device__ __forceinline__ void sturm_steps(const double *__restrict__ Tb, int N, int k0,
                                            double sigma, double pivmin, double (&R)[(KD + 1) * (KD + 2) / 2],
                                            int &cnt) {
  if constexpr (M <= KD) {
    constexpr int W = KD + 1;
    const int k = k0 + M;
    if (k < N) {
      // relative row i of the window lives in slot (M + i) % W
      double d = R[tri(M, M)];
      if (fabs(d) < pivmin) d = -pivmin;
      cnt += d < 0.0 ? 1 : 0;
      const double inv = 1.0 / d;
#pragma unroll
      for (int i = 1; i <= KD; ++i) {
        const int si = (M + i) % W;
        const double li = R[tri(si, M)];
#pragma unroll
        for (int j = 1; j <= i; ++j) {
          const int sj = (M + j) % W;
          R[tri(si, sj)] -= li * R[tri(sj, M)] * inv;
        }
      }
      // row k + W enters in the freed slot M: T[k+W][k+W-t], t = 0..KD
      const int nr = k + W;
#pragma unroll
      for (int t = 0; t <= KD; ++t) {
        double v = 0.0;
        if (nr < N) {
          v = Tb[(int64_t)nr * W + t];
          if (t == 0) v -= sigma;
        }
        R[tri(M, (M + W - t) % W)] = v;
      }
      sturm_steps<KD, M + 1>(Tb, N, k0, sigma, pivmin, R, cnt);
    }
  }
}

template <int KD>
__global__ __launch_bounds__(64) void k_sturm_reg(const double *__restrict__ Tb, int N,
                                                  const double *__restrict__ shifts, int nshift,
                                                  int *__restrict__ counts, double pivmin) {
  constexpr int W = KD + 1;
  constexpr int NP = W * (W + 1) / 2;
  const int id = blockIdx.x * 64 + threadIdx.x;
  const double sigma = id < nshift ? shifts[id] : 0.0;
  double R[NP];
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
  int cnt = 0;
  for (int k0 = 0; k0 < N; k0 += W) {
    sturm_steps<KD, 0>(Tb, N, k0, sigma, pivmin, R, cnt);
  }
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

// Narrow each target's bracket from the counts of the last round, then lay
// out S_next shifts inside every bracket.  Target t < k is eigenvalue index t;
// target k is index N - 1 (the largest).  count(sigma) = #eigenvalues < sigma,
// so lambda_idx lies in [max{sigma: count <= idx}, min{sigma: count > idx}].
__global__ __launch_bounds__(256) void k_bisect_update(int shared_round, const double *shifts,
                                                       const int *counts, int S_per, int N,
                                                       int k, double *brk, int S_next,
                                                       double *next_shifts) {
  __shared__ double slo[256], shi[256];
  const int NT = k + 1;
  for (int tg = 0; tg < NT; ++tg) {
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
    if (threadIdx.x == 0) {
      double l = slo[0], h = shi[0];
      if (l > h) {  // rounding made the counts non-monotone: keep the crossing
        const double m = 0.5 * (l + h);
        l = m;
        h = m;
      }
      brk[2 * tg] = l;
      brk[2 * tg + 1] = h;
    }
    __syncthreads();
  }
  if (next_shifts) {
    for (int e = threadIdx.x; e < NT * S_next; e += blockDim.x) {
      const int tg = e / S_next, s = e % S_next;
      const double l = brk[2 * tg], h = brk[2 * tg + 1];
      next_shifts[e] = l + (h - l) * (double)(s + 1) / (double)(S_next + 1);
    }
  }
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
__global__ __launch_bounds__(256) void k_rr(const double *__restrict__ Tb, int N, int kd, int k,
                                            double *X, double *TX,
                                            const double *__restrict__ Bj, int b,
                                            const double *__restrict__ brk, double *S,
                                            double *res) {
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

constexpr int kShifts1 = 1024;   // first round, shared by all targets
constexpr int kShiftsT = 256;    // later rounds, per target
constexpr int kRounds = 5;       // total multisection rounds
constexpr int kInvIters = 2;

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
  const int nshift = std::max(kShifts1, NT * kShiftsT);
  L.gersh = take(2 * sizeof(double));
  L.shifts_a = take(nshift * sizeof(double));
  L.shifts_b = take(nshift * sizeof(double));
  L.counts = take(nshift * sizeof(int));
  L.brk = take(2 * NT * sizeof(double));
  L.Lscr = take((size_t)k * N * std::max(kd, 1) * sizeof(double));
  L.Dscr = take((size_t)k * N * sizeof(double));
  L.X = take((size_t)N * k * sizeof(double));
  L.TX = take((size_t)N * k * sizeof(double));
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
  hipLaunchKernelGGL(k_bisect_init, dim3(4), dim3(256), 0, s, gersh, kShifts1, sh_a, brk, NT);
  check_launch("k_bisect_init");
  const size_t smem_s = (size_t)((kdd + 1) * (kdd + 1) + kChunk * (kdd + 1)) * sizeof(double);
  sturm_counts(band, N, kdd, sh_a, kShifts1, counts, pivmin, smem_s, s);
  hipLaunchKernelGGL(k_bisect_update, dim3(1), dim3(256), 0, s, 1, sh_a, counts, kShifts1, N, k,
                     brk, kShiftsT, sh_b);
  check_launch("k_bisect_update");
  for (int r = 1; r < kRounds; ++r) {
    sturm_counts(band, N, kdd, sh_b, NT * kShiftsT, counts, pivmin, smem_s, s);
    const bool last = (r == kRounds - 1);
    hipLaunchKernelGGL(k_bisect_update, dim3(1), dim3(256), 0, s, 0, sh_b, counts, kShiftsT, N,
                       k, brk, kShiftsT, last ? nullptr : sh_a);
    check_launch("k_bisect_update");
    std::swap(sh_a, sh_b);
  }
  // inverse iteration (x staged in LDS)
  const size_t smem = (size_t)((kdd + 1) * (kdd + 1) + kChunk * (kdd + 1) + N) * sizeof(double);
  BBL_REQUIRE(smem <= 150 * 1024, "band eigensolve: band matrix too large for LDS staging");
  if (smem > 64 * 1024)
    BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_invit),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  hipLaunchKernelGGL(k_invit, dim3(k), dim3(64), smem, s, band, N, kdd, brk, k, 1e-200, Lscr,
                     Dscr, X, kInvIters);
  check_launch("k_invit");
  hipLaunchKernelGGL(k_rr, dim3(1), dim3(256), 0, s, band, N, kdd, k, X, TX, Bj, b, brk, S, res);
  check_launch("k_rr");
}

}  // namespace bbl
