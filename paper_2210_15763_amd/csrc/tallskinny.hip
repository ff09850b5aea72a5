// Tall-skinny products of the block recurrence on FP64 matrix cores
// (v_mfma_f64_16x16x4_f64):
//   gram   C = X^T Y     -- A_n = V_n^T W_n, the full reorthogonalisation
//                           coefficients V_{1:j}^T W', the overlap W'^T W'
//   update Y <- beta Y + alpha X C
//                        -- the three-term step W' = W - V_n A_n - V_{n-1} B^T,
//                           W' -= V_{1:j} C, right-multiplication by b x b
//                           factors, Ritz vectors X = V_{1:j} S
// X is a set of column blocks of width bx stored block-major (the Krylov
// basis: block i is a row-major n x bx array at X + i*xstride), promoted to
// float64 on load.  All sums run in a fixed order (partials per row chunk,
// then a serial reduction), so results are reproducible bit for bit.
//
// MFMA operand layout used (16x16x4 f64, one block, wave64):
//   A[i][k]: lane l holds i = l % 16, k = l / 16
//   B[k][j]: lane l holds j = l % 16, k = l / 16
//   D[i][j]: lane l, element q holds i = l / 16 + 4 * q, j = l % 16
// (the accumulator's four 64-bit elements are rows strided by 4; checked
// against numpy by the gram/update parity tests)
#include "common.h"

namespace bbl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ double ld(const T *p) { return (double)*p; }

constexpr int kTilesPerWG = 8;   // 16-column tiles of X handled by one gram WG

// partial[p][m][c] for p = blockIdx.x (row chunk), m in this WG's tile group.
template <typename XT, typename YT, int NT>
__global__ __launch_bounds__(256) void k_gram(int64_t n, const XT *__restrict__ X, int bx, int M,
                                              int64_t xstride, const YT *__restrict__ Y, int ny,
                                              int64_t chunk, double *__restrict__ partial,
                                              const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tile0 = blockIdx.y * kTilesPerWG;
  const int ntiles_total = (M + 15) / 16;
  const int ntile = min(kTilesPerWG, ntiles_total - tile0);
  int64_t xoff[kTilesPerWG];
  bool xok[kTilesPerWG];
#pragma unroll
  for (int t = 0; t < kTilesPerWG; ++t) {
    const int m = (tile0 + t) * 16 + li;
    xok[t] = (t < ntile) && (m < M);
    const int blk = xok[t] ? m / bx : 0;
    const int a = xok[t] ? m - blk * bx : 0;
    xoff[t] = (int64_t)blk * xstride + a;
  }
  d4 acc[NT][kTilesPerWG];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int t = 0; t < kTilesPerWG; ++t) acc[u][t] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t r_begin = (int64_t)blockIdx.x * chunk;
  const int64_t r_end = min(n, r_begin + chunk);
  for (int64_t r4 = r_begin + wave * 4; r4 < r_end; r4 += 16) {
    const int64_t r = r4 + lk;
    const bool rok = r < r_end;
    double yv[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int c = u * 16 + li;
      yv[u] = (rok && c < ny) ? ld(Y + r * ny + c) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kTilesPerWG; ++t) {
      if (t < ntile) {
        const double xv = (rok && xok[t]) ? ld(X + xoff[t] + r * bx) : 0.0;
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[u][t] = mfma16(xv, yv[u], acc[u][t]);
      }
    }
  }
  // combine the four waves through LDS (one n-tile at a time)
  __shared__ double red[4][kTilesPerWG][4][64];
  double *out = partial + (int64_t)blockIdx.x * M * ny;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
#pragma unroll
    for (int t = 0; t < kTilesPerWG; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wave][t][q][lane] = acc[u][t][q];
    __syncthreads();
    if (wave == 0) {
      for (int t = 0; t < ntile; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double v = red[0][t][q][lane] + red[1][t][q][lane] + red[2][t][q][lane] +
                           red[3][t][q][lane];
          const int m = (tile0 + t) * 16 + lk + 4 * q;
          const int c = u * 16 + li;
          if (m < M && c < ny) out[(int64_t)m * ny + c] = v;
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partial, int P,
                                                int MN, double *__restrict__ out,
                                                const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= MN) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) s += partial[(int64_t)p * MN + idx];
  out[idx] = s;
}

// Yout[r][c] = beta*Yin[r][c] + alpha*sum_m X[r][m] C[m][c].  One wave per
// 16-row tile.  K-step q of a 16-column slab uses columns m16 + 4*lk + q, so
// each lane reads 4 consecutive columns of its row.
template <typename XT, typename YIT, typename YOT, int NT>
__global__ __launch_bounds__(256) void k_update(int64_t n, const XT *X, int bx,
                                                int M, int64_t xstride,
                                                const double *__restrict__ C, int ny,
                                                double alpha, const YIT *Yin, double beta,
                                                YOT *Yout, const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (r0 >= n) return;
  const int64_t row = r0 + li;
  const bool rok = row < n;
  d4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
  // running (block, column-in-block) of column m16 + 4*lk + q
  int blk[4], a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = 4 * lk + q;
    blk[q] = m / bx;
    a[q] = m - blk[q] * bx;
  }
  for (int m16 = 0; m16 < M; m16 += 16) {
    double xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m16 + 4 * lk + q;
      xv[q] = (rok && m < M) ? ld(X + (int64_t)blk[q] * xstride + row * bx + a[q]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m16 + 4 * lk + q;
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int c = u * 16 + li;
        const double cv = (m < M && c < ny) ? C[(int64_t)m * ny + c] : 0.0;
        acc[u] = mfma16(xv[q], cv, acc[u]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] += 16;
      while (a[q] >= bx) {
        a[q] -= bx;
        ++blk[q];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int c = u * 16 + li;
    if (c >= ny) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + lk + 4 * q;
      if (r < n) {
        double v = alpha * acc[u][q];
        if (beta != 0.0) v = fma(beta, (double)Yin[r * ny + c], v);
        Yout[r * ny + c] = (YOT)v;
      }
    }
  }
}

__global__ void k_fill(double *p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- Philox
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.v[0];
    const uint64_t p1 = (uint64_t)M1 * c.v[2];
    U4 o;
    o.v[0] = (uint32_t)(p1 >> 32) ^ c.v[1] ^ k0;
    o.v[1] = (uint32_t)p1;
    o.v[2] = (uint32_t)(p0 >> 32) ^ c.v[3] ^ k1;
    o.v[3] = (uint32_t)p0;
    c = o;
  }
  return c;
}

__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6) + 0.5) *
         (1.0 / 9007199254740992.0);
}

__global__ void k_gauss(int64_t n, int nvec, int ld, int col0, uint64_t key, uint32_t tag,
                        double *__restrict__ out, const int32_t *__restrict__ colmask,
                        const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int64_t total = n * nvec;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / nvec;
    const int a = (int)(idx - i * nvec);
    if (colmask && colmask[a] == 0) continue;
    U4 c;
    c.v[0] = (uint32_t)i;
    c.v[1] = (uint32_t)((uint64_t)i >> 32);
    c.v[2] = (uint32_t)(a + col0);
    c.v[3] = tag;
    const U4 w = philox4x32_10(c, (uint32_t)key, (uint32_t)(key >> 32));
    const double u1 = u53(w.v[0], w.v[1]);
    const double u2 = u53(w.v[2], w.v[3]);
    out[i * ld + a] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
  }
}

template <typename XT, typename YT>
int gram_typed(int64_t n, const XT *X, int bx, int nblk, int64_t xstride, const YT *Y, int ny,
               double *partial, int max_partials, const int *when, hipStream_t s) {
  const int M = nblk * bx;
  const int tiles = (M + 15) / 16;
  const int gy = (tiles + kTilesPerWG - 1) / kTilesPerWG;
  // row chunk: enough workgroups to fill the chip, bounded partial count
  int64_t gx = std::max<int64_t>(1, std::min<int64_t>(1024 / gy + 1, ceil_div(n, 512)));
  gx = std::min<int64_t>(gx, max_partials);
  int64_t chunk = ceil_div(n, gx);
  chunk = ceil_div(chunk, 16) * 16;
  gx = ceil_div(n, chunk);
  if (ny <= 16)
    hipLaunchKernelGGL((k_gram<XT, YT, 1>), dim3((unsigned)gx, gy), dim3(256), 0, s, n, X, bx, M,
                       xstride, Y, ny, chunk, partial, when);
  else
    hipLaunchKernelGGL((k_gram<XT, YT, 2>), dim3((unsigned)gx, gy), dim3(256), 0, s, n, X, bx, M,
                       xstride, Y, ny, chunk, partial, when);
  check_launch("k_gram");
  return (int)gx;
}

template <typename XT, typename YIT, typename YOT>
void update_typed(int64_t n, const XT *X, int bx, int nblk, int64_t xstride, const double *C,
                  int ny, double alpha, const YIT *Yin, double beta, YOT *Yout, const int *when,
                  hipStream_t s) {
  const int M = nblk * bx;
  const int64_t grid = ceil_div(n, 64);
  if (ny <= 16)
    hipLaunchKernelGGL((k_update<XT, YIT, YOT, 1>), dim3((unsigned)grid), dim3(256), 0, s, n, X,
                       bx, M, xstride, C, ny, alpha, Yin, beta, Yout, when);
  else
    hipLaunchKernelGGL((k_update<XT, YIT, YOT, 2>), dim3((unsigned)grid), dim3(256), 0, s, n, X,
                       bx, M, xstride, C, ny, alpha, Yin, beta, Yout, when);
  check_launch("k_update");
}

}  // namespace

int launch_gram_when(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                     const void *Y, int ydtype, int ny, double *partial, int max_partials,
                     const int *when, hipStream_t s) {
  if (n <= 0 || nblk <= 0) return 0;
  if (xdtype == BBL_F32 && ydtype == BBL_F64)
    return gram_typed(n, (const float *)X, bx, nblk, xstride, (const double *)Y, ny, partial,
                      max_partials, when, s);
  if (xdtype == BBL_F64 && ydtype == BBL_F64)
    return gram_typed(n, (const double *)X, bx, nblk, xstride, (const double *)Y, ny, partial,
                      max_partials, when, s);
  if (xdtype == BBL_F32 && ydtype == BBL_F32)
    return gram_typed(n, (const float *)X, bx, nblk, xstride, (const float *)Y, ny, partial,
                      max_partials, when, s);
  if (xdtype == BBL_F64 && ydtype == BBL_F32)
    return gram_typed(n, (const double *)X, bx, nblk, xstride, (const float *)Y, ny, partial,
                      max_partials, when, s);
  throw Error{BBL_E_INVALID, "gram: dtype"};
}

int launch_gram(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                const void *Y, int ydtype, int ny, double *partial, int max_partials,
                hipStream_t s) {
  return launch_gram_when(n, X, xdtype, bx, nblk, xstride, Y, ydtype, ny, partial, max_partials,
                          nullptr, s);
}

void launch_reduce_when(const double *partial, int P, int M, int ny, double *out,
                        const int *when, hipStream_t s) {
  const int MN = M * ny;
  hipLaunchKernelGGL(k_reduce, dim3((MN + 255) / 256), dim3(256), 0, s, partial, P, MN, out,
                     when);
  check_launch("k_reduce");
}

void launch_reduce(const double *partial, int P, int M, int ny, double *out, hipStream_t s) {
  launch_reduce_when(partial, P, M, ny, out, nullptr, s);
}

void launch_update_when(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                        const double *C, int ny, double alpha, const void *Yin, int yindtype,
                        double beta, void *Yout, int youtdtype, const int *when,
                        hipStream_t s) {
  if (n <= 0) return;
  if (nblk <= 0) {  // empty product: Yout = beta * Yin
    BBL_REQUIRE(false, "update: empty X");
  }
  const bool xf = xdtype == BBL_F32, yif = yindtype == BBL_F32, yof = youtdtype == BBL_F32;
#define BBL_UPD(XT, YIT, YOT)                                                                 \
  update_typed(n, (const XT *)X, bx, nblk, xstride, C, ny, alpha, (const YIT *)Yin, beta,     \
               (YOT *)Yout, when, s)
  if (xf && yif && yof) BBL_UPD(float, float, float);
  else if (xf && yif && !yof) BBL_UPD(float, float, double);
  else if (xf && !yif && yof) BBL_UPD(float, double, float);
  else if (xf && !yif && !yof) BBL_UPD(float, double, double);
  else if (!xf && yif && yof) BBL_UPD(double, float, float);
  else if (!xf && yif && !yof) BBL_UPD(double, float, double);
  else if (!xf && !yif && yof) BBL_UPD(double, double, float);
  else BBL_UPD(double, double, double);
#undef BBL_UPD
}

void launch_update(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                   const double *C, int ny, double alpha, const void *Yin, int yindtype,
                   double beta, void *Yout, int youtdtype, hipStream_t s) {
  launch_update_when(n, X, xdtype, bx, nblk, xstride, C, ny, alpha, Yin, yindtype, beta, Yout,
                     youtdtype, nullptr, s);
}

void launch_fill(double *p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  const int64_t grid = std::min<int64_t>(4096, ceil_div(count, 256));
  hipLaunchKernelGGL(k_fill, dim3((unsigned)grid), dim3(256), 0, s, p, count, v);
  check_launch("k_fill");
}

void launch_gauss(int64_t n, int nvec, int ld, int col0, uint64_t key, uint32_t tag, double *out,
                  const int32_t *colmask, const int *when, hipStream_t s) {
  if (n <= 0) return;
  const int64_t grid = std::min<int64_t>(8192, ceil_div(n * nvec, 256));
  hipLaunchKernelGGL(k_gauss, dim3((unsigned)grid), dim3(256), 0, s, n, nvec, ld, col0, key, tag,
                     out, colmask, when);
  check_launch("k_gauss");
}

}  // namespace bbl
