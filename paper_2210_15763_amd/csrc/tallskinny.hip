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
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.h"
#include "philox.h"

namespace bbl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ double ld(const T *p) { return (double)*p; }

constexpr int kTilesPerWG = 8;   // 16-column tiles of X handled by one gram WG
#ifndef BBL_GRAM_WAVES
#define BBL_GRAM_WAVES 1
#endif
#ifndef BBL_GRAM_WAVE_TARGET
#define BBL_GRAM_WAVE_TARGET 6144
#endif
// FP64-MFMA gram over 8-wide FP32 blocks: waves per workgroup, and the
// number of waves (row chunks x column groups) the grid is sized to
constexpr int kGramWaves = BBL_GRAM_WAVES;
constexpr int kGramWaveTarget = BBL_GRAM_WAVE_TARGET;
// most row chunks of the 8- and 10-wide grams: with one or two column groups
// (up to 16 blocks of 8) the wave target needs 3072-6144 chunks; at 2048 the
// grid left the chip a third full (n = 1e8, 5 / 8 / 16 blocks: 2.7 / 3.5 /
// 5.2 TB/s, now 5.3 / 5.9 / 5.9)
constexpr int kGramMaxChunks = 8192;
#ifndef BBL_GRAM_SMALL_U
#define BBL_GRAM_SMALL_U 8
#endif
#ifndef BBL_GRAM_SMALL_CHUNK
#define BBL_GRAM_SMALL_CHUNK 64
#endif
#ifndef BBL_GRAM1_MIN_ROWS
#define BBL_GRAM1_MIN_ROWS 128
#endif
// short row counts (a truncated problem), where every kernel is bound by the
// latency of its serial load rounds, not by bandwidth: row groups of four in
// flight per wave and rows per wave of the 8-wide FP64-MFMA gram; fewest rows
// per wave of the one-block gram
constexpr int kGramSmallU = BBL_GRAM_SMALL_U;
constexpr int kGramSmallChunk = BBL_GRAM_SMALL_CHUNK;
constexpr int kGram1MinRows = BBL_GRAM1_MIN_ROWS;
#ifndef BBL_GRAMV_MIN_CHUNK
#define BBL_GRAMV_MIN_CHUNK 64
#endif
#ifndef BBL_GRAMV_U
#define BBL_GRAMV_U 4
#endif
// fewest rows per wave of the VALU gram, and its rows in flight per wave
constexpr int kGramVMinChunk = BBL_GRAMV_MIN_CHUNK;
#ifndef BBL_GRAM10_U
#define BBL_GRAM10_U 2
#endif
// row groups of four in flight per wave of the 10-wide FP64-MFMA gram
constexpr int kGram10U = BBL_GRAM10_U;
#ifndef BBL_G16_CG
#define BBL_G16_CG 1
#endif
#ifndef BBL_G16_U
#define BBL_G16_U 2
#endif
#ifndef BBL_G16_WAVES
#define BBL_G16_WAVES 49152
#endif
#ifndef BBL_G16_MIN_WAVES
#define BBL_G16_MIN_WAVES 6144
#endif
#ifndef BBL_G16_MIN_ROWS
#define BBL_G16_MIN_ROWS 1024
#endif
#ifndef BBL_U16_U
#define BBL_U16_U 4
#endif
#ifndef BBL_U16_WAVES
#define BBL_U16_WAVES 8192
#endif
// 16-wide blocks on FP64 matrix cores: gram blocks per wave, 16-row tiles
// in flight and the waves its grid is sized to; update tiles per wave step
// and grid waves (each wave strides over the row tiles).  The gram's waves
// of one row chunk (one per block, on one XCD) share the chunk's rows of W'
// through the L2, which holds them only while the chunk is short: its grid
// aims at kG16Waves waves (at most 2048 row chunks, and no more partial sums
// than the buffer holds) but takes chunks of no fewer than kG16MinRows rows
// beyond kG16MinWaves waves, so short problems keep their partial-sum traffic
// small.  Measured at n = 2e7 (4 / 8 / 20 / 40 blocks): 4.5-5.0 / 4.4 /
// 3.8 / 3.6 TB/s with 6144 waves (154 chunks of 130,000 rows at 40 blocks),
// 4.7-5.4 / 4.7-4.8 / 4.5 / 4.4 with 49152 (840 chunks at 40 blocks, the
// buffer's cap), no faster with the buffer and the chunk cap raised to
// 98,304 or 196,608 waves; one block per wave (two or four per wave:
// slower, fewer waves resident).  Update 5.3 / 5.0 / 4.7 / 4.4 TB/s (2 / 8 /
// 20 / 40 blocks; 1-2 % faster at 32768 waves, not taken: its fused Gram's
// partials grow with the grid)
constexpr int kG16CG = BBL_G16_CG, kG16U = BBL_G16_U, kG16Waves = BBL_G16_WAVES;
constexpr int kG16MinWaves = BBL_G16_MIN_WAVES, kG16MinRows = BBL_G16_MIN_ROWS;
constexpr int kU16U = BBL_U16_U, kU16Waves = BBL_U16_WAVES;
inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

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

// Sum of partial[p0..p1)[idx] in a fixed order: eight interleaved running
// sums (p = p0 + u mod 8) so that eight loads are in flight at a time, then
// a fixed pairwise combination.
__device__ __forceinline__ double sum_strided(const double *__restrict__ partial, int p0, int p1,
                                              int MN, int idx) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double *q = partial + (int64_t)p0 * MN + idx;
  int p = p0;
  for (; p + 8 <= p1; p += 8, q += (int64_t)8 * MN) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += q[(int64_t)u * MN];
  }
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (p + u < p1) a[u] += q[(int64_t)u * MN];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partial, int P,
                                                int MN, double *__restrict__ out,
                                                const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= MN) return;
  out[idx] = sum_strided(partial, 0, P, MN, idx);
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

// ---------------------------------------------------------------------------
// 16-wide blocks on v_mfma_f64_4x4x4f64.  At b = 16 the products carry 8 flop
// per basis byte, near the FP64 ridge, so the VALU forms (scalar C operands,
// 256 FMAs per row and block) run far below the HBM rate; these kernels put
// the four independent 4x4x4 products of one instruction on four groups of
// four rows (operand layout as in k_gram_mfma8: A[i][k] at lane 16k + 4g + i,
// B[k][j] at 16k + 4g + j, D[i][j] at 16i + 4g + j) and read 16-row tiles,
// four lanes per row, each lane one 4-column quarter (one float4 or two
// double2): a load instruction reads 16 whole rows, one contiguous run.

__device__ __forceinline__ void ld4(const float *p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const double *p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0];
  const double2 b = reinterpret_cast<const double2 *>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <typename T>
__device__ __forceinline__ void st4(T *p, const double (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  } else {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
  }
}

// Gram C = X^T Y, X: nblk blocks of 16 columns, Y: n x 16.  Lane l reads row
// t + (l >> 2) of each 16-row tile, columns 4 (l & 3) .. +3 of X and of Y.
// As an A operand (k = l >> 4, g = (l >> 2) & 3, i = l & 3) component q of
// the X quarter is X[t + 4k + g][4i + q]; as a B operand component h of the
// Y quarter is Y[t + 4k + g][4j + h] (j = l & 3): product g sums over the
// rows t + 4k + g, k = 0..3, and D(q, h)[i][j] = C[4i + q][4j + h].  The four
// products' sums are added by two lane shuffles at the end.  One wave takes
// CG blocks over one row chunk, U tiles in flight; workgroup order as in
// k_gram_mfma8 (the column groups of a row chunk on one XCD).
template <typename XT, typename YT, int CG, int U>
__global__ __launch_bounds__(64) void k_gram_mfma16(int64_t n, const XT *__restrict__ X, int nblk,
                                                    int64_t xstride, const YT *__restrict__ Y,
                                                    int64_t chunk, int gx, int gy,
                                                    double *__restrict__ partial,
                                                    const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int sb = blockIdx.x / (8 * gy), rem = blockIdx.x % (8 * gy);
  const int cy = rem / 8, cx = sb * 8 + rem % 8;
  if (cx >= gx) return;
  const int l = threadIdx.x;
  const int rl = l >> 2, e = l & 3;
  const int b0 = cy * CG;
  double acc[CG][4][4];
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 4; ++h) acc[c][q][h] = 0.0;
  const int64_t r0 = (int64_t)cx * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  for (int64_t t = r0; t < r1; t += 16 * U) {
    XT x[U][CG][4];
    YT y[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = t + 16 * u + rl;
      const bool ok = r < r1;
      if (ok) ld4(Y + r * 16 + 4 * e, y[u]);
      else
#pragma unroll
        for (int h = 0; h < 4; ++h) y[u][h] = YT(0);
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        if (ok && b0 + c < nblk) ld4(X + (int64_t)(b0 + c) * xstride + r * 16 + 4 * e, x[u][c]);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) x[u][c][q] = XT(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CG; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int h = 0; h < 4; ++h)
            acc[c][q][h] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)x[u][c][q], (double)y[u][h],
                                                              acc[c][q][h], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double v = acc[c][q][h];
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        acc[c][q][h] = v;
      }
  if (((l >> 2) & 3) == 0) {
    const int i = l >> 4, j = l & 3;
    const int64_t M = (int64_t)nblk * 16;
    double *out = partial + (int64_t)cx * M * 16;
#pragma unroll
    for (int c = 0; c < CG; ++c)
      if (b0 + c < nblk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double v4[4] = {acc[c][q][0], acc[c][q][1], acc[c][q][2], acc[c][q][3]};
          st4(out + ((int64_t)(b0 + c) * 16 + 4 * i + q) * 16 + 4 * j, v4);
        }
  }
}

// Yout = beta Yin + alpha X C over 16-wide blocks, C: (16 nblk) x 16.  A
// operand (k = l >> 4, g = (l >> 2) & 3, i = l & 3): lane l reads row
// t + (l & 15) of the tile, basis columns 4k .. 4k + 3 (component q is column
// 4k + q); B operand (q, h): C[16 blk + 4k + q][4j + h], j = l & 3, which each
// lane loads per block (four 32-byte runs); D(h)[i][j] at lane 16i + 4g + j is
// Yout[t + 4g + i][4j + h].  A wave strides over tiles of 16 U rows.
// GRAM: the wave also sums the Gram matrix of the values it stored: as an A
// (or B) operand, lane 16k + 4g + j holds row t + 4g + k, columns 4j + h, so
// the output registers feed sixteen more products per tile directly;
// gpart[wave][16][16], the four groups' sums added by lane shuffles.
template <typename XT, typename YIT, typename YOT, int U, bool GRAM>
__global__ __launch_bounds__(64) void k_update_mfma16(int64_t n, const XT *__restrict__ X, int nblk,
                                                      int64_t xstride, const double *__restrict__ C,
                                                      double alpha, const YIT *Yin, double beta,
                                                      YOT *Yout, const int *__restrict__ when,
                                                      double *__restrict__ gpart) {
  if (when && *when == 0) return;
  const int l = threadIdx.x;
  const int kq = l >> 4, e = l & 3, ra = l & 15;     // A operand: quarter kq of row ra
  const int rd = 4 * ((l >> 2) & 3) + (l >> 4);      // D: row of the tile this lane holds
  double gacc[GRAM ? 4 : 1][GRAM ? 4 : 1];
  if constexpr (GRAM) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 4; ++h) gacc[q][h] = 0.0;
  }
  const int64_t tiles = (n + 16 * U - 1) / (16 * U);
  for (int64_t tt = blockIdx.x; tt < tiles; tt += gridDim.x) {
    const int64_t t = tt * (16 * U);
    double acc[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < 4; ++h) acc[u][h] = 0.0;
    for (int blk = 0; blk < nblk; ++blk) {
      double cb[4][4];
      const double *cp = C + ((int64_t)blk * 16 + 4 * kq) * 16 + 4 * e;
#pragma unroll
      for (int q = 0; q < 4; ++q) ld4(cp + q * 16, cb[q]);
      XT x[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = t + 16 * u + ra;
        if (r < n) ld4(X + (int64_t)blk * xstride + r * 16 + 4 * kq, x[u]);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) x[u][q] = XT(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int h = 0; h < 4; ++h)
            acc[u][h] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)x[u][q], cb[q][h], acc[u][h],
                                                           0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = t + 16 * u + rd;
      double o[4] = {0.0, 0.0, 0.0, 0.0};
      if (r < n) {
        if (beta != 0.0) {
          YIT yi[4];
          ld4(Yin + r * 16 + 4 * e, yi);
#pragma unroll
          for (int h = 0; h < 4; ++h) o[h] = fma(beta, (double)yi[h], alpha * acc[u][h]);
        } else {
#pragma unroll
          for (int h = 0; h < 4; ++h) o[h] = alpha * acc[u][h];
        }
        st4(Yout + r * 16 + 4 * e, o);
#pragma unroll
        for (int h = 0; h < 4; ++h) o[h] = (double)(YOT)o[h];  // the values as stored
      }
      if constexpr (GRAM) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int h = 0; h < 4; ++h)
            gacc[q][h] = __builtin_amdgcn_mfma_f64_4x4x4f64(o[q], o[h], gacc[q][h], 0, 0, 0);
      }
    }
  }
  if constexpr (GRAM) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double v = gacc[q][h];
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        gacc[q][h] = v;
      }
    if (((l >> 2) & 3) == 0) {
      const int i = l >> 4, j = l & 3;
      double *out = gpart + (int64_t)blockIdx.x * 256;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v4[4] = {gacc[q][0], gacc[q][1], gacc[q][2], gacc[q][3]};
        st4(out + (4 * i + q) * 16 + 4 * j, v4);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// VALU FP64 variants for the common block widths.  At nvec <= 10 the gram's
// 16x16x4 MFMA would spend most of its FMAs on padding (N = nvec of 16),
// while plain v_fma_f64 runs at the same peak with no padding; the uniform
// operand (a row of Y in gram, a row of C in update) is wave-uniform and is
// fetched with scalar loads into SGPRs.
template <typename T, int N>
struct Vec {
  T v[N];
};

template <typename T, int N>
__device__ __forceinline__ Vec<T, N> vload(const T *p) {
  Vec<T, N> r;
  constexpr int bytes = (int)sizeof(T) * N;
  if constexpr (bytes % 16 == 0) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    uint4 tmp[bytes / 16];
#pragma unroll
    for (int i = 0; i < bytes / 16; ++i) tmp[i] = q[i];
    __builtin_memcpy(r.v, tmp, bytes);
  } else if constexpr (bytes % 8 == 0) {
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
    uint2 tmp[bytes / 8];
#pragma unroll
    for (int i = 0; i < bytes / 8; ++i) tmp[i] = q[i];
    __builtin_memcpy(r.v, tmp, bytes);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) r.v[i] = p[i];
  }
  return r;
}

// Gram over 8-wide FP32 basis blocks on v_mfma_f64_4x4x4f64 (four independent
// 4x4x4 products per instruction; operand layout: block g = (l % 16) / 4,
// A[i][k] at lane 16k + 4g + i, B[k][j] at lane 16k + 4g + j, D[i][j] at lane
// 16i + 4g + j).  K runs over rows.  Lane (k, g, e) loads ONE float4 of row
// r0 + k: X columns c0 + 16g + 4e .. +3 (inside one 8-wide block row), so one
// load instruction reads four whole 128-byte lines (rows r0..r0+3 of eight
// basis blocks) and no X element is loaded twice.  Its four components feed
// four MFMA pairs q = 0..3; in pair q, block g computes the 4x4 tiles of X
// columns c0 + 16g + 4i + q against Y columns 2j and 2j + 1 (lane j = e loads
// both with one 16-byte load: half the Y load instructions of columns j and
// 4 + j, 5-9 % faster at 90-181 blocks).  Each wave covers 64*CG columns and
// keeps U row groups of four in flight.
//
// Workgroup order: the gy column groups of one row chunk share that chunk of
// Y, so they are given workgroup ids congruent modulo 8 (the same XCD, whose
// L2 then serves Y to all of them) and close in dispatch order.  Linear id i:
// super-block i / (8 gy) holds row chunks 8 sb .. 8 sb + 7, inside it
// column group (i % (8 gy)) / 8 and row chunk 8 sb + i % 8.
//
// WPG waves per workgroup: the waves of one workgroup take WPG consecutive
// column groups of the same row chunk (so they read the same rows of Y at
// about the same time, from the CU's vector cache), gq = ceil(gy / WPG)
// workgroups per row chunk in the order above.
template <int CG, int U, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_gram_mfma8(int64_t n, const float *__restrict__ X,
                                                         int M, int64_t xstride,
                                                         const double *__restrict__ Y,
                                                         int64_t chunk, int gx, int gy,
                                                         double *__restrict__ partial,
                                                         const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int gq = (gy + WPG - 1) / WPG;
  const int sb = blockIdx.x / (8 * gq), rem = blockIdx.x % (8 * gq);
  const int cy = (rem / 8) * WPG + (int)(threadIdx.x >> 6), cx = sb * 8 + rem % 8;
  if (cx >= gx || cy >= gy) return;
  const int l = threadIdx.x & 63;
  const int k = l >> 4, g = (l & 15) >> 2, e = l & 3;
  const int c00 = cy * (64 * CG);
  int64_t xo[CG];
  bool ok[CG];
#pragma unroll
  for (int c = 0; c < CG; ++c) {
    const int col = c00 + 64 * c + 16 * g + 4 * e;  // first of 4 columns
    ok[c] = col < M;
    const int blk = col >> 3, a = col & 7;
    xo[c] = (int64_t)blk * xstride + a;
  }
  double acc[CG][4][2];
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[c][q][0] = acc[c][q][1] = 0.0;
  const int64_t r0 = (int64_t)cx * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  for (int64_t rb = r0; rb < r1; rb += 4 * U) {
    double y0[U], y1[U];
    float4 x[U][CG];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = rb + 4 * u + k;
      const bool rok = r < r1;
      const double2 yy = rok ? *reinterpret_cast<const double2 *>(Y + r * 8 + 2 * e)
                             : make_double2(0.0, 0.0);
      y0[u] = yy.x;
      y1[u] = yy.y;
#pragma unroll
      for (int c = 0; c < CG; ++c)
        x[u][c] = (rok && ok[c]) ? *reinterpret_cast<const float4 *>(X + xo[c] + r * 8)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        const double xs[4] = {(double)x[u][c].x, (double)x[u][c].y, (double)x[u][c].z,
                              (double)x[u][c].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[c][q][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(xs[q], y0[u], acc[c][q][0], 0, 0, 0);
          acc[c][q][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(xs[q], y1[u], acc[c][q][1], 0, 0, 0);
        }
      }
  }
  // D lane l = 16i + 4g + j holds tile (g, q) element (i, j): X column
  // c0 + 16g + 4i + q with i = k (l >> 4), Y columns 2j and 2j + 1, j = e
  double *out = partial + (int64_t)cx * M * 8;
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = c00 + 64 * c + 16 * g + 4 * k + q;
      if (m < M) {
        *reinterpret_cast<double2 *>(out + (int64_t)m * 8 + 2 * e) =
            make_double2(acc[c][q][0], acc[c][q][1]);
      }
    }
}

// Gram over 10-wide FP32 basis blocks (Y: n x 10) on v_mfma_f64_4x4x4f64,
// with the operand layout of k_gram_mfma8.  Each block's 10 columns take 12
// padded columns (three quads, the last ending in two zero columns), so no
// quad of four consecutive columns straddles two blocks: lane (k, g, e) loads
// padded columns 64 cy + 16 g + 4 e .. +3 of row r0 + k, two float2 runs
// (one for the last quad; rows of 40 bytes keep them 8-byte aligned); Y's 10
// columns are three B operands: columns 2e and 2e + 1 (one load) and 8 + e
// (lanes e < 2; zeros in the others).  D lane 16i + 4g + j of product (q, t)
// holds padded X column 64 cy + 16 g + 4 i + q against Y column 2j + t
// (t < 2) or 8 + j (t = 2, j < 2); padded columns are not stored.  Work
// split, grid and workgroup order as in k_gram_mfma8.
template <typename YT, int U>
__global__ __launch_bounds__(64) void k_gram_mfma10(int64_t n, const float *__restrict__ X,
                                                    int nblk, int64_t xstride,
                                                    const YT *__restrict__ Y, int64_t chunk,
                                                    int gx, int gy, double *__restrict__ partial,
                                                    const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int sb = blockIdx.x / (8 * gy), rem = blockIdx.x % (8 * gy);
  const int cy = rem / 8, cx = sb * 8 + rem % 8;
  if (cx >= gx) return;
  const int l = threadIdx.x;
  const int k = l >> 4, g = (l & 15) >> 2, e = l & 3;
  const int Mp = nblk * 12;
  const int cp = cy * 64 + 16 * g + 4 * e;  // first padded column of this lane's quad
  const bool ok = cp < Mp;
  const int a0 = cp % 12;                   // 0, 4 or 8
  const float *xp = X + (int64_t)(ok ? cp / 12 : 0) * xstride + a0;
  double acc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[q][t] = 0.0;
  const int64_t r0 = (int64_t)cx * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  for (int64_t rb = r0; rb < r1; rb += 4 * U) {
    float x[U][4];
    double y[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = rb + 4 * u + k;
      const bool rok = r < r1;
      // columns 2e, 2e + 1 and 8 + e
      if (rok) {
        if constexpr (sizeof(YT) == 8) {
          const double2 yy = *reinterpret_cast<const double2 *>(Y + r * 10 + 2 * e);
          y[u][0] = yy.x;
          y[u][1] = yy.y;
        } else {
          const float2 yy = *reinterpret_cast<const float2 *>(Y + r * 10 + 2 * e);
          y[u][0] = yy.x;
          y[u][1] = yy.y;
        }
      } else {
        y[u][0] = y[u][1] = 0.0;
      }
      y[u][2] = (rok && e < 2) ? (double)Y[r * 10 + 8 + e] : 0.0;
      float2 p0 = make_float2(0.f, 0.f), p1 = make_float2(0.f, 0.f);
      if (rok && ok) {
        p0 = *reinterpret_cast<const float2 *>(xp + r * 10);
        if (a0 < 8) p1 = *reinterpret_cast<const float2 *>(xp + r * 10 + 2);
      }
      x[u][0] = p0.x;
      x[u][1] = p0.y;
      x[u][2] = p1.x;
      x[u][3] = p1.y;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 3; ++t)
          acc[q][t] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)x[u][q], y[u][t], acc[q][t], 0,
                                                         0, 0);
  }
  double *out = partial + (int64_t)cx * nblk * 10 * 10;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cy * 64 + 16 * g + 4 * k + q;  // padded X column of row i = k of D
    const int a = c % 12;
    if (c < Mp && a < 10) {
      const int64_t m = (int64_t)(c / 12) * 10 + a;
      out[m * 10 + 2 * e] = acc[q][0];
      out[m * 10 + 2 * e + 1] = acc[q][1];
      if (e < 2) out[m * 10 + 8 + e] = acc[q][2];
    }
  }
}

// Single-block gram C = X^T Y (X, Y: n x B row-major): lane = row, each lane
// accumulates the B x B outer products of its rows, then one butterfly per
// wave combines the lanes (fixed order).  partial[p][a][j], p = wave index.
template <typename XT, typename YT, int B>
__global__ __launch_bounds__(256) void k_gram1(int64_t n, const XT *__restrict__ X,
                                               const YT *__restrict__ Y, int64_t rows_per_wave,
                                               double *__restrict__ partial,
                                               const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = wave * rows_per_wave;
  const int64_t r1 = min(n, r0 + rows_per_wave);
  double acc[B][B];
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int j = 0; j < B; ++j) acc[a][j] = 0.0;
  for (int64_t r = r0 + lane; r < r1; r += 64) {
    const Vec<XT, B> x = vload<XT, B>(X + r * B);
    const Vec<YT, B> y = vload<YT, B>(Y + r * B);
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int j = 0; j < B; ++j) acc[a][j] = fma((double)x.v[a], (double)y.v[j], acc[a][j]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int j = 0; j < B; ++j) acc[a][j] += __shfl_xor(acc[a][j], off, 64);
  if (lane == 0) {
    double *out = partial + wave * B * B;
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int j = 0; j < B; ++j) out[a * B + j] = acc[a][j];
  }
}

// Single-block gram over 10 columns (X, Y: n x 10 row-major): a lane pair
// shares a row, lane 2p + h taking X columns 5h .. 5h + 4 against all ten Y
// columns (50 sums per lane, so the wave keeps three-way occupancy where
// k_gram1's 100 sums per lane would leave one); one butterfly over the lanes
// of each parity adds them (fixed order).  partial[p][a][j], p = wave index.
template <typename XT, typename YT>
__global__ __launch_bounds__(256) void k_gram1_10(int64_t n, const XT *__restrict__ X,
                                                  const YT *__restrict__ Y,
                                                  int64_t rows_per_wave,
                                                  double *__restrict__ partial,
                                                  const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int lane = threadIdx.x & 63, h = lane & 1;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t r0 = wave * rows_per_wave;
  const int64_t r1 = min(n, r0 + rows_per_wave);
  double acc[5][10];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[a][j] = 0.0;
  for (int64_t r = r0 + (lane >> 1); r < r1; r += 32) {
    double x[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) x[a] = (double)X[r * 10 + 5 * h + a];
    const Vec<YT, 10> y = vload<YT, 10>(Y + r * 10);
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int j = 0; j < 10; ++j) acc[a][j] = fma(x[a], (double)y.v[j], acc[a][j]);
  }
#pragma unroll
  for (int off = 32; off > 1; off >>= 1)
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int j = 0; j < 10; ++j) acc[a][j] += __shfl_xor(acc[a][j], off, 64);
  if (lane < 2) {
    double *out = partial + wave * 100 + 50 * h;
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int j = 0; j < 10; ++j) out[a * 10 + j] = acc[a][j];
  }
}

// One wave per workgroup; lane owns CPL consecutive columns of X (inside one
// block) and accumulates their products with all NY columns of Y over the
// wave's contiguous row range.  partial[p][m][j], p = blockIdx.x.
template <typename XT, typename YT, int NY, int CPL>
__global__ __launch_bounds__(64) void k_gram_v(int64_t n, const XT *__restrict__ X, int bx, int M,
                                               int64_t xstride, const YT *__restrict__ Y,
                                               int64_t chunk, double *__restrict__ partial,
                                               const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int lane = threadIdx.x;
  const int m0 = (blockIdx.y * 64 + lane) * CPL;
  const bool ok = m0 < M;
  const int blk = ok ? m0 / bx : 0;
  const int a = ok ? m0 - blk * bx : 0;
  const XT *xp = X + (int64_t)blk * xstride + a;
  double acc[CPL][NY];
#pragma unroll
  for (int c = 0; c < CPL; ++c)
#pragma unroll
    for (int j = 0; j < NY; ++j) acc[c][j] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  int64_t r = r0;
  constexpr int U = BBL_GRAMV_U;
  for (; r + U <= r1; r += U) {
    Vec<XT, CPL> xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok) xv[u] = vload<XT, CPL>(xp + (r + u) * bx);
      else
#pragma unroll
        for (int c = 0; c < CPL; ++c) xv[u].v[c] = XT(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const YT *yr = Y + (r + u) * NY;
#pragma unroll
      for (int j = 0; j < NY; ++j) {
        const double y = (double)yr[j];
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c][j] = fma((double)xv[u].v[c], y, acc[c][j]);
      }
    }
  }
  for (; r < r1; ++r) {
    Vec<XT, CPL> xv;
    if (ok) xv = vload<XT, CPL>(xp + r * bx);
    else
#pragma unroll
      for (int c = 0; c < CPL; ++c) xv.v[c] = XT(0);
    const YT *yr = Y + r * NY;
#pragma unroll
    for (int j = 0; j < NY; ++j) {
      const double y = (double)yr[j];
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c][j] = fma((double)xv.v[c], y, acc[c][j]);
    }
  }
  if (ok) {
    double *out = partial + ((int64_t)blockIdx.x * M + m0) * NY;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
      for (int j = 0; j < NY; ++j) out[c * NY + j] = acc[c][j];
  }
}

// Yout[r][j] = beta*Yin[r][j] + alpha*sum_m X[r][m] C[m][j], X blocks of width
// BX, one row per lane (RPL rows per lane, 256-row stride), C rows scalar.
//
// GRAM: also the Gram matrix of the rows this workgroup wrote,
// gpart[blockIdx.x][a][c] = sum_r Yout[r][a] Yout[r][c] (the values as
// stored), which saves a separate pass over Yout when the next step needs
// Yout^T Yout.  Each 256-row tile of output goes through LDS; thread
// (e, s) sums entry e over the tile rows s, s + S, ... and the S slices
// are added in a fixed order, so the result is deterministic and the main
// loop keeps its register budget (occupancy).
//
// PF > 1: the loads of PF blocks are issued before their products (for short
// grids, where each lane's walk over the blocks is latency-bound).
template <typename XT, typename YIT, typename YOT, int BX, int NY, int RPL, bool GRAM, int PF,
          bool TL = false>
__global__ __launch_bounds__(256) void k_update_v(int64_t n, const XT *X, int nblk,
                                                  int64_t xstride, const double *__restrict__ C,
                                                  double alpha, const YIT *Yin, double beta,
                                                  YOT *Yout, const int *__restrict__ when,
                                                  double *__restrict__ gpart) {
  if (when && *when == 0) return;
  constexpr int NP = NY * (NY + 1) / 2;
  constexpr int S = (256 / NP) > 0 ? 256 / NP : 1;  // slices per Gram entry
  static_assert(NP <= 256, "Gram epilogue: too many entries");
  __shared__ double tile[GRAM ? 256 : 1][GRAM ? NY : 1];
  __shared__ double red[GRAM ? 256 : 1];
  const int t = threadIdx.x;
  int ga = 0, gc = 0;  // Gram entry (a <= c) of this thread
  if (GRAM && t < NP * S) {
    const int e = t / S;
    while ((gc + 1) * (gc + 2) / 2 <= e) ++gc;
    ga = e - gc * (gc + 1) / 2;
  }
  double gsum = 0.0;
  // tiles of 256 RPL rows: one per workgroup, or (TL: the grid was capped to
  // bound the Gram partials) a workgroup strides over them
  auto do_tile = [&](int64_t tl) __attribute__((always_inline)) {
    const int64_t base = tl * 256 * RPL + threadIdx.x;
    double acc[RPL][NY];
#pragma unroll
    for (int u = 0; u < RPL; ++u)
#pragma unroll
      for (int j = 0; j < NY; ++j) acc[u][j] = 0.0;
    int blk0 = 0;
    if constexpr (PF > 1) {
      for (; blk0 + PF <= nblk; blk0 += PF) {
        Vec<XT, BX> xp[PF][RPL];
#pragma unroll
        for (int p = 0; p < PF; ++p)
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int64_t r = base + (int64_t)u * 256;
            if (r < n) xp[p][u] = vload<XT, BX>(X + (int64_t)(blk0 + p) * xstride + r * BX);
            else
#pragma unroll
              for (int c = 0; c < BX; ++c) xp[p][u].v[c] = XT(0);
          }
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const double *cb = C + (int64_t)(blk0 + p) * BX * NY;
#pragma unroll
          for (int a = 0; a < BX; ++a) {
#pragma unroll
            for (int j = 0; j < NY; ++j) {
              const double cv = cb[a * NY + j];
#pragma unroll
              for (int u = 0; u < RPL; ++u) acc[u][j] = fma((double)xp[p][u].v[a], cv, acc[u][j]);
            }
          }
        }
      }
    }
    for (int blk = blk0; blk < nblk; ++blk) {
      Vec<XT, BX> xv[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int64_t r = base + (int64_t)u * 256;
        if (r < n) xv[u] = vload<XT, BX>(X + (int64_t)blk * xstride + r * BX);
        else
#pragma unroll
          for (int c = 0; c < BX; ++c) xv[u].v[c] = XT(0);
      }
      const double *cb = C + (int64_t)blk * BX * NY;
#pragma unroll
      for (int a = 0; a < BX; ++a) {
#pragma unroll
        for (int j = 0; j < NY; ++j) {
          const double cv = cb[a * NY + j];
#pragma unroll
          for (int u = 0; u < RPL; ++u) acc[u][j] = fma((double)xv[u].v[a], cv, acc[u][j]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int64_t r = base + (int64_t)u * 256;
      double ov[NY];
#pragma unroll
      for (int j = 0; j < NY; ++j) ov[j] = 0.0;
      if (r < n) {
        YOT o[NY];
        if (beta != 0.0) {
          const Vec<YIT, NY> yi = vload<YIT, NY>(Yin + r * NY);
#pragma unroll
          for (int j = 0; j < NY; ++j) o[j] = (YOT)fma(beta, (double)yi.v[j], alpha * acc[u][j]);
        } else {
#pragma unroll
          for (int j = 0; j < NY; ++j) o[j] = (YOT)(alpha * acc[u][j]);
        }
#pragma unroll
        for (int j = 0; j < NY; ++j) {
          Yout[r * NY + j] = o[j];
          ov[j] = (double)o[j];
        }
      }
      if constexpr (GRAM) {
        __syncthreads();  // the previous tile is consumed
#pragma unroll
        for (int j = 0; j < NY; ++j) tile[t][j] = ov[j];
        __syncthreads();
        if (t < NP * S)
          for (int q = t % S; q < 256; q += S) gsum = fma(tile[q][ga], tile[q][gc], gsum);
      }
    }
  };
  if constexpr (TL) {
    const int64_t ntiles = (n + 256 * RPL - 1) / (256 * RPL);
    for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) do_tile(tl);
  } else {
    do_tile(blockIdx.x);
  }
  if constexpr (GRAM) {
    red[t] = gsum;
    __syncthreads();
    if (t < NP) {
      int c = 0;
      while ((c + 1) * (c + 2) / 2 <= t) ++c;
      const int a = t - c * (c + 1) / 2;
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += red[t * S + q];
      double *out = gpart + (int64_t)blockIdx.x * NY * NY;
      out[a * NY + c] = v;
      out[c * NY + a] = v;
    }
  }
}

// Update for short row counts (a truncated problem): Yout = beta Yin +
// alpha X C with the basis blocks split over the eight waves of a workgroup
// (wave w takes blocks w, w + 8, ...) and one row per lane, so the grid holds
// eight times as many waves as one row per lane over all blocks would; the
// eight partial sums of each row are added in LDS in fixed order, thread t
// finishing component t / 64 of row t % 64.  Lane l loads entry l of a
// block's BX x NY slice of C (one vector load per block) and the products
// take the entries with v_readlane: scalar loads of C, whose slices of all
// blocks do not fit the scalar cache, ran at half this speed (n = 20,000,
// 91 blocks: 48 against 26 us).
//
// GRAM: also gpart[blockIdx.x][a][c] = sum over the workgroup's 64 rows of
// Yout[r][a] Yout[r][c] (the values as stored): thread (e, q) sums entry e
// over rows q, q + S, ... and the S slices are added in fixed order.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <typename XT, typename YIT, typename YOT, int BX, int NY, bool GRAM>
__global__ __launch_bounds__(512) void k_update_w8(int64_t n, const XT *X, int nblk,
                                                   int64_t xstride, const double *__restrict__ C,
                                                   double alpha, const YIT *Yin, double beta,
                                                   YOT *Yout, const int *__restrict__ when,
                                                   double *__restrict__ gpart) {
  static_assert(NY <= 8, "one component per wave");
  static_assert(BX * NY <= 64, "one C entry per lane");
  constexpr int NP = NY * (NY + 1) / 2;
  constexpr int S = 512 / NP;  // slices per Gram entry
  if (when && *when == 0) return;
  __shared__ double part[8][64][NY];
  __shared__ double gt[GRAM ? 64 : 1][NY + 1];
  __shared__ double red[GRAM ? 512 : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  double acc[NY];
#pragma unroll
  for (int j = 0; j < NY; ++j) acc[j] = 0.0;
  // the loop is uniform over the wave (v_readlane reads a lane whether it is
  // active or not, so every lane loads its C entry); rows past n load zeros
  for (int blk = w; blk < nblk; blk += 8) {
    Vec<XT, BX> xv;
    if (r < n) xv = vload<XT, BX>(X + (int64_t)blk * xstride + r * BX);
    else
#pragma unroll
      for (int c = 0; c < BX; ++c) xv.v[c] = XT(0);
    const double cl = lane < BX * NY ? C[(int64_t)blk * BX * NY + lane] : 0.0;
#pragma unroll
    for (int a = 0; a < BX; ++a)
#pragma unroll
      for (int j = 0; j < NY; ++j) acc[j] = fma((double)xv.v[a], readlane_f64(cl, a * NY + j), acc[j]);
  }
#pragma unroll
  for (int j = 0; j < NY; ++j) part[w][lane][j] = acc[j];
  __syncthreads();
  double o = 0.0;
  if (w < NY && r < n) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) v += part[q][lane][w];
    o = beta != 0.0 ? fma(beta, (double)Yin[r * NY + w], alpha * v) : alpha * v;
    const YOT ov = (YOT)o;
    Yout[r * NY + w] = ov;
    o = (double)ov;
  }
  if constexpr (GRAM) {
    if (w < NY) gt[lane][w] = o;
    __syncthreads();
    const int t = threadIdx.x;
    double gsum = 0.0;
    int ga = 0, gc = 0;
    if (t < NP * S) {
      const int e = t / S;
      while ((gc + 1) * (gc + 2) / 2 <= e) ++gc;
      ga = e - gc * (gc + 1) / 2;
      for (int q = t % S; q < 64; q += S) gsum = fma(gt[q][ga], gt[q][gc], gsum);
    }
    red[t] = gsum;
    __syncthreads();
    if (t < NP) {
      int c = 0;
      while ((c + 1) * (c + 2) / 2 <= t) ++c;
      const int a = t - c * (c + 1) / 2;
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += red[t * S + q];
      double *out = gpart + (int64_t)blockIdx.x * NY * NY;
      out[a * NY + c] = v;
      out[c * NY + a] = v;
    }
  }
}

// Two-stage fixed-order reduction of partial[P][MN]: stage 1 sums S
// contiguous ranges of p, stage 2 sums the S results.
__global__ __launch_bounds__(256) void k_reduce1(const double *__restrict__ partial, int P, int MN,
                                                 int S, double *__restrict__ tmp,
                                                 const int *__restrict__ when) {
  if (when && *when == 0) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int sidx = blockIdx.y;
  if (idx >= MN) return;
  const int p0 = (int)((int64_t)P * sidx / S), p1 = (int)((int64_t)P * (sidx + 1) / S);
  tmp[(int64_t)sidx * MN + idx] = sum_strided(partial, p0, p1, MN, idx);
}

__global__ void k_fill(double *p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- Philox
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

template <typename XT, typename YT, int NY, int CPL>
int gram_valu(int64_t n, const XT *X, int bx, int nblk, int64_t xstride, const YT *Y,
              double *partial, int max_partials, const int *when, hipStream_t s) {
  const int M = nblk * bx;
  const int gy = (M + 64 * CPL - 1) / (64 * CPL);
  int64_t gx = std::max<int64_t>(1, std::min<int64_t>(2048 / gy + 1, ceil_div(n, kGramVMinChunk)));
  gx = std::min<int64_t>(gx, std::max(1, max_partials));
  int64_t chunk = ceil_div(n, gx);
  gx = ceil_div(n, chunk);
  hipLaunchKernelGGL((k_gram_v<XT, YT, NY, CPL>), dim3((unsigned)gx, gy), dim3(64), 0, s, n, X, bx,
                     M, xstride, Y, chunk, partial, when);
  check_launch("k_gram_v");
  return (int)gx;
}

template <typename XT, typename YT, int CG, int U>
int gram_mfma16(int64_t n, const XT *X, int nblk, int64_t xstride, const YT *Y, double *partial,
                int max_partials, const int *when, hipStream_t s) {
  const int gy = (int)ceil_div(nblk, CG);
  int64_t gx = std::max(ceil_div(kG16MinWaves, gy),
                        std::min(ceil_div(kG16Waves, gy), ceil_div(n, kG16MinRows)));
  gx = std::min<int64_t>(2048, gx);
  gx = std::max<int64_t>(1, std::min<int64_t>(gx, ceil_div(n, 16 * U)));
  gx = std::min<int64_t>(gx, std::max(1, max_partials));
  const int64_t chunk = ceil_div(ceil_div(n, gx), 16 * U) * (16 * U);
  gx = ceil_div(n, chunk);
  const int64_t grid = ceil_div(gx, 8) * 8 * gy;
  hipLaunchKernelGGL((k_gram_mfma16<XT, YT, CG, U>), dim3((unsigned)grid), dim3(64), 0, s, n, X,
                     nblk, xstride, Y, chunk, (int)gx, gy, partial, when);
  check_launch("k_gram_mfma16");
  return (int)gx;
}

template <typename XT, typename YT>
int gram_typed(int64_t n, const XT *X, int bx, int nblk, int64_t xstride, const YT *Y, int ny,
               double *partial, int max_partials, const int *when, hipStream_t s) {
  const int M = nblk * bx;
  constexpr bool f32 = sizeof(XT) == 4;
  if (bx == 16 && ny == 16 && aligned16(X) && aligned16(Y)) {
    // one block with float32 operands (A_J = V_J^T W) streams fastest with
    // one tile in flight (4.6 against 3.4 TB/s at n = 2e7)
    if (nblk == 1 && sizeof(YT) == 4)
      return gram_mfma16<XT, YT, 1, 1>(n, X, nblk, xstride, Y, partial, max_partials, when, s);
    return gram_mfma16<XT, YT, kG16CG, kG16U>(n, X, nblk, xstride, Y, partial, max_partials,
                                              when, s);
  }
  if (nblk == 1 && ny == bx && (bx == 4 || bx == 8 || bx == 10)) {
    // one block: rows across lanes (10 columns: lane pairs), 1024 waves at
    // most (4096 ran slower at n = 2e6: 36 against 30 us)
    const int64_t waves = std::max<int64_t>(1, std::min<int64_t>({(int64_t)max_partials - 4, (int64_t)1024,
                                                                    ceil_div(n, kGram1MinRows)}));
    const int64_t rpw = ceil_div(ceil_div(n, waves), 64) * 64;
    const int64_t nw = ceil_div(n, rpw);
    const int64_t grid = ceil_div(nw, 4);
    if (bx == 4)
      hipLaunchKernelGGL((k_gram1<XT, YT, 4>), dim3((unsigned)grid), dim3(256), 0, s, n, X, Y, rpw,
                         partial, when);
    else if (bx == 8)
      hipLaunchKernelGGL((k_gram1<XT, YT, 8>), dim3((unsigned)grid), dim3(256), 0, s, n, X, Y, rpw,
                         partial, when);
    else
      hipLaunchKernelGGL((k_gram1_10<XT, YT>), dim3((unsigned)grid), dim3(256), 0, s, n, X, Y,
                         rpw, partial, when);
    check_launch("k_gram1");
    return (int)(grid * 4);
  }
  if (bx == 10 && ny == 10 && f32 && nblk >= 2) {
    // 64 padded columns (5 1/3 blocks) per one-wave workgroup, grid and row
    // chunks as for 8-wide blocks below
    const int gy = (nblk * 12 + 63) / 64;
    int64_t gx = std::min<int64_t>(kGramMaxChunks, ceil_div(kGramWaveTarget, gy));
    const bool small = ceil_div(n, 256) < gx;
    constexpr int U = kGram10U;
    gx = std::max<int64_t>(1, std::min<int64_t>(gx, ceil_div(n, small ? kGramSmallChunk : 256)));
    gx = std::min<int64_t>(gx, std::max(1, max_partials));
    const int64_t chunk = ceil_div(ceil_div(n, gx), 4 * U) * (4 * U);
    gx = ceil_div(n, chunk);
    const int64_t grid = ceil_div(gx, 8) * 8 * gy;
    hipLaunchKernelGGL((k_gram_mfma10<YT, U>), dim3((unsigned)grid), dim3(64), 0, s, n,
                       (const float *)X, nblk, xstride, Y, chunk, (int)gx, gy, partial, when);
    check_launch("k_gram_mfma10");
    return (int)gx;
  }
  if (bx == 8 && ny == 8 && f32 && std::is_same<YT, double>::value && nblk >= 2) {
    // 64 basis columns per one-wave workgroup; about 6k workgroups in all, so
    // that the whole grid is resident at once (measured on MI355X at n = 2e6:
    // 45, 90 and 181 blocks run fastest with 1024, 512 and 256 row chunks,
    // 5.1-5.3 TB/s; 20 blocks with 2048 chunks, 4.8 TB/s against 3.6 with
    // 1024)
    constexpr int CG = 1, WPG = kGramWaves;
    const int gy = (M + 64 * CG - 1) / (64 * CG);
    int64_t gx = std::min<int64_t>(kGramMaxChunks, ceil_div(kGramWaveTarget, gy));
    // short row counts: shorter row chunks with more rows in flight, so each
    // wave takes a few load rounds instead of dozens
    const bool small = ceil_div(n, 256) < gx;
    const int U = small ? kGramSmallU : 2;
    gx = std::max<int64_t>(1, std::min<int64_t>(gx, ceil_div(n, small ? kGramSmallChunk : 256)));
    gx = std::min<int64_t>(gx, std::max(1, max_partials));
    int64_t chunk = ceil_div(ceil_div(n, gx), 4 * U) * (4 * U);
    gx = ceil_div(n, chunk);
    const int64_t grid = ceil_div(gx, 8) * 8 * ceil_div(gy, WPG);
    if (small)
      hipLaunchKernelGGL((k_gram_mfma8<CG, kGramSmallU, WPG>), dim3((unsigned)grid),
                         dim3(64 * WPG), 0, s, n, (const float *)X, M, xstride,
                         (const double *)Y, chunk, (int)gx, gy, partial, when);
    else
      hipLaunchKernelGGL((k_gram_mfma8<CG, 2, WPG>), dim3((unsigned)grid), dim3(64 * WPG), 0, s,
                         n, (const float *)X, M, xstride, (const double *)Y, chunk, (int)gx, gy,
                         partial, when);
    check_launch("k_gram_mfma8");
    return (int)gx;
  }
  if (ny == bx) {
    switch (bx) {
      case 4: return gram_valu<XT, YT, 4, f32 ? 4 : 2>(n, X, bx, nblk, xstride, Y, partial, max_partials, when, s);
      case 8: return gram_valu<XT, YT, 8, f32 ? 4 : 2>(n, X, bx, nblk, xstride, Y, partial, max_partials, when, s);
      case 10: return gram_valu<XT, YT, 10, 2>(n, X, bx, nblk, xstride, Y, partial, max_partials, when, s);
      case 16: return gram_valu<XT, YT, 16, 2>(n, X, bx, nblk, xstride, Y, partial, max_partials, when, s);
      default: break;
    }
  }
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

constexpr int kUpdRPL = 2;  // rows per lane of k_update_v (256-row stride)
// Workgroups of k_update_v when it also leaves Gram partials (one per
// workgroup): beyond this many row tiles the workgroups stride over them, so
// the partials stay within the caller's buffer at any n
constexpr int64_t kUpdMaxGramParts = 16384;
inline int64_t update_tiles(int64_t n) { return ceil_div(n, 256 * kUpdRPL); }
inline int64_t update_gram_parts(int64_t n) {
  return std::min<int64_t>(update_tiles(n), kUpdMaxGramParts);
}
// the wave-split kernel k_update_w8 (short grids, many blocks); its Gram
// partials are one per 64 rows
inline bool update_split(int64_t n, int nblk, int ny) {
  return update_tiles(n) < 512 && nblk >= 16 && ny <= 8;
}
inline int64_t update_parts(int64_t n, int nblk, int ny) {
  return update_split(n, nblk, ny) ? ceil_div(n, 64) : update_gram_parts(n);
}

template <typename XT, typename YIT, typename YOT, int B, int NY = B>
void update_valu(int64_t n, const XT *X, int nblk, int64_t xstride, const double *C, double alpha,
                 const YIT *Yin, double beta, YOT *Yout, const int *when, double *gpart,
                 hipStream_t s) {
  const int64_t grid = gpart ? update_gram_parts(n) : update_tiles(n);
  // a short grid (few rows) with many blocks: split the blocks over waves
  // (no fused Gram then); a short grid with a few blocks: prefetch four at a
  // time
  if (update_split(n, nblk, NY)) {
    if constexpr (NY <= 8) {
      const dim3 grid8((unsigned)ceil_div(n, 64)), wg8(512);
      if (gpart)
        hipLaunchKernelGGL((k_update_w8<XT, YIT, YOT, B, NY, true>), grid8, wg8, 0, s, n,
                           X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart);
      else
        hipLaunchKernelGGL((k_update_w8<XT, YIT, YOT, B, NY, false>), grid8, wg8, 0, s, n,
                           X, nblk, xstride, C, alpha, Yin, beta, Yout, when, nullptr);
      check_launch("k_update_w8");
      return;
    }
  }
  const bool pf = grid < 512 && nblk >= 8;
#define BBL_UPDV(G, PF)                                                                        \
  hipLaunchKernelGGL((k_update_v<XT, YIT, YOT, B, NY, kUpdRPL, G, PF>), dim3((unsigned)grid),    \
                     dim3(256), 0, s, n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart)
  if (gpart && update_tiles(n) > grid) {  // capped grid: workgroups stride over the tiles
    hipLaunchKernelGGL((k_update_v<XT, YIT, YOT, B, NY, kUpdRPL, true, 1, true>),
                       dim3((unsigned)grid), dim3(256), 0, s, n, X, nblk, xstride, C, alpha, Yin,
                       beta, Yout, when, gpart);
  } else if (gpart) {
    if (pf) BBL_UPDV(true, 4);
    else BBL_UPDV(true, 1);
  } else {
    if (pf) BBL_UPDV(false, 4);
    else BBL_UPDV(false, 1);
  }
#undef BBL_UPDV
  check_launch("k_update_v");
}

// 16-wide blocks on FP64 matrix cores; the fused Gram needs (P + P/8 + 64)
// x 256 doubles of gpart (partials and the reduction's second stage).
template <typename XT, typename YIT, typename YOT>
int update_mfma16(int64_t n, const XT *X, int nblk, int64_t xstride, const double *C,
                  double alpha, const YIT *Yin, double beta, YOT *Yout, const int *when,
                  double *gpart, size_t gcap_doubles, hipStream_t s) {
  constexpr int U = kU16U;
  const int64_t P = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 16 * U), kU16Waves));
  if (gpart && (size_t)(P + P / 8 + 64) * 256 > gcap_doubles) gpart = nullptr;
  if (gpart)
    hipLaunchKernelGGL((k_update_mfma16<XT, YIT, YOT, U, true>), dim3((unsigned)P), dim3(64), 0, s,
                       n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart);
  else
    hipLaunchKernelGGL((k_update_mfma16<XT, YIT, YOT, U, false>), dim3((unsigned)P), dim3(64), 0,
                       s, n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, nullptr);
  check_launch("k_update_mfma16");
  return gpart ? (int)P : 0;
}

// gpart: where the Gram partials of Yout may go (nullptr: none wanted).
// Returns the number of partials written, 0 if this shape has no fused Gram.
template <typename XT, typename YIT, typename YOT>
int update_typed(int64_t n, const XT *X, int bx, int nblk, int64_t xstride, const double *C,
                 int ny, double alpha, const YIT *Yin, double beta, YOT *Yout, const int *when,
                 double *gpart, hipStream_t s) {
  const int M = nblk * bx;
  const int P = (int)update_parts(n, nblk, ny);
  if (bx == 8 && ny == 10) {  // Ritz vectors of b = 8 blocks, k = 10
    update_valu<XT, YIT, YOT, 8, 10>(n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart, s);
    return gpart ? P : 0;
  }
  if (ny == bx) {
    switch (bx) {
      case 4: update_valu<XT, YIT, YOT, 4>(n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart, s); return gpart ? P : 0;
      case 8: update_valu<XT, YIT, YOT, 8>(n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart, s); return gpart ? P : 0;
      case 10: update_valu<XT, YIT, YOT, 10>(n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart, s); return gpart ? P : 0;
      case 16: update_valu<XT, YIT, YOT, 16>(n, X, nblk, xstride, C, alpha, Yin, beta, Yout, when, gpart, s); return gpart ? P : 0;
      default: break;
    }
  }
  // four work-items per row: beyond kMaxLaunchItems of them the rows go in
  // several launches (row offsets into every block of X and into Y)
  const int64_t max_rows = kMaxLaunchItems / 4;
  for (int64_t r0 = 0; r0 < n; r0 += max_rows) {
    const int64_t nr = std::min<int64_t>(max_rows, n - r0);
    const unsigned grid = (unsigned)ceil_div(nr, 64);
    const XT *Xc = X + r0 * bx;
    const YIT *Yi = Yin ? Yin + r0 * ny : nullptr;
    YOT *Yo = Yout + r0 * ny;
    if (ny <= 16)
      hipLaunchKernelGGL((k_update<XT, YIT, YOT, 1>), dim3(grid), dim3(256), 0, s, nr, Xc, bx, M,
                         xstride, C, ny, alpha, Yi, beta, Yo, when);
    else
      hipLaunchKernelGGL((k_update<XT, YIT, YOT, 2>), dim3(grid), dim3(256), 0, s, nr, Xc, bx, M,
                         xstride, C, ny, alpha, Yi, beta, Yo, when);
    check_launch("k_update");
  }
  return 0;
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
  // stage 1 writes S partial sums behind the P partials (the caller's partial
  // buffer holds (P + S) * MN doubles), stage 2 sums them in order.  S ~ sqrt(P)
  // balances the serial length of the two stages.
  // (up to 64 partials: one stage, one launch)
  const int S_room = std::max(1, 8192 / ((MN + 255) / 256));
  const int S = P <= 64 ? 1
                        : std::max(1, std::min({P / 8, S_room, (int)std::ceil(std::sqrt((double)P))}));
  if (S > 1) {
    double *tmp = const_cast<double *>(partial) + (size_t)P * MN;
    hipLaunchKernelGGL(k_reduce1, dim3((MN + 255) / 256, S), dim3(256), 0, s, partial, P, MN, S,
                       tmp, when);
    check_launch("k_reduce1");
    hipLaunchKernelGGL(k_reduce, dim3((MN + 255) / 256), dim3(256), 0, s, tmp, S, MN, out, when);
  } else {
    hipLaunchKernelGGL(k_reduce, dim3((MN + 255) / 256), dim3(256), 0, s, partial, P, MN, out,
                       when);
  }
  check_launch("k_reduce");
}

void launch_reduce(const double *partial, int P, int M, int ny, double *out, hipStream_t s) {
  launch_reduce_when(partial, P, M, ny, out, nullptr, s);
}

int launch_update_gram_when(int64_t n, const void *X, int xdtype, int bx, int nblk,
                            int64_t xstride, const double *C, int ny, double alpha,
                            const void *Yin, int yindtype, double beta, void *Yout, int youtdtype,
                            double *gpart, size_t gcap_doubles, const int *when, hipStream_t s) {
  if (n <= 0) return 0;
  if (nblk <= 0) {  // empty product: Yout = beta * Yin
    BBL_REQUIRE(false, "update: empty X");
  }
  const bool xf = xdtype == BBL_F32, yif = yindtype == BBL_F32, yof = youtdtype == BBL_F32;
  if (bx == 16 && ny == 16 && aligned16(X) && aligned16(C) && aligned16(Yout) &&
      (beta == 0.0 || aligned16(Yin))) {
#define BBL_U16(XT, YIT, YOT)                                                                 \
  return update_mfma16(n, (const XT *)X, nblk, xstride, C, alpha, (const YIT *)Yin, beta,     \
                       (YOT *)Yout, when, gpart, gcap_doubles, s)
    if (xf && yif && yof) BBL_U16(float, float, float);
    else if (xf && yif && !yof) BBL_U16(float, float, double);
    else if (xf && !yif && yof) BBL_U16(float, double, float);
    else if (xf && !yif && !yof) BBL_U16(float, double, double);
    else if (!xf && yif && yof) BBL_U16(double, float, float);
    else if (!xf && yif && !yof) BBL_U16(double, float, double);
    else if (!xf && !yif && yof) BBL_U16(double, double, float);
    else BBL_U16(double, double, double);
#undef BBL_U16
  }
  // room for the partials and the reduction's stage-1 sums behind them
  const int64_t P = update_parts(n, nblk, ny);
  if (gpart && (size_t)(P + P / 8 + 64) * ny * ny > gcap_doubles) gpart = nullptr;
#define BBL_UPD(XT, YIT, YOT)                                                                 \
  return update_typed(n, (const XT *)X, bx, nblk, xstride, C, ny, alpha, (const YIT *)Yin,    \
                      beta, (YOT *)Yout, when, gpart, s)
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

void launch_update_when(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                        const double *C, int ny, double alpha, const void *Yin, int yindtype,
                        double beta, void *Yout, int youtdtype, const int *when,
                        hipStream_t s) {
  (void)launch_update_gram_when(n, X, xdtype, bx, nblk, xstride, C, ny, alpha, Yin, yindtype,
                                beta, Yout, youtdtype, nullptr, 0, when, s);
}

void launch_update(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                   const double *C, int ny, double alpha, const void *Yin, int yindtype,
                   double beta, void *Yout, int youtdtype, hipStream_t s) {
  launch_update_when(n, X, xdtype, bx, nblk, xstride, C, ny, alpha, Yin, yindtype, beta, Yout,
                     youtdtype, nullptr, s);
}

__global__ void k_store_int(int *p, int v) {
  if (threadIdx.x == 0) *p = v;
}

void launch_store_int(int *p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_store_int, dim3(1), dim3(64), 0, s, p, v);
  check_launch("k_store_int");
}

__global__ void k_copy_pair(double *dd, const double *ds, int *id, const int *is) {
  if (threadIdx.x == 0) {
    *dd = *ds;
    *id = *is;
  }
}

void launch_copy_pair(double *dd, const double *ds, int *id, const int *is, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_pair, dim3(1), dim3(64), 0, s, dd, ds, id, is);
  check_launch("k_copy_pair");
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
