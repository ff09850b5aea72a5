// CSR block SpMM  W = H V  (w_{a,i} = sum_j H_ij v_{a,j}; Methods, "Block
// Lanczos algorithm").  The block index a is innermost, as in the paper, so
// each matrix element (value + column) is streamed from HBM once per block of
// vectors; on the GPU the loop over a lives in registers of one lane.
//
// Mapping: LPR lanes of a 64-wide wavefront share one row; each lane takes
// every LPR-th element of the row (coalesced reads of col/val), gathers the
// whole row of V for that column with vector loads, and accumulates nvec
// partial sums; a butterfly over the LPR lanes finishes the row.  Rows are
// independent, no atomics, so results are bitwise reproducible.
#include <type_traits>

#include "common.h"

namespace bbl {
namespace {

template <typename T, int B>
struct RowIO {
  // loads B consecutive elements starting at p (p aligned to sizeof(T)*B's
  // largest power-of-two divisor up to 16 bytes)
  __device__ __forceinline__ static void load(const T *__restrict__ p, T (&v)[B]) {
    constexpr int bytes = (int)sizeof(T) * B;
    if constexpr (bytes % 16 == 0) {
      constexpr int nv = bytes / 16;
      const uint4 *q = reinterpret_cast<const uint4 *>(p);
      uint4 tmp[nv];
#pragma unroll
      for (int i = 0; i < nv; ++i) tmp[i] = q[i];
      __builtin_memcpy(v, tmp, bytes);
    } else if constexpr (bytes % 8 == 0) {
      constexpr int nv = bytes / 8;
      const uint2 *q = reinterpret_cast<const uint2 *>(p);
      uint2 tmp[nv];
#pragma unroll
      for (int i = 0; i < nv; ++i) tmp[i] = q[i];
      __builtin_memcpy(v, tmp, bytes);
    } else {
#pragma unroll
      for (int i = 0; i < B; ++i) v[i] = p[i];
    }
  }
};

template <typename T>
__device__ __forceinline__ T ldg_stream(const T *p) {
  return *p;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w runs on
// XCD w % 8), each XCD with its own L2.  The launch pads the grid to a
// multiple of 8 and this remap hands XCD x the contiguous row range
// [x G/8, (x+1) G/8) of blocks, so the workgroups resident on one XCD at a
// time cover a few neighbouring sectors and their V-row gathers share that
// XCD's L2 instead of every XCD caching every sector.
__device__ __forceinline__ int64_t xcd_block(int64_t w) {
  const int64_t per = gridDim.x / kXcds;
  return (w % kXcds) * per + w / kXcds;
}

// four consecutive values from a 16-byte aligned (float) / 32-byte aligned
// (double) address
template <typename T>
struct Quad {
  T v[4];
};
template <typename T>
__device__ __forceinline__ Quad<T> load_quad(const T *__restrict__ p) {
  Quad<T> q;
  if constexpr (sizeof(T) == 4) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    __builtin_memcpy(q.v, &u, 16);
  } else {
    const uint4 *w = reinterpret_cast<const uint4 *>(p);
    const uint4 u0 = w[0], u1 = w[1];
    __builtin_memcpy(q.v, &u0, 16);
    __builtin_memcpy(q.v + 2, &u1, 16);
  }
  return q;
}

template <typename VT, typename XT, typename AT, typename YT, int B, int LPR>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int64_t *__restrict__ rp,
                                              const int32_t *__restrict__ col,
                                              const VT *__restrict__ val,
                                              const XT *__restrict__ X, YT *__restrict__ Y) {
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int64_t wave_id = xcd_block(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int64_t row = wave_id * RPW + lane / LPR;
  AT acc[B];
#pragma unroll
  for (int a = 0; a < B; ++a) acc[a] = AT(0);
  if (row < n) {
    const int64_t p0 = rp[row], p1 = rp[row + 1];
    int64_t p = p0 + sub;
    // four independent gathers in flight per lane
    constexpr int UNR = 4;
    for (; p + (UNR - 1) * LPR < p1; p += UNR * LPR) {
      int c[UNR];
      AT h[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        c[u] = ldg_stream(col + p + u * LPR);
        h[u] = (AT)ldg_stream(val + p + u * LPR);
      }
      XT x[UNR][B];
#pragma unroll
      for (int u = 0; u < UNR; ++u) RowIO<XT, B>::load(X + (int64_t)c[u] * B, x[u]);
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int a = 0; a < B; ++a) acc[a] = fma(h[u], (AT)x[u][a], acc[a]);
    }
    for (; p < p1; p += LPR) {
      const int c0 = ldg_stream(col + p);
      const AT h0 = (AT)ldg_stream(val + p);
      XT x0[B];
      RowIO<XT, B>::load(X + (int64_t)c0 * B, x0);
#pragma unroll
      for (int a = 0; a < B; ++a) acc[a] = fma(h0, (AT)x0[a], acc[a]);
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < B; ++a) acc[a] += __shfl_xor(acc[a], off, LPR);
  }
  if (row < n) {
    // lane `sub` stores column `sub` (coalesced), looping for B > LPR
#pragma unroll
    for (int a0 = 0; a0 < B; a0 += LPR) {
      AT v = acc[0];
#pragma unroll
      for (int a = 1; a < B; ++a)
        if (a == a0 + sub) v = acc[a];
      if (a0 + sub < B) Y[row * B + a0 + sub] = (YT)v;
    }
  }
}

// Generic width (runtime nvec <= 32), used for block sizes without a
// dedicated instantiation.
template <typename VT, typename XT, typename AT, typename YT, int LPR>
__global__ __launch_bounds__(256) void k_spmm_generic(int64_t n, const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      const VT *__restrict__ val,
                                                      const XT *__restrict__ X,
                                                      YT *__restrict__ Y, int nvec) {
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int64_t wave_id = xcd_block(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const int64_t row = wave_id * RPW + lane / LPR;
  AT acc[kMaxBlock];
#pragma unroll
  for (int a = 0; a < kMaxBlock; ++a) acc[a] = AT(0);
  if (row < n) {
    const int64_t p0 = rp[row], p1 = rp[row + 1];
    for (int64_t p = p0 + sub; p < p1; p += LPR) {
      const int c = ldg_stream(col + p);
      const AT h = (AT)ldg_stream(val + p);
      const XT *x = X + (int64_t)c * nvec;
#pragma unroll
      for (int a = 0; a < kMaxBlock; ++a)
        if (a < nvec) acc[a] = fma(h, (AT)x[a], acc[a]);
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) acc[a] += __shfl_xor(acc[a], off, LPR);
  }
  if (row < n && sub == 0) {
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a)
      if (a < nvec) Y[row * nvec + a] = (YT)acc[a];
  }
}

// The same residual for a compile-time vector count NV: each gather reads a
// row of X with 16-byte loads, and workgroup w takes a contiguous run of rows
// (XCD-aware order, so the XCD's L2 serves neighbouring rows' gathers).
template <typename VT, int LPR, int NV>
__global__ __launch_bounds__(256) void k_residual_t(int64_t n, const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col,
                                                    const VT *__restrict__ val,
                                                    const double *__restrict__ X,
                                                    const double *__restrict__ theta,
                                                    int64_t chunk, double *__restrict__ partial) {
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int wave = threadIdx.x / kWave;
  __shared__ double red[4][NV];
  double sq[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) sq[a] = 0.0;
  const int64_t w = xcd_block(blockIdx.x);
  const int64_t r0 = w * chunk, r1 = min(n, r0 + chunk);
  for (int64_t base = r0 + (int64_t)wave * RPW; base < r1; base += 4 * RPW) {
    const int64_t row = base + lane / LPR;
    double acc[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) acc[a] = 0.0;
    if (row < r1) {
      // U entries per lane in flight: their index and value loads, then their
      // gathers (past the row's end a lane reloads its first entry of the
      // step and drops the product)
      constexpr int U = NV <= 4 ? 4 : NV <= 8 ? 3 : 2;
      const int64_t q1 = rp[row + 1];
      for (int64_t p = rp[row] + sub; p < q1; p += U * LPR) {
        double h[U];
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t pu = p + u * LPR < q1 ? p + u * LPR : p;
          h[u] = (double)val[pu];
          c[u] = col[pu];
        }
        double x[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) RowIO<double, NV>::load(X + (int64_t)c[u] * NV, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = p + u * LPR < q1;
#pragma unroll
          for (int a = 0; a < NV; ++a) acc[a] = fma(h[u], ok ? x[u][a] : 0.0, acc[a]);
        }
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int a = 0; a < NV; ++a) acc[a] += __shfl_xor(acc[a], off, LPR);
    }
    if (row < r1 && sub == 0) {
      double xr[NV];
      RowIO<double, NV>::load(X + row * NV, xr);
#pragma unroll
      for (int a = 0; a < NV; ++a) {
        const double r = acc[a] - theta[a] * xr[a];
        sq[a] = fma(r, r, sq[a]);
      }
    }
  }
#pragma unroll
  for (int off = LPR; off < kWave; off <<= 1) {
#pragma unroll
    for (int a = 0; a < NV; ++a) sq[a] += __shfl_xor(sq[a], off, kWave);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) red[wave][a] = sq[a];
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    const double v = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                     (red[2][threadIdx.x] + red[3][threadIdx.x]);
    partial[w * NV + threadIdx.x] = v;
  }
}

// Explicit FP64 residual: per workgroup g, partial[g][c] = sum over its rows of
// ((H X)_{r,c} - theta_c X_{r,c})^2.  Grid-stride over rows, fixed order.
template <typename VT, int LPR>
__global__ __launch_bounds__(256) void k_residual(int64_t n, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const VT *__restrict__ val,
                                                  const double *__restrict__ X, int nvec,
                                                  const double *__restrict__ theta,
                                                  double *__restrict__ partial) {
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int wave = threadIdx.x / kWave;
  __shared__ double red[4][kMaxBlock];
  double sq[kMaxBlock];
#pragma unroll
  for (int a = 0; a < kMaxBlock; ++a) sq[a] = 0.0;
  const int64_t rows_per_wg = (int64_t)RPW * (blockDim.x / kWave);
  for (int64_t base = (int64_t)blockIdx.x * rows_per_wg; base < n;
       base += (int64_t)gridDim.x * rows_per_wg) {
    const int64_t row = base + (int64_t)wave * RPW + lane / LPR;
    double acc[kMaxBlock];
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) acc[a] = 0.0;
    if (row < n) {
      for (int64_t p = rp[row] + sub; p < rp[row + 1]; p += LPR) {
        const int c = col[p];
        const double h = (double)val[p];
        const double *x = X + (int64_t)c * nvec;
#pragma unroll
        for (int a = 0; a < kMaxBlock; ++a)
          if (a < nvec) acc[a] = fma(h, x[a], acc[a]);
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int a = 0; a < kMaxBlock; ++a) acc[a] += __shfl_xor(acc[a], off, LPR);
    }
    if (row < n && sub == 0) {
#pragma unroll
      for (int a = 0; a < kMaxBlock; ++a) {
        if (a < nvec) {
          const double r = acc[a] - theta[a] * X[row * nvec + a];
          sq[a] = fma(r, r, sq[a]);
        }
      }
    }
  }
  // reduce sq over the lanes holding rows (sub == 0 lanes), then over waves
#pragma unroll
  for (int off = LPR; off < kWave; off <<= 1) {
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) sq[a] += __shfl_xor(sq[a], off, kWave);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) red[wave][a] = sq[a];
  }
  __syncthreads();
  if (threadIdx.x < nvec) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[w][threadIdx.x];
    partial[(int64_t)blockIdx.x * nvec + threadIdx.x] = s;
  }
}

// Lanes per row.  Measured on MI355X (n = 2e6, ~200 nnz/row, b = 8 FP32):
// 16 lanes per row with four gathers in flight per lane was the fastest
// layout; the kernel is bound by the random V-row gathers, not by the CSR
// stream (which alone reads at ~5.9 TB/s).
int pick_lpr(const bbl_csr &H) {
  const double z = H.n > 0 ? (double)H.nnz / (double)H.n : 0.0;
  return z < 400.0 ? 16 : 32;
}

template <typename VT, typename XT, typename AT, typename YT, int LPR>
void spmm_dispatch_b(const bbl_csr &H, const XT *X, YT *Y, int nvec, hipStream_t s) {
  const int rows_per_wg = (256 / kWave) * (kWave / LPR);
  const VT *val = static_cast<const VT *>(H.val);
  // LPR work-items per row: beyond kMaxLaunchItems of them the rows go in
  // several launches (row_ptr and Y offset; columns stay global)
  const int64_t max_rows = kMaxLaunchItems / 256 / kXcds * kXcds * rows_per_wg;
  for (int64_t r0 = 0; r0 < H.n; r0 += max_rows) {
    const int64_t nr = std::min<int64_t>(max_rows, H.n - r0);
    const int64_t grid = ceil_div(ceil_div(nr, rows_per_wg), kXcds) * kXcds;
    const int64_t *rp = H.row_ptr + r0;
    YT *Yc = Y + r0 * nvec;
#define BBL_SPMM_CASE(BV)                                                                      \
  case BV:                                                                                     \
    hipLaunchKernelGGL((k_spmm<VT, XT, AT, YT, BV, LPR>), dim3(grid), dim3(256), 0, s, nr, rp, \
                       H.col, val, X, Yc);                                                     \
    break;
    switch (nvec) {
      BBL_SPMM_CASE(1)
      BBL_SPMM_CASE(2)
      BBL_SPMM_CASE(4)
      BBL_SPMM_CASE(8)
      BBL_SPMM_CASE(10)
      BBL_SPMM_CASE(12)
      BBL_SPMM_CASE(16)
      BBL_SPMM_CASE(32)
      default:
        hipLaunchKernelGGL((k_spmm_generic<VT, XT, AT, YT, LPR>), dim3(grid), dim3(256), 0, s, nr,
                           rp, H.col, val, X, Yc, nvec);
    }
#undef BBL_SPMM_CASE
    check_launch("k_spmm");
  }
}

template <typename VT, typename XT, typename AT, typename YT>
void spmm_dispatch(const bbl_csr &H, const XT *X, YT *Y, int nvec, hipStream_t s) {
  switch (pick_lpr(H)) {
    case 16: spmm_dispatch_b<VT, XT, AT, YT, 16>(H, X, Y, nvec, s); break;
    case 32: spmm_dispatch_b<VT, XT, AT, YT, 32>(H, X, Y, nvec, s); break;
    default: spmm_dispatch_b<VT, XT, AT, YT, 64>(H, X, Y, nvec, s); break;
  }
}

// ------------------------------------------------------------ planned SpMM
// Prepared form of a matrix whose rows come in aligned groups of G rows
// (bbl_csr.block_rows).  For every group the plan names up to four column
// blocks -- its own and the partner blocks holding most of its other entries
// -- and reorders each row: entries inside those blocks first, stored as an
// LDS row index slot*G + (col - block start), then the others with their
// global column.  The fused kernel stages the blocks' rows of V in LDS once
// per group and, per row, issues the global gathers of the remote entries
// before it walks the local ones through LDS, so the long-latency gathers
// overlap the LDS work.

constexpr int kPlanHash = 1024;



// blocks[g][0] = g; blocks[g][1..width) = the other column blocks with the
// most entries in group g, busiest first (ties to the smaller block id), -1
// when fewer exist
__global__ __launch_bounds__(256) void k_plan_blocks(int64_t n, int64_t G, int width,
                                                     const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t *__restrict__ blocks) {
  __shared__ int keys[kPlanHash];
  __shared__ int cnts[kPlanHash];
  const int64_t g = blockIdx.x;
  const int64_t r0 = g * G, r1 = min(n, r0 + G);
  for (int i = threadIdx.x; i < kPlanHash; i += blockDim.x) {
    keys[i] = -1;
    cnts[i] = 0;
  }
  __syncthreads();
  const int64_t p0 = rp[r0], p1 = rp[r1];
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int b = (int)((int64_t)col[p] / G);
    if (b == (int)g) continue;
    unsigned h = ((unsigned)b * 2654435761u) >> 22;
    for (int probe = 0; probe < kPlanHash; ++probe) {
      const int k = atomicCAS(&keys[h], -1, b);
      if (k == -1 || k == b) {
        atomicAdd(&cnts[h], 1);
        break;
      }
      h = (h + 1) & (kPlanHash - 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    blocks[g * width] = (int32_t)g;
    for (int sl = 1; sl < width; ++sl) {
      int best = -1, bi = -1, bc = 0;
      for (int i = 0; i < kPlanHash; ++i) {
        const int k = keys[i], c = cnts[i];
        if (k < 0 || c <= 0) continue;
        if (c > bc || (c == bc && k < best)) {
          bc = c;
          best = k;
          bi = i;
        }
      }
      if (bi >= 0) cnts[bi] = 0;
      blocks[g * width + sl] = best;
    }
  }
}

// Reorders every row (one wave per row), each kind in the original order:
// entries in a set-A block (blocks[g][0..slots)) first, as slot*G + offset;
// then entries in a set-B block (blocks[g][slots..width), present when width
// = 2 slots) and then the rest, both with their global column in col2.
// n_local = count of the first kind.  lcol (if present) holds the LDS index
// of set-A and set-B entries within their set (slot*G + offset); rdesc (if
// present) the row's {first entry, first set-B entry, first remote entry,
// end} as offsets from its group's first entry rounded down to a multiple of
// 8; bcount[2 row + 1] (if present) its number of set-B entries.
template <typename VT>
__global__ __launch_bounds__(256) void k_plan_rows(int64_t n, int64_t G, int slots, int width,
                                                   const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const VT *__restrict__ val,
                                                   const int32_t *__restrict__ blocks,
                                                   int32_t *__restrict__ n_local,
                                                   int32_t *__restrict__ col2,
                                                   VT *__restrict__ val2,
                                                   uint16_t *__restrict__ lcol,
                                                   int32_t *__restrict__ rdesc,
                                                   int32_t *__restrict__ bcount) {
  // one wave per row, uniform per wave; the grid strides over the rows
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n;
       row += (int64_t)gridDim.x * 4) {
    const int lane = threadIdx.x & 63;
    const int64_t g = row / G;
    int64_t base[2 * kPlanMaxSlots];
#pragma unroll
    for (int k = 0; k < 2 * kPlanMaxSlots; ++k) {
      const int b = k < width ? blocks[g * width + k] : -1;
      base[k] = b >= 0 ? (int64_t)b * G : -((int64_t)1 << 62);
    }
    // kind (0: set A, 1: set B, 2: remote) and LDS index within the set
    auto classify = [&](int32_t c, int &loc) {
      int kind = 2;
      loc = -1;
#pragma unroll
      for (int k = 2 * kPlanMaxSlots - 1; k >= 0; --k) {
        const int64_t o = (int64_t)c - base[k];
        if (o >= 0 && o < G) {
          kind = k < slots ? 0 : 1;
          loc = (int)((k < slots ? k : k - slots) * G + o);
        }
      }
      return kind;
    };
    const int64_t p0 = rp[row], p1 = rp[row + 1];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int na = 0, nb = 0;
    for (int64_t p = p0 + lane; p - lane < p1; p += 64) {
      int loc;
      const int kind = p < p1 ? classify(col[p], loc) : 3;
      na += __popcll(__ballot(kind == 0));
      nb += __popcll(__ballot(kind == 1));
    }
    int ia = 0, ib = 0, ir = 0;
    for (int64_t p = p0 + lane; p - lane < p1; p += 64) {
      const bool in = p < p1;
      const int32_t c = in ? col[p] : 0;
      int loc = -1;
      const int kind = in ? classify(c, loc) : 3;
      const uint64_t ma = __ballot(kind == 0), mb = __ballot(kind == 1), mr = __ballot(kind == 2);
      int64_t q = -1;
      if (kind == 0) q = p0 + ia + __popcll(ma & below);
      else if (kind == 1) q = p0 + na + ib + __popcll(mb & below);
      else if (kind == 2) q = p0 + na + nb + ir + __popcll(mr & below);
      if (q >= 0) {
        col2[q] = kind == 0 ? loc : c;
        val2[q] = val[p];
        if (lcol && kind < 2) lcol[q] = (uint16_t)loc;
      }
      ia += __popcll(ma);
      ib += __popcll(mb);
      ir += __popcll(mr);
    }
    if (lane == 0) {
      n_local[row] = na;
      if (bcount) bcount[2 * row + 1] = nb;
      if (rdesc) {
        const int64_t gb = rp[g * G] & ~(int64_t)7;
        const int4 d = make_int4((int)(p0 - gb), (int)(p0 + na - gb), (int)(p0 + na + nb - gb),
                                 (int)(p1 - gb));
        *reinterpret_cast<int4 *>(rdesc + 4 * row) = d;
      }
    }
  }
}

// Dense copies of the set-A and set-B entries, rows in order, for the first
// and second passes, and the list of rows with entries outside both sets,
// for the third.  (See the kernels' own comments.)
// k_plan_bgroup (one workgroup per group): arow[2 r] / brow[2 r] = set-A /
// set-B entries of the group's rows before r, agroup[g + 1] / bgroup[g + 1] =
// the group's totals.  k_plan_gscan (one workgroup): agroup[g] / bgroup[g] =
// first copy entry of group g.  k_plan_bfill (one wave per row): copies the
// row's LDS indices and values of both sets and leaves arow[r] / brow[r] =
// {first, end} relative to agroup[g] / bgroup[g] rounded down to 8.
// Exclusive prefix over the group's rows of f(r) by one 256-thread
// workgroup: each thread takes a contiguous run of rows; returns the group
// total to every thread and calls put(r, prefix) for each row.
template <typename F, typename Put>
__device__ __forceinline__ int64_t group_scan(int64_t r0, int64_t r1, int64_t *part, F f,
                                              Put put) {
  const int t = threadIdx.x;
  const int64_t per = (r1 - r0 + 255) / 256;
  const int64_t a0 = r0 + t * per, a1 = min(r1, a0 + per);
  int64_t sum = 0;
  for (int64_t r = a0; r < a1; ++r) sum += f(r);
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = t > 0 ? part[t - 1] : 0;
  for (int64_t r = a0; r < a1; ++r) {
    const int64_t c = f(r);
    put(r, run);
    run += c;
  }
  const int64_t total = part[255];
  __syncthreads();
  return total;
}

// Also: rpos[r] = index of row r among the group's rows with entries outside
// both sets (-1 if it has none), rgroup[g + 1] = their number.
__global__ __launch_bounds__(256) void k_plan_bgroup(int64_t n, int64_t G,
                                                     const int32_t *__restrict__ rdesc,
                                                     const int32_t *__restrict__ n_local,
                                                     int32_t *__restrict__ arow,
                                                     int64_t *__restrict__ agroup,
                                                     int32_t *__restrict__ brow,
                                                     int64_t *__restrict__ bgroup,
                                                     int32_t *__restrict__ rpos,
                                                     int64_t *__restrict__ rgroup) {
  __shared__ int64_t part[256];
  const int64_t g = blockIdx.x;
  const int64_t r0 = g * G, r1 = min(n, r0 + G);
  const int64_t na = group_scan(
      r0, r1, part, [&](int64_t r) { return (int64_t)n_local[r]; },
      [&](int64_t r, int64_t pre) { arow[2 * r] = (int)pre; });
  const int64_t nb = group_scan(
      r0, r1, part, [&](int64_t r) { return (int64_t)brow[2 * r + 1]; },
      [&](int64_t r, int64_t pre) { brow[2 * r] = (int)pre; });
  auto has_rest = [&](int64_t r) { return (int64_t)(rdesc[4 * r + 3] > rdesc[4 * r + 2]); };
  const int64_t nrest = group_scan(r0, r1, part, has_rest, [&](int64_t r, int64_t pre) {
    rpos[r] = has_rest(r) ? (int)pre : -1;
  });
  if (threadIdx.x == 0) {
    agroup[g + 1] = na;
    bgroup[g + 1] = nb;
    rgroup[g + 1] = nrest;
    if (g == 0) agroup[0] = bgroup[0] = rgroup[0] = 0;
  }
}

__global__ __launch_bounds__(1024) void k_plan_gscan(int64_t *__restrict__ a, int64_t m) {
  // inclusive scan of a[1..m] in place
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (m + 1023) / 1024;
  const int64_t b0 = 1 + t * per, b1 = min(m + 1, b0 + per);
  int64_t sum = 0;
  for (int64_t i = b0; i < b1; ++i) sum += a[i];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = t > 0 ? part[t - 1] : 0;
  for (int64_t i = b0; i < b1; ++i) {
    run += a[i];
    a[i] = run;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_plan_bfill(int64_t n, int64_t G,
                                                    const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ n_local,
                                                    const uint16_t *__restrict__ lcol,
                                                    const VT *__restrict__ val2,
                                                    const int64_t *__restrict__ agroup,
                                                    int32_t *__restrict__ arow,
                                                    uint16_t *__restrict__ alcol,
                                                    VT *__restrict__ aval,
                                                    const int64_t *__restrict__ bgroup,
                                                    int32_t *__restrict__ brow,
                                                    uint16_t *__restrict__ blcol,
                                                    VT *__restrict__ bval,
                                                    const int32_t *__restrict__ rdesc,
                                                    const int32_t *__restrict__ rpos,
                                                    const int64_t *__restrict__ rgroup,
                                                    int4 *__restrict__ rlist) {
  // one wave per row, uniform per wave; the grid strides over the rows
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n;
       row += (int64_t)gridDim.x * 4) {
    const int lane = threadIdx.x & 63;
    const int64_t g = row / G;
    const int na = n_local[row];
    const int64_t asrc = rp[row], adst = agroup[g] + arow[2 * row];
    for (int i = lane; i < na; i += 64) {
      alcol[adst + i] = lcol[asrc + i];
      aval[adst + i] = val2[asrc + i];
    }
    const int64_t src = asrc + na;
    const int cnt = brow[2 * row + 1];
    const int64_t dst = bgroup[g] + brow[2 * row];
    for (int i = lane; i < cnt; i += 64) {
      blcol[dst + i] = lcol[src + i];
      bval[dst + i] = val2[src + i];
    }
    if (lane == 0) {
      const int64_t ga = agroup[g] & ~(int64_t)7;
      *reinterpret_cast<int2 *>(arow + 2 * row) = make_int2((int)(adst - ga), (int)(adst + na - ga));
      const int64_t gb = bgroup[g] & ~(int64_t)7;
      *reinterpret_cast<int2 *>(brow + 2 * row) = make_int2((int)(dst - gb), (int)(dst + cnt - gb));
      if (rpos[row] >= 0) {
        // {row, count, first entry (64-bit, low and high word)}
        const int64_t first = (rp[g * G] & ~(int64_t)7) + rdesc[4 * row + 2];
        rlist[rgroup[g] + rpos[row]] =
            make_int4((int)row, rdesc[4 * row + 3] - rdesc[4 * row + 2], (int)(uint32_t)first,
                      (int)(first >> 32));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Multi-set plan (groups whose entries spread over more column blocks than
// two sets of LDS slots hold, or more than 2^31 entries): the group's busiest
// nsets * slots blocks form nsets sets of `slots` blocks, staged in LDS one
// set after the other; every set has a dense copy of its entries (group by
// group, rows in order, 16-bit LDS index within the set and value), and the
// entries outside every set are kept compactly (global column and value) for
// the gather pass.  Built straight from H: nothing of the size of H beside
// the copies.  Layout of the copies (one region of 8 (nnz + 16) bytes):
// set values from the front of the value half, rest values from its back;
// set LDS indices packed from the front of the index half, rest columns
// from its back.

// Set of an entry of group g with column c: the position of its block among
// the group's blocks divided by slots, nsets for none.  loc receives the LDS
// row index within the set.
__device__ __forceinline__ int ms_classify(int32_t c, const int64_t *base, int width, int slots,
                                           int64_t G, int &loc) {
  int kind = width / slots;
  loc = 0;
  for (int k = width - 1; k >= 0; --k) {
    const int64_t o = (int64_t)c - base[k];
    if (o >= 0 && o < G) {
      kind = k / slots;
      loc = (int)((k % slots) * G + o);
    }
  }
  return kind;
}

constexpr int kMsMaxWidth = 16;  // blocks of all sets of a group
#ifndef BBL_MS_ROWS_PER_WAVE
#define BBL_MS_ROWS_PER_WAVE 16
#endif
constexpr int kMsRowsPerWave = BBL_MS_ROWS_PER_WAVE;  // rows per wave of the plan's count and fill

// Per row (one wave per row): entries per set into srow[(s n + row) 2 + 1],
// entries outside every set into rcnt[row].
__global__ __launch_bounds__(256) void k_ms_count(int64_t n, int64_t G, int slots, int width,
                                                  const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const int32_t *__restrict__ blocks,
                                                  int32_t *__restrict__ srow,
                                                  int32_t *__restrict__ rcnt) {
  // one wave per row, uniform per wave; each wave takes a run of rows, so
  // the group's block bases are loaded once per group it meets
  const int64_t nw = (int64_t)gridDim.x * 4, wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t rpw = (n + nw - 1) / nw, ra = wv * rpw, rb = min(n, ra + rpw);
  const int lane = threadIdx.x & 63;
  const int nsets = width / slots;
  int64_t gcur = -1;
  int64_t base[kMsMaxWidth];
  for (int64_t row = ra; row < rb; ++row) {
    const int64_t g = row / G;
    if (g != gcur) {
      gcur = g;
      for (int k = 0; k < width; ++k) {
        const int b = blocks[g * width + k];
        base[k] = b >= 0 ? (int64_t)b * G : -((int64_t)1 << 62);
      }
    }
    int cnt[kMsMaxWidth + 1] = {};
    const int64_t p0 = rp[row], p1 = rp[row + 1];
    for (int64_t p = p0 + lane; p - lane < p1; p += 64) {
      int loc;
      const int kind = p < p1 ? ms_classify(col[p], base, width, slots, G, loc) : -1;
      for (int s = 0; s <= nsets; ++s) cnt[s] += __popcll(__ballot(kind == s));
    }
    if (lane == 0) {
      for (int s = 0; s < nsets; ++s) srow[(s * n + row) * 2 + 1] = cnt[s];
      rcnt[row] = cnt[nsets];
    }
  }
}

// One workgroup per group: per set, the rows' offsets within the group's
// copy (srow[..].x) and the group's total (sgroup[s][g + 1]); for the rest,
// each row's offset among the group's rest entries (rpre), the group's rest
// total (rtot[g + 1]), and the position of every row that has rest entries
// among such rows (rpos, -1 if none) with their count (rgroup[g + 1]).
__global__ __launch_bounds__(256) void k_ms_group(int64_t n, int64_t G, int nsets, int64_t groups,
                                                  int32_t *__restrict__ srow,
                                                  int64_t *__restrict__ sgroup,
                                                  const int32_t *__restrict__ rcnt,
                                                  int32_t *__restrict__ rpre,
                                                  int64_t *__restrict__ rtot,
                                                  int32_t *__restrict__ rpos,
                                                  int64_t *__restrict__ rgroup) {
  __shared__ int64_t part[256];
  const int64_t g = blockIdx.x;
  const int64_t r0 = g * G, r1 = min(n, r0 + G);
  for (int s = 0; s < nsets; ++s) {
    int32_t *sr = srow + (int64_t)s * n * 2;
    const int64_t tot = group_scan(
        r0, r1, part, [&](int64_t r) { return (int64_t)sr[2 * r + 1]; },
        [&](int64_t r, int64_t pre) { sr[2 * r] = (int)pre; });
    if (threadIdx.x == 0) {
      sgroup[s * (groups + 1) + g + 1] = tot;
      if (g == 0) sgroup[s * (groups + 1)] = 0;
    }
  }
  const int64_t rt = group_scan(
      r0, r1, part, [&](int64_t r) { return (int64_t)rcnt[r]; },
      [&](int64_t r, int64_t pre) { rpre[r] = (int)pre; });
  const int64_t nr = group_scan(
      r0, r1, part, [&](int64_t r) { return (int64_t)(rcnt[r] > 0); },
      [&](int64_t r, int64_t pre) { rpos[r] = rcnt[r] > 0 ? (int)pre : -1; });
  if (threadIdx.x == 0) {
    rtot[g + 1] = rt;
    rgroup[g + 1] = nr;
    if (g == 0) rtot[0] = rgroup[0] = 0;
  }
}

// Per row (one wave per row): the entries into their set's copy or the rest
// arrays, each kind in the row's order; then srow[s][row] = {first, end}
// relative to the group's first copy entry rounded down to 8, and the row's
// rest list entry {row, count, first rest entry (low, high)}.
template <typename VT>
__global__ __launch_bounds__(256) void k_ms_fill(int64_t n, int64_t G, int slots, int width,
                                                 int64_t groups, const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col,
                                                 const VT *__restrict__ val,
                                                 const int32_t *__restrict__ blocks,
                                                 int32_t *__restrict__ srow,
                                                 const int64_t *__restrict__ sgroup,
                                                 uint16_t *__restrict__ slcol,
                                                 VT *__restrict__ sval,
                                                 const int32_t *__restrict__ rcnt,
                                                 const int32_t *__restrict__ rpre,
                                                 const int64_t *__restrict__ rtot,
                                                 const int32_t *__restrict__ rpos,
                                                 const int64_t *__restrict__ rgroup,
                                                 int32_t *__restrict__ rcol, VT *__restrict__ rval,
                                                 int4 *__restrict__ rlist) {
  // one wave per row, uniform per wave; each wave takes a run of rows, so
  // the group's block bases are loaded once per group it meets
  const int64_t nw = (int64_t)gridDim.x * 4, wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t rpw = (n + nw - 1) / nw, ra = wv * rpw, rb = min(n, ra + rpw);
  const int lane = threadIdx.x & 63;
  const int nsets = width / slots;
  int64_t gcur = -1;
  int64_t base[kMsMaxWidth];
  for (int64_t row = ra; row < rb; ++row) {
    const int64_t g = row / G;
    if (g != gcur) {
      gcur = g;
      for (int k = 0; k < width; ++k) {
        const int b = blocks[g * width + k];
        base[k] = b >= 0 ? (int64_t)b * G : -((int64_t)1 << 62);
      }
    }
    // the per-set destinations stay in registers: every loop over the sets
    // runs to kMsMaxWidth with a guard (a loop to the run-time set count
    // indexed them dynamically, which put them in scratch memory: the fill
    // took 346 against 121 ms on the n = 2e7 plan)
    int64_t dst[kMsMaxWidth + 1];
#pragma unroll
    for (int s = 0; s <= kMsMaxWidth; ++s)
      dst[s] = s < nsets ? sgroup[s * (groups + 1) + g] + srow[((int64_t)s * n + row) * 2]
                         : rtot[g] + rpre[row];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t p0 = rp[row], p1 = rp[row + 1];
    for (int64_t p = p0 + lane; p - lane < p1; p += 64) {
      const bool in = p < p1;
      const int32_t c = in ? col[p] : 0;
      const VT v = in ? val[p] : VT(0);
      int loc = 0;
      const int kind = in ? ms_classify(c, base, width, slots, G, loc) : -1;
      int64_t q = 0;  // this lane's destination in its kind's array
#pragma unroll
      for (int s = 0; s <= kMsMaxWidth; ++s) {
        if (s <= nsets) {
          const uint64_t m = __ballot(kind == s);
          if (kind == s) q = dst[s] + __popcll(m & below);
          dst[s] += __popcll(m);
        }
      }
      if (in) {
        if (kind < nsets) {
          slcol[q] = (uint16_t)loc;
          sval[q] = v;
        } else {
          rcol[q] = c;
          rval[q] = v;
        }
      }
    }
    if (lane == 0) {
      for (int s = 0; s < nsets; ++s) {
        int32_t *d = srow + ((int64_t)s * n + row) * 2;
        const int64_t gb = sgroup[s * (groups + 1) + g] & ~(int64_t)7;
        const int64_t first = sgroup[s * (groups + 1) + g] + d[0];
        d[0] = (int)(first - gb);
        d[1] = (int)(first + d[1] - gb);
      }
      if (rpos[row] >= 0) {
        const int64_t first = rtot[g] + rpre[row];
        rlist[rgroup[g] + rpos[row]] =
            make_int4((int)row, rcnt[row], (int)(uint32_t)first, (int)(first >> 32));
      }
    }
  }
}

template <typename VT, typename XT, typename AT, typename YT, int B, int LPR, bool LC16>
__global__ __launch_bounds__(1024) void k_spmm_planned(int64_t n, int64_t G, int slots, int width,
                                                       int parts,
                                                       const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ n_local,
                                                       const int32_t *__restrict__ col2,
                                                       const VT *__restrict__ val2,
                                                       const uint16_t *__restrict__ lcol,
                                                       const int32_t *__restrict__ blocks,
                                                       const XT *__restrict__ X,
                                                       YT *__restrict__ Y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XT *sX = reinterpret_cast<XT *>(smem_raw);
  // `parts` workgroups share a group (each stages its blocks, takes a slice of
  // its rows); they are consecutive in the XCD-aware order, so they run on one
  // XCD together and the group's partner data is read from HBM once per L2
  const int64_t L = xcd_block(blockIdx.x);
  const int64_t g = L / parts, part = L % parts;
  const int64_t gr0 = g * G;
  if (gr0 >= n) return;  // grid padding: the whole workgroup leaves
  const int64_t slice = (G + parts - 1) / parts;
  const int64_t r0 = gr0 + part * slice;
  const int64_t r1 = min(min(n, gr0 + G), r0 + slice);
  if (r0 >= r1) return;
  for (int k = 0; k < slots; ++k) {
    const int b = blocks[g * width + k];
    if (b < 0) continue;
    const int64_t b0 = (int64_t)b * G, b1 = min(n, b0 + G);
    constexpr int bytes = (int)sizeof(XT) * B;
    const unsigned char *src = reinterpret_cast<const unsigned char *>(X + b0 * B);
    unsigned char *dst = smem_raw + (size_t)k * G * bytes;
    const int64_t total = (b1 - b0) * bytes;
    if constexpr (bytes % 16 == 0) {
      for (int64_t i = threadIdx.x; i < total / 16; i += blockDim.x)
        reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
    } else if constexpr (bytes % 8 == 0) {
      for (int64_t i = threadIdx.x; i < total / 8; i += blockDim.x)
        reinterpret_cast<uint2 *>(dst)[i] = reinterpret_cast<const uint2 *>(src)[i];
    } else {
      for (int64_t i = threadIdx.x; i < total / 4; i += blockDim.x)
        reinterpret_cast<uint32_t *>(dst)[i] = reinterpret_cast<const uint32_t *>(src)[i];
    }
  }
  __syncthreads();
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  // Each lane takes four consecutive entries per chunk (one 16-byte load of
  // indices and one of values; chunks start at multiples of four entries, the
  // plan pads its arrays so the last load stays inside them).
  constexpr int CH = 4 * LPR;
  // the loop bound is uniform per wave, so every lane joins the butterfly
  for (int64_t base = r0 + (int64_t)wave * RPW; base < r1; base += (int64_t)nwaves * RPW) {
    const int64_t row = base + lane / LPR;
    AT acc[B];
#pragma unroll
    for (int a = 0; a < B; ++a) acc[a] = AT(0);
    if (row < r1) {
      const int64_t p0 = rp[row], p1 = rp[row + 1];
      const int64_t pl = p0 + n_local[row];
      int64_t qr = (pl & ~(int64_t)3) + 4 * sub;   // remote chunk cursor
      int64_t ql = (p0 & ~(int64_t)3) + 4 * sub;   // local chunk cursor
      while (qr < p1 || ql < pl) {
        // remote entries of this chunk: indices, values, then the gathers
        XT rx[4][B];
        AT rh[4];
        {
          int4 c4 = make_int4(0, 0, 0, 0);
          Quad<VT> v4;
#pragma unroll
          for (int e = 0; e < 4; ++e) v4.v[e] = VT(0);
          if (qr < p1) {
            c4 = *reinterpret_cast<const int4 *>(col2 + qr);
            v4 = load_quad(val2 + qr);
          }
          const int cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t pe = qr + e;
            const bool ok = pe >= pl && pe < p1;
            rh[e] = ok ? (AT)v4.v[e] : AT(0);
#pragma unroll
            for (int a = 0; a < B; ++a) rx[e][a] = XT(0);
            if (ok) RowIO<XT, B>::load(X + (int64_t)cc[e] * B, rx[e]);
          }
        }
        // local entries: LDS gathers while the remote ones are in flight
        if (ql < pl) {
          int cc[4];
          if constexpr (LC16) {  // four 16-bit LDS indices in one 8-byte load
            const uint2 c2 = *reinterpret_cast<const uint2 *>(lcol + ql);
            cc[0] = (int)(c2.x & 0xffffu);
            cc[1] = (int)(c2.x >> 16);
            cc[2] = (int)(c2.y & 0xffffu);
            cc[3] = (int)(c2.y >> 16);
          } else {
            const int4 c4 = *reinterpret_cast<const int4 *>(col2 + ql);
            cc[0] = c4.x;
            cc[1] = c4.y;
            cc[2] = c4.z;
            cc[3] = c4.w;
          }
          const Quad<VT> v4 = load_quad(val2 + ql);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t pe = ql + e;
            if (pe >= p0 && pe < pl) {
              XT lx[B];
              RowIO<XT, B>::load(sX + (int64_t)cc[e] * B, lx);
              const AT h = (AT)v4.v[e];
#pragma unroll
              for (int a = 0; a < B; ++a) acc[a] = fma(h, (AT)lx[a], acc[a]);
            }
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int a = 0; a < B; ++a) acc[a] = fma(rh[e], (AT)rx[e][a], acc[a]);
        qr += CH;
        ql += CH;
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int a = 0; a < B; ++a) acc[a] += __shfl_xor(acc[a], off, LPR);
    }
    if (row < r1) {
#pragma unroll
      for (int a0 = 0; a0 < B; a0 += LPR) {
        AT v = acc[0];
#pragma unroll
        for (int a = 1; a < B; ++a)
          if (a == a0 + sub) v = acc[a];
        if (a0 + sub < B) Y[row * B + a0 + sub] = (YT)v;
      }
    }
  }
}

// Three-pass planned SpMM for FP32 plans with 16-bit LDS indices and row
// descriptors.  The plan names two sets of column blocks per row group: set
// A (the group's own block and its busiest partners) and set B (the next
// busiest), and orders every row's entries: set A, set B, then the rest.
// Pass 1 stages set A in LDS and streams each row's set-A entries, writing
// the row sums; pass 2 stages set B, streams a dense copy of the set-B
// entries and adds its sums; pass 3 gathers the rows of V the few remaining
// entries need from global memory and adds theirs.  On sectored matrices the
// two sets hold nearly every entry, so rows of V are read from LDS rather
// than gathered one by one through the vector caches, and the pipelined
// passes carry no gather path.
//
// Passes 1 and 2 run the same software pipeline.  LPR lanes share a row and
// walk it in steps of LE * LPR entries (LE per lane, loaded 16 bytes at a
// time); the loads of the following step -- of the group's next row when
// this one ends -- are issued before this step's LDS reads and FMAs, so one
// step of the stream is always in flight behind the arithmetic.  Entries
// outside a lane's part of the row read an all-zero LDS row kept after the
// staged blocks, with a zero weight, so the LDS reads carry no branches.

// Sum over the 16 lanes of one DPP row (lanes 16r .. 16r + 15), every lane
// ending with the total, on the VALU: partners lane ^ 1 and lane ^ 2 (quad
// permutations), then 7 - i within eight lanes and 15 - i within sixteen
// (half mirror, mirror); each step adds sums over disjoint lane sets.  An
// xor butterfly through __shfl_xor is a ds_bpermute per value and step,
// which queues behind the LDS gathers of the product.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double x) {
  const unsigned long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// The partner's value in round `off` of a halving exchange over LPR lanes
// (16: off = 8, 4, 2, 1; 2: off = 1), on DPP: lane i ^ 8 (row rotation by
// 8), lane 7 - i within eight (half mirror; with lane pairs, whose lowest
// bit names the column half, i ^ 6 by a quad permutation and the half
// mirror), lane i ^ 2, lane i ^ 1.  Each partner differs from the lane in
// bit `off` of its index, in no higher bit, and (lane pairs) not in the
// lowest, so the rounds keep and send the same halves as an xor butterfly
// would, and afterwards every lane holds the sums over all LPR lanes (lane
// pairs: over those of its half) of the same components.
template <bool PAIR, typename T>
__device__ __forceinline__ T halving_partner(T x, int off) {
  if (off == 8) return dpp_f<0x128>(x);
  if (off == 4) return PAIR ? dpp_f<0x141>(dpp_f<0xB1>(x)) : dpp_f<0x141>(x);
  if (off == 2) return dpp_f<0x4E>(x);
  return dpp_f<0xB1>(x);
}
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f<0x141>(v);  // row_half_mirror
  v += dpp_f<0x140>(v);  // row_mirror
  return v;
}

// lanes per row and entries per lane and step: pass 1 takes ~90 % of each
// row's entries, pass 2 ~10 %
// T: the value and vector type (float, or double for float64 plans, whose
// rows of B doubles are staged as they are); double values and 64-byte rows
// (W: "wide") take fewer entries per lane in pass 2 and fewer LDS rows per
// product group, within the register budget of a 1024-thread workgroup
// (128 per lane).
template <bool P2>
constexpr int pipe_lpr() { return P2 ? 2 : 16; }
template <typename T, int B>
constexpr bool pipe_wide() { return sizeof(T) == 8 || sizeof(T) * B >= 64; }
template <bool P2, bool W = false>
constexpr int pipe_le() { return P2 ? (W ? 8 : 16) : 8; }
template <bool P2, bool W = false>
constexpr int pipe_lg() { return W ? (P2 ? 1 : 2) : (P2 ? 2 : 4); }
template <typename T>
__device__ __forceinline__ T pipe_fma(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return fmaf(a, b, c);
  else return fma(a, b, c);
}

// PAIR (16 float columns in one pass): the lanes of a row work in pairs on
// the same entries, the even lane on columns 0-7 of each staged row, the odd
// lane on 8-15, so a lane holds the sums and LDS rows of 8 columns (as at
// B = 8) while the entries are streamed once for all 16.
template <int B, bool P2, typename T = float, bool PAIR = false>
struct PipeStage {
  static constexpr int LPR = pipe_lpr<P2>();
  static constexpr int BL = PAIR ? B / 2 : B;          // columns per lane
  static constexpr int LPE = PAIR ? LPR / 2 : LPR;     // lanes per row with distinct entries
  static constexpr int NO = BL / LPE > 0 ? BL / LPE : 1;  // sums per lane after the reduction
  static constexpr int LE = pipe_le<P2, pipe_wide<T, BL>()>();
  uint4 lc[LE / 8];             // 16-bit LDS row indices
  T lv[LE];
  T yp[P2 ? NO : 1];            // the row's sums so far (pass 2)
  int llo, lhi;                 // valid entries e: llo <= e < lhi
};

// NO consecutive values from a sizeof(T) * NO-byte aligned address
template <int NO>
__device__ __forceinline__ void pipe_vload(const double *p, double (&v)[NO]) {
  if constexpr (NO % 2 == 0) {
#pragma unroll
    for (int i = 0; i < NO / 2; ++i) {
      const double2 y = reinterpret_cast<const double2 *>(p)[i];
      v[2 * i] = y.x, v[2 * i + 1] = y.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NO; ++i) v[i] = p[i];
  }
}
template <int NO>
__device__ __forceinline__ void pipe_vstore(double *p, const double (&v)[NO]) {
  if constexpr (NO % 2 == 0) {
#pragma unroll
    for (int i = 0; i < NO / 2; ++i)
      reinterpret_cast<double2 *>(p)[i] = make_double2(v[2 * i], v[2 * i + 1]);
  } else {
#pragma unroll
    for (int i = 0; i < NO; ++i) p[i] = v[i];
  }
}
template <int NO>
__device__ __forceinline__ void pipe_vload(const float *p, float (&v)[NO]) {
  if constexpr (NO == 4) {
    const float4 y = *reinterpret_cast<const float4 *>(p);
    v[0] = y.x, v[1] = y.y, v[2] = y.z, v[3] = y.w;
  } else if constexpr (NO == 2) {
    const float2 y = *reinterpret_cast<const float2 *>(p);
    v[0] = y.x, v[1] = y.y;
  } else {
#pragma unroll
    for (int i = 0; i < NO; ++i) v[i] = p[i];
  }
}
template <int NO>
__device__ __forceinline__ void pipe_vstore(float *p, const float (&v)[NO]) {
  if constexpr (NO == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (NO == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
  } else {
#pragma unroll
    for (int i = 0; i < NO; ++i) p[i] = v[i];
  }
}

// Loads the lane's share of one step: entries [ql, ql + LE) of a row whose
// entries in this pass are [p0, pl), and in pass 2 the row's sums so far.
// Positions are relative to a base that is a multiple of 8 and ql is a
// multiple of LE, so the loads are aligned; the plan pads its arrays by 16
// entries.  Every lane issues the same loads whether or not its entries exist
// (those without any read position 0 and are masked by the range), so the
// number of loads in flight is the same on every path.
template <int B, bool P2, typename T, bool PAIR>
__device__ __forceinline__ void pipe_load(PipeStage<B, P2, T, PAIR> &st,
                                          const uint16_t *__restrict__ lcol,
                                          const T *__restrict__ val, int ql, int p0, int pl,
                                          const T *yrow) {
  constexpr int LE = PipeStage<B, P2, T, PAIR>::LE;
  constexpr int PER = 16 / (int)sizeof(T);  // values per 16-byte load
  st.llo = p0 - ql;
  st.lhi = pl - ql;
  const int lq = st.lhi > 0 ? ql : 0;
#pragma unroll
  for (int i = 0; i < LE / 8; ++i) st.lc[i] = reinterpret_cast<const uint4 *>(lcol + lq)[i];
#pragma unroll
  for (int i = 0; i < LE / PER; ++i) {
    const uint4 a = reinterpret_cast<const uint4 *>(val + lq)[i];
    __builtin_memcpy(st.lv + PER * i, &a, 16);
  }
  if constexpr (P2) pipe_vload<PipeStage<B, P2, T, PAIR>::NO>(yrow, st.yp);
}

// Row loads from LDS.  With par = 1 (odd lanes of pass 1 at B = 8) the lane
// keeps its sums rotated by four components (v[a] holds component
// (a + 4) % 8): the first 16-byte half it reads is the row's second, so the
// lanes of one LDS read spread over twice as many bank positions.  The row
// reduction undoes it.
template <int B>
__device__ __forceinline__ void pipe_row(const double *p, int, double (&v)[B]) {
  RowIO<double, B>::load(p, v);
}
template <int B>
__device__ __forceinline__ void pipe_row(const float *p, int par, float (&v)[B]) {
  if constexpr (B == 8) {
    const float4 a = *reinterpret_cast<const float4 *>(p + 4 * par);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4 - 4 * par);
    __builtin_memcpy(v, &a, 16);
    __builtin_memcpy(v + 4, &b, 16);
  } else {
    RowIO<float, B>::load(p, v);
  }
}

template <int N>
__device__ __forceinline__ int pipe_lidx(const uint4 (&c)[N], int e) {
  const uint4 &q = c[e / 8];
  const int f = e % 8;
  const unsigned w = f < 2 ? q.x : f < 4 ? q.y : f < 6 ? q.z : q.w;
  return (int)((f & 1) ? (w >> 16) : (w & 0xffffu));
}

// A workgroup's copy of `slots` column blocks of V (B columns of rows `ld`
// floats apart) into LDS (slot k at k G rows of B), in pieces of 4, 8 or 16
// bytes, piece item = thread + 1024 j:
// issue() loads this thread's pieces J0 .. J0 + NJ - 1 into registers,
// commit() writes them; every load is in flight before the first write.
template <int B, typename T = float>
constexpr int stage_pieces() {
  constexpr int bytes = (int)sizeof(T) * B;
  constexpr int piece = bytes % 16 == 0 ? 16 : bytes % 8 == 0 ? 8 : 4;
  return (int)((kPlanLds / piece + 1023) / 1024);
}
template <int B, typename T = float, int J0 = 0, int NJ = stage_pieces<B, T>()>
struct StageFill {
  static constexpr int bytes = (int)sizeof(T) * B;
  static constexpr int piece = bytes % 16 == 0 ? 16 : bytes % 8 == 0 ? 8 : 4;
  using P = unsigned __attribute__((ext_vector_type(piece / 4)));
  static_assert(NJ <= 64, "one bit per piece");
  P tmp[NJ];
  uint64_t keep;  // bit j: piece j is written
  // Every load is unconditional (out-of-range pieces read from the last row
  // of V and are not written), so all pieces are in flight before the first
  // wait.  1 <= slots <= kPlanMaxSlots.
  __device__ __forceinline__ void issue(int64_t n, int64_t G, int slots,
                                        const int32_t *__restrict__ bl,
                                        const T *__restrict__ X, int ld) {
    constexpr int ppr = bytes / piece;  // pieces per row
    const int per_slot = (int)G * ppr;
    const int total = slots * per_slot;
    // opaque to the compiler, so that the piece positions are computed here
    // and not shared with (and held live until) another fill
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    // the set's block numbers are the same for the whole workgroup
    int bs[kPlanMaxSlots];
#pragma unroll
    for (int k = 0; k < kPlanMaxSlots; ++k) bs[k] = bl[min(k, slots - 1)];
    keep = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int item = tid + (J0 + j) * 1024;
      const int k = item / per_slot, off = item - k * per_slot;
      int bk = bs[0];
#pragma unroll
      for (int q = 1; q < kPlanMaxSlots; ++q) bk = k == q ? bs[q] : bk;
      const int rin = off / ppr;
      const int64_t r = (int64_t)max(bk, 0) * G + rin;
      tmp[j] = *reinterpret_cast<const P *>(X + min(r, n - 1) * ld +
                                            (off - rin * ppr) * (piece / (int)sizeof(T)));
      if (item < total && bk >= 0 && r < n) keep |= uint64_t(1) << j;
    }
  }
  __device__ __forceinline__ void commit(unsigned char *smem_raw) const {
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      if ((keep >> j) & 1) reinterpret_cast<P *>(smem_raw)[threadIdx.x + (J0 + j) * 1024] = tmp[j];
  }
};

// Pass 1 (P2 = false) or pass 2 (P2 = true) over the row groups; `bl` is the
// set's `slots` block ids for group g.  Each pass streams the
// plan's dense copy of its set's entries: bases = the per-group offsets into
// it, descriptors [n][2] = {first, end} of each row as 32-bit offsets from
// its group's first entry rounded down to a multiple of 8.
// One pass over group g, run by the whole workgroup (every thread calls it:
// it holds a barrier).  pre: the set's blocks already loaded by this thread
// (nullptr: loaded here).
template <int B, bool P2, typename T = float, bool PAIR = false>
__device__ __forceinline__ void pipe_run(int64_t g, int64_t n, int64_t G, int slots,
                                         const int64_t *__restrict__ bases,
                                         const T *__restrict__ val,
                                         const uint16_t *__restrict__ lcol,
                                         const int32_t *__restrict__ rdesc,
                                         const int32_t *__restrict__ bl,
                                         const T *__restrict__ X, T *__restrict__ Y,
                                         unsigned char *smem_raw, int ld,
                                         const StageFill<B, T> *pre = nullptr) {
  using Desc = int2;
  using Stage = PipeStage<B, P2, T, PAIR>;
  // pass 1 at 8 float columns keeps odd lanes' sums rotated (pipe_row)
  constexpr bool kRot = sizeof(T) == 4 && B == 8 && !P2 && !PAIR;
  constexpr int LPR = Stage::LPR, NO = Stage::NO, LE = Stage::LE;
  constexpr int BL = Stage::BL, LPE = Stage::LPE;
  static_assert(!P2 || BL >= LPE, "pass 2 keeps whole components per lane");
  static_assert(!PAIR || (B == 16 && sizeof(T) == 4), "lane pairs: 16 float columns");
  const T *sX = reinterpret_cast<const T *>(smem_raw);
  const int64_t r0 = g * G;
  const int nr = (int)(min(n, r0 + G) - r0);
  constexpr int RPW = kWave / LPR;
  constexpr int LCH = LE * LPE;  // entries of a row per step
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int half = PAIR ? (sub & 1) : 0;        // the lane's 8-column half (PAIR)
  const int esub = PAIR ? (sub >> 1) : sub;     // the lane's share of the row's entries
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const int stride = nwaves * RPW;
  const int zrow = slots * (int)G;  // the all-zero LDS row
  const int par = kRot ? (sub & 1) : 0;
  // first of the lane's sums after the reduction (BL >= LPE)
  const int cb = BL * half + NO * esub;
  const int64_t base = bases[g] & ~(int64_t)7;
  const uint16_t *lc_b = lcol + base;
  const T *v_b = val + base;
  const Desc *desc = reinterpret_cast<const Desc *>(rdesc) + r0;
  T *Yw = Y + r0 * ld;
  auto yrow = [&](int r) { return Yw + (int64_t)(r < nr ? r : 0) * ld + (BL >= LPE ? cb : 0); };

  // this row group's first row (relative to r0) and the descriptor of its second
  int row = wave * RPW + lane / LPR;
  int nrow = row + stride;
  const Desc d0 = desc[row < nr ? row : 0];
  Desc dn = desc[nrow < nr ? nrow : 0];
  int pl = d0.y;
  int qlb = d0.x & ~(LE - 1);
  Stage cur;
  pipe_load<B, P2, T, PAIR>(cur, lc_b, v_b, qlb + LE * esub, d0.x, pl, yrow(row));

  // stage the set's column blocks (loaded here unless the caller loaded them
  // already), then the all-zero row
  if (pre) {
    pre->commit(smem_raw);
  } else {
    // in two halves where the whole would not fit in registers beside the
    // first stage
    constexpr int kAll = stage_pieces<B, T>(), kHalf = (kAll + 1) / 2;
    if constexpr (kAll <= 10 && !pipe_wide<T, B>()) {
      StageFill<B, T> fill;
      fill.issue(n, G, slots, bl, X, ld);
      fill.commit(smem_raw);
    } else {
      StageFill<B, T, 0, kHalf> f0;
      f0.issue(n, G, slots, bl, X, ld);
      f0.commit(smem_raw);
      StageFill<B, T, kHalf, kAll - kHalf> f1;
      f1.issue(n, G, slots, bl, X, ld);
      f1.commit(smem_raw);
    }
  }
  if (threadIdx.x < B) reinterpret_cast<T *>(smem_raw)[(int64_t)zrow * B + threadIdx.x] = T(0);
  __syncthreads();
  if (row >= nr) return;  // no rows for this group of lanes

  T acc[BL];
#pragma unroll
  for (int a = 0; a < BL; ++a) acc[a] = T(0);
  // A finished row's sums, stored at the start of the following step: a store
  // issued after the step's loads would have to complete before the next
  // step's first wait.
  constexpr int NOUT = kRot ? 1 : (BL >= LPE ? NO : BL);
  T out[NOUT];
  T *yp = nullptr;
  auto store_out = [&]() __attribute__((always_inline)) {
    if constexpr (kRot) {
      if ((sub & 1) == 0) yp[sub >> 1] = out[0];
    } else if constexpr (BL >= LPE) {
      pipe_vstore<NO>(yp + cb, out);
    } else {
#pragma unroll
      for (int a = 0; a < B; ++a)
        if (a % LPR == sub) yp[a] = out[a];
    }
  };
  // One step on the entries in `cur`, loading the following step into `nxt`;
  // false once the group has no rows left.  The loop below alternates the two
  // buffers so that no load result is copied between registers (a copy would
  // wait for the load).  Per step, in issue order: the pending store, the
  // loads of the next step and the next descriptor.
  auto step = [&](const Stage &cur, Stage &nxt) __attribute__((always_inline)) {
    // everything the previous step loaded (this step's entries and the next
    // descriptor) is needed now; waiting here, before the pending store, keeps
    // that store out of the wait
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // where the next step starts: the rest of this row, else the group's next row
    const bool last = qlb + LCH >= pl;
    const bool more = !last || nrow < nr;
    int sp0 = 0, spl = pl, sqlb = qlb + LCH;
    int srow = row;
    if (last) {
      sp0 = dn.x;
      spl = dn.y;
      sqlb = sp0 & ~(LE - 1);
      srow = nrow;
    }
    if (!more) sp0 = spl = sqlb = 0;  // nothing left: an empty range
    if (yp) {
      store_out();
      yp = nullptr;
    }
    pipe_load<B, P2, T, PAIR>(nxt, lc_b, v_b, sqlb + LE * esub, sp0, spl, yrow(srow));
    // the descriptor of the row after the one the next step works on
    {
      const int r = last ? nrow + stride : nrow;
      dn = desc[r < nr ? r : 0];
    }
    // the step's entries, LG LDS rows at a time (fewer in pass 2, whose lanes
    // hold more entries and sums)
    constexpr int LG = pipe_lg<P2, pipe_wide<T, BL>()>();
#pragma unroll
    for (int hf = 0; hf < LE; hf += LG) {
      T lx[LG][BL];
      T h[LG];
#pragma unroll
      for (int e = 0; e < LG; ++e) {
        const bool ok = cur.llo <= hf + e && hf + e < cur.lhi;
        const int idx = ok ? pipe_lidx(cur.lc, hf + e) : zrow;
        h[e] = ok ? cur.lv[hf + e] : T(0);
        pipe_row<BL>(sX + idx * B + BL * half, par, lx[e]);
      }
#pragma unroll
      for (int e = 0; e < LG; ++e)
#pragma unroll
        for (int a = 0; a < BL; ++a) acc[a] = pipe_fma(h[e], lx[e][a], acc[a]);
    }
    if (last) {
      yp = Yw + (int64_t)row * ld;
      if constexpr (kRot) {
        // halving exchange with the DPP partners of halving_partner: lane
        // 15 - sub first (the opposite parity, so the halves each lane keeps
        // and sends are chosen by h8 ^ par, which also undoes the odd lanes'
        // rotation), then 7 - sub within eight, sub ^ 2 and sub ^ 1;
        // afterwards lanes sub and sub ^ 1 hold component sub >> 1
        const bool h8 = sub & 8, h4 = sub & 4, h2 = sub & 2;
        const bool f = h8 != (par != 0);
        T k4[4], k2[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const T send = f ? acc[i] : acc[i + 4];
          const T keep = f ? acc[i + 4] : acc[i];
          k4[i] = keep + dpp_f<0x140>(send);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const T send = h4 ? k4[i] : k4[i + 2];
          const T keep = h4 ? k4[i + 2] : k4[i];
          k2[i] = keep + dpp_f<0x141>(send);
        }
        const T send = h2 ? k2[0] : k2[1];
        const T k1 = (h2 ? k2[1] : k2[0]) + dpp_f<0x4E>(send);
        out[0] = k1 + dpp_f<0xB1>(k1);
      } else if constexpr (BL >= LPE) {
        // halving exchange: each round keeps the half of the sums selected by
        // one bit of esub, so the lane ends with components [NO esub, NO esub
        // + NO) of its columns (lane pairs: the rounds skip the lowest bit of
        // sub, which names the half)
        T v[BL];
#pragma unroll
        for (int a = 0; a < BL; ++a) v[a] = acc[a];
#pragma unroll
        for (int off = LPR / 2, K = BL; off >= (PAIR ? 2 : 1); off >>= 1, K >>= 1) {
          const bool up = sub & off;
#pragma unroll
          for (int i = 0; i < K / 2; ++i) {
            const T send = up ? v[i] : v[i + K / 2];
            const T keep = up ? v[i + K / 2] : v[i];
            v[i] = keep + halving_partner<PAIR>(send, off);
          }
        }
#pragma unroll
        for (int i = 0; i < NO; ++i) out[i] = v[i] + (P2 ? cur.yp[i] : T(0));
      } else {
        static_assert(!P2 && !PAIR, "pass 2 and lane pairs need BL >= LPE");
        static_assert(LPR == 16, "one DPP row per matrix row");
#pragma unroll
        for (int a = 0; a < B; ++a) out[a] = row16_sum(acc[a]);
      }
#pragma unroll
      for (int a = 0; a < BL; ++a) acc[a] = T(0);
      row = nrow;
      nrow += stride;
    }
    pl = spl;
    qlb = sqlb;
    return more;
  };
  Stage alt;
  while (step(cur, alt) && step(alt, cur)) {
  }
  store_out();  // the last row's sums
}

// Passes 1 and 2 of one group in one workgroup: each thread loads its share
// of set B as soon as its pass-1 rows are done, pass 2 writes set B over set
// A in LDS once every thread is past pass 1, and reads pass 1's row sums back
// while they are still in the L2.
template <int B, bool S, typename T = float>
__global__ __launch_bounds__(1024) void k_spmm_pipe12(int64_t n, int64_t G, int slots,
                                                      const int64_t *__restrict__ abases,
                                                      const T *__restrict__ aval,
                                                      const uint16_t *__restrict__ alcol,
                                                      const int32_t *__restrict__ arow,
                                                      const int64_t *__restrict__ bbases,
                                                      const T *__restrict__ bval,
                                                      const uint16_t *__restrict__ blcol,
                                                      const int32_t *__restrict__ brow,
                                                      const int32_t *__restrict__ blocks,
                                                      const T *__restrict__ X,
                                                      T *__restrict__ Y, int ld_arg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ld = S ? ld_arg : B;  // row stride of V and W (S: strided halves)
  const int64_t g = xcd_block(blockIdx.x);
  if (g * G >= n) return;  // grid padding: the whole workgroup leaves
  pipe_run<B, false, T>(g, n, G, slots, abases, aval, alcol, arow, blocks + g * (2 * slots), X,
                        Y, smem_raw, ld);
  // set B's blocks are loaded while the rest of the workgroup finishes pass 1
  // (where 16-byte pieces of float rows up to 32 bytes keep the held loads
  // within the register budget of 1024 threads; otherwise pass 2 loads them
  // after the barrier)
  constexpr bool kEarly = StageFill<B, T>::piece == 16 && !pipe_wide<T, B>();
  StageFill<B, T> fill;
  if (kEarly) fill.issue(n, G, slots, blocks + g * (2 * slots) + slots, X, ld);
  // pass 1's row sums written and its LDS reads done, workgroup-wide
  __syncthreads();
  pipe_run<B, true, T>(g, n, G, slots, bbases, bval, blcol, brow,
                       blocks + g * (2 * slots) + slots, X, Y, smem_raw, ld,
                       kEarly ? &fill : nullptr);
}

// The multi-set pipelined SpMM: one 1024-thread workgroup per group stages
// set s's blocks and streams its copy, for s = 0 .. nsets - 1; set 0 writes
// the row sums (16 lanes per row), later sets add theirs (2 lanes per row,
// reading the previous sums back while they are in the L2).  A set with no
// entries in the group is skipped.  The rest pass follows as its own kernel.
template <int B, bool S, bool PAIR = false>
__global__ __launch_bounds__(1024) void k_spmm_pipe_ms(int64_t n, int64_t G, int slots, int nsets,
                                                       int64_t groups,
                                                       const int64_t *__restrict__ sgroup,
                                                       const float *__restrict__ sval,
                                                       const uint16_t *__restrict__ slcol,
                                                       const int32_t *__restrict__ srow,
                                                       const int32_t *__restrict__ blocks,
                                                       const float *__restrict__ X,
                                                       float *__restrict__ Y, int ld_arg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ld = S ? ld_arg : B;  // row stride of V and W (S: strided halves)
  const int64_t g = xcd_block(blockIdx.x);
  if (g * G >= n) return;  // grid padding: the whole workgroup leaves
  const int width = nsets * slots;
  pipe_run<B, false, float, PAIR>(g, n, G, slots, sgroup, sval, slcol, srow, blocks + g * width,
                                  X, Y, smem_raw, ld);
  for (int s = 1; s < nsets; ++s) {
    const int64_t *sg = sgroup + s * (groups + 1);
    if (sg[g + 1] == sg[g]) continue;  // uniform: no entries of set s in this group
    // the previous set's row sums written and its LDS reads done
    __syncthreads();
    pipe_run<B, true, float, PAIR>(g, n, G, slots, sg, sval, slcol, srow + (int64_t)s * n * 2,
                                   blocks + g * width + s * slots, X, Y, smem_raw, ld);
  }
}

// Pass 3: kRestLanes lanes per listed row (rows with entries outside both
// staged sets, {row, count, first entry}; the list's length is
// rgroup[groups]).  Lane s takes the row's entries s, s + L, s + 2L, ..., U
// of them in flight per round, read in place from the plan's arrays, and
// gathers the rows of V they need; a butterfly adds the lanes' sums (every
// lane ends with the same, fixed-order total) and lane s adds components
// s, s + L, ... to the row of W.  A grid-stride loop covers any length.
constexpr int kRestLanes = 8;
template <int B, bool S, typename T = float>
__global__ __launch_bounds__(256) void k_spmm_rest(const int64_t *__restrict__ rgroup,
                                                   int64_t groups,
                                                   const int4 *__restrict__ rlist,
                                                   const int32_t *__restrict__ col2,
                                                   const T *__restrict__ val2,
                                                   const T *__restrict__ X,
                                                   T *__restrict__ Y, int ld_arg) {
  constexpr int L = kRestLanes, U = 4, NC = (B + L - 1) / L;
  const int ld = S ? ld_arg : B;  // row stride of V and W (S: strided halves)
  const int64_t total = rgroup[groups];
  const int s = (int)(threadIdx.x & (L - 1));
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / L);
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L; i < total; i += stride) {
    const int4 d = rlist[i];
    const int64_t row = d.x;
    const int cnt = d.y;
    const int64_t first = (int64_t)(uint32_t)d.z | ((int64_t)d.w << 32);
    T y[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) y[k] = s + k * L < B ? Y[row * ld + s + k * L] : T(0);
    T acc[B];
#pragma unroll
    for (int a = 0; a < B; ++a) acc[a] = T(0);
    // the same trip count on all L lanes of the row; every load is issued
    // (past the row's end a lane reloads its last entry and drops the product)
    for (int t0 = 0; t0 < cnt; t0 += L * U) {
      int c[U];
      T h[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = first + min(t0 + s + L * u, cnt - 1);
        c[u] = col2[q];
        h[u] = val2[q];
      }
      T x[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u) RowIO<T, B>::load(X + (int64_t)c[u] * ld, x[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = t0 + s + L * u < cnt;
#pragma unroll
        for (int a = 0; a < B; ++a) acc[a] = pipe_fma(h[u], ok ? x[u][a] : T(0), acc[a]);
      }
    }
#pragma unroll
    for (int m = 1; m < L; m <<= 1)
#pragma unroll
      for (int a = 0; a < B; ++a) acc[a] += __shfl_xor(acc[a], m, L);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int a = s + k * L;
      T v = T(0);
#pragma unroll
      for (int a2 = 0; a2 < B; ++a2) v = a2 == a ? acc[a2] : v;
      if (a < B) Y[row * ld + a] = y[k] + v;
    }
  }
}

constexpr int kPlanThreads = 1024;
constexpr int kPlanParts = 2;   // workgroups per row group

// entries per group of the block table: a second set (for the two-pass
// kernel) whenever the plan has 16-bit LDS indices and row descriptors
int plan_width(const bbl_spmm_plan &P) { return P.lcol && P.rdesc ? 2 * P.slots : P.slots; }

template <typename VT, typename XT, int BV, bool LC16>
void planned_launch_t(const bbl_spmm_plan &P, const XT *X, XT *Y, hipStream_t s) {
  auto kern = k_spmm_planned<VT, XT, XT, XT, BV, 16, LC16>;
  const size_t lds = (size_t)P.slots * P.block_rows * BV * sizeof(XT);
  if (lds > 65536) {
    static bool attr_set = false;
    if (!attr_set) {
      BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlanLds));
      attr_set = true;
    }
  }
  const int parts = (int)std::min<int64_t>(kPlanParts, ceil_div(P.block_rows, 64));
  const int64_t groups = ceil_div(P.n, P.block_rows);
  const int64_t grid = ceil_div(groups * parts, kXcds) * kXcds;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPlanThreads), lds, s, P.n,
                     (int64_t)P.block_rows, P.slots, plan_width(P), parts, P.row_ptr, P.n_local,
                     P.col, static_cast<const VT *>(P.val), P.lcol, P.blocks, X, Y);
  check_launch("k_spmm_planned");
}

// Whether a plan can run through the pipelined kernels at BK vectors per
// pass: 16-bit LDS indices, the per-row descriptors and dense copies, and
// the staged sets plus the all-zero row within the LDS.
bool plan_pipe_ok(bool local16, bool copies, int slots, int64_t block_rows, int BK,
                  size_t elem = sizeof(float)) {
  return local16 && copies && ((size_t)slots * block_rows + 1) * BK * elem <= kPlanLds;
}

// Passes 1 and 2 in one workgroup per group (pass 1: 16 lanes per row over
// set A; pass 2: 2 lanes per row over set B), then pass 3 for the rest, one
// lane per listed row.
template <int BV, bool S, typename T = float>
void planned_launch_pipe(const bbl_spmm_plan &P, const T *X, T *Y, int ld, hipStream_t s) {
  auto kern = k_spmm_pipe12<BV, S, T>;
  const size_t lds = ((size_t)P.slots * P.block_rows + 1) * BV * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlanLds));
    attr_set = true;
  }
  const int64_t groups = ceil_div(P.n, P.block_rows);
  hipLaunchKernelGGL(kern, dim3((unsigned)(ceil_div(groups, kXcds) * kXcds)), dim3(kPlanThreads),
                     lds, s, P.n, (int64_t)P.block_rows, P.slots, P.agroup,
                     static_cast<const T *>(P.aval), P.alcol, P.arow, P.bgroup,
                     static_cast<const T *>(P.bval), P.blcol, P.brow, P.blocks, X, Y, ld);
  check_launch("k_spmm_pipe12");
  // the list's length is on the device: a grid of at most 4096 workgroups
  // (32 rows each) strides over it
  const int64_t grid =
      std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(P.n * kRestLanes, 256)));
  hipLaunchKernelGGL((k_spmm_rest<BV, S, T>), dim3((unsigned)grid), dim3(256), 0, s, P.rgroup,
                     groups, reinterpret_cast<const int4 *>(P.rlist), P.col,
                     static_cast<const T *>(P.val), X, Y, ld);
  check_launch("k_spmm_rest");
}

// The multi-set plan: its sets in one workgroup per group, then the rest pass.
template <int BV, bool S, bool PAIR = false>
void planned_launch_ms(const bbl_spmm_plan &P, const float *X, float *Y, int ld, hipStream_t s) {
  auto kern = k_spmm_pipe_ms<BV, S, PAIR>;
  const size_t lds = ((size_t)P.slots * P.block_rows + 1) * BV * sizeof(float);
  static bool attr_set = false;
  if (!attr_set) {
    BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlanLds));
    attr_set = true;
  }
  const int64_t groups = ceil_div(P.n, P.block_rows);
  hipLaunchKernelGGL(kern, dim3((unsigned)(ceil_div(groups, kXcds) * kXcds)), dim3(kPlanThreads),
                     lds, s, P.n, (int64_t)P.block_rows, P.slots, P.nsets, groups, P.sgroup,
                     static_cast<const float *>(P.sval), P.slcol, P.srow, P.blocks, X, Y, ld);
  check_launch("k_spmm_pipe_ms");
  const int64_t grid =
      std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(P.n * kRestLanes, 256)));
  hipLaunchKernelGGL((k_spmm_rest<BV, S>), dim3((unsigned)grid), dim3(256), 0, s, P.rgroup, groups,
                     reinterpret_cast<const int4 *>(P.rlist), P.rcol,
                     static_cast<const float *>(P.rval), X, Y, ld);
  check_launch("k_spmm_rest");
}

template <typename VT, typename XT, int BV>
void planned_launch(const bbl_spmm_plan &P, const XT *X, XT *Y, hipStream_t s) {
  // float64 values and vectors at 4 or 8 columns: the same three passes on
  // rows of doubles (32 or 64 bytes in LDS)
  if constexpr (std::is_same<VT, double>::value && std::is_same<XT, double>::value &&
                (BV == 4 || BV == 8)) {
    if (plan_pipe_ok(P.local16 && P.lcol, P.rdesc && P.arow && P.brow && P.rlist, P.slots,
                     P.block_rows, BV, sizeof(double))) {
      planned_launch_pipe<BV, false, double>(P, X, Y, BV, s);
      return;
    }
  }
  if constexpr (std::is_same<VT, float>::value && std::is_same<XT, float>::value &&
                (BV == 4 || BV == 8 || BV == 10 || BV == 16)) {
    if (P.nsets > 0) {
      if constexpr (BV == 16) {
        // a plan whose sets hold 16-wide rows: one pass with lane pairs;
        // else (slots sized for 8 columns) two passes over the halves
        if (((size_t)P.slots * P.block_rows + 1) * 16 * sizeof(float) <= kPlanLds) {
          planned_launch_ms<16, false, true>(P, X, Y, 16, s);
        } else {
          planned_launch_ms<8, true>(P, X, Y, 16, s);
          planned_launch_ms<8, true>(P, X + 8, Y + 8, 16, s);
        }
      } else {
        planned_launch_ms<BV, false>(P, X, Y, BV, s);
      }
      return;
    }
    // the pipelined kernel also keeps one all-zero row of V in LDS and takes
    // 32-bit entry offsets; 16 vectors go through it as two halves of 8
    constexpr int BK = BV == 16 ? 8 : BV;
    if (plan_pipe_ok(P.local16 && P.lcol, P.rdesc && P.arow && P.brow && P.rlist, P.slots,
                     P.block_rows, BK)) {
      planned_launch_pipe<BK, BV != BK>(P, X, Y, BV, s);
      if constexpr (BV == 16) planned_launch_pipe<BK, true>(P, X + 8, Y + 8, BV, s);
      return;
    }
    if constexpr (BV == 16)
      BBL_REQUIRE((size_t)P.slots * P.block_rows * BV * sizeof(float) <= kPlanLds,
                  "planned SpMM: plan built for the two-half kernel cannot run here");
  }
  if (P.local16 && P.lcol) planned_launch_t<VT, XT, BV, true>(P, X, Y, s);
  else planned_launch_t<VT, XT, BV, false>(P, X, Y, s);
}

template <typename VT, typename XT>
void planned_dispatch(const bbl_spmm_plan &P, const XT *X, XT *Y, hipStream_t s) {
  switch (P.nvec) {
    case 1: planned_launch<VT, XT, 1>(P, X, Y, s); break;
    case 2: planned_launch<VT, XT, 2>(P, X, Y, s); break;
    case 4: planned_launch<VT, XT, 4>(P, X, Y, s); break;
    case 8: planned_launch<VT, XT, 8>(P, X, Y, s); break;
    case 10: planned_launch<VT, XT, 10>(P, X, Y, s); break;
    case 12:  // float32 only (float64 rows of 12 exceed the register budget)
      if constexpr (std::is_same<XT, float>::value) planned_launch<VT, XT, 12>(P, X, Y, s);
      else throw Error{BBL_E_INVALID, "planned SpMM: 12 float64 vectors are not planned"};
      break;
    case 16: planned_launch<VT, XT, 16>(P, X, Y, s); break;
    default: throw Error{BBL_E_INVALID, "planned SpMM: unsupported nvec"};
  }
}

}  // namespace

void launch_spmm(const bbl_csr &H, const void *X, int xdtype, void *Y, int ydtype, int nvec,
                 hipStream_t s) {
  if (H.n == 0) return;
  if (H.val_dtype == BBL_F32 && xdtype == BBL_F32 && ydtype == BBL_F32) {
    spmm_dispatch<float, float, float, float>(H, static_cast<const float *>(X),
                                              static_cast<float *>(Y), nvec, s);
  } else if (H.val_dtype == BBL_F64 && xdtype == BBL_F64 && ydtype == BBL_F64) {
    spmm_dispatch<double, double, double, double>(H, static_cast<const double *>(X),
                                                  static_cast<double *>(Y), nvec, s);
  } else if (H.val_dtype == BBL_F32 && xdtype == BBL_F64 && ydtype == BBL_F64) {
    spmm_dispatch<float, double, double, double>(H, static_cast<const double *>(X),
                                                 static_cast<double *>(Y), nvec, s);
  } else {
    throw Error{BBL_E_INVALID, "spmm: unsupported dtype combination"};
  }
}

template <int NV>
int residual_t(const bbl_csr &H, const double *X, const double *theta, double *partial,
               int max_partials, int lpr, hipStream_t s) {
  // whole multiple of 8 workgroups (XCD order), each a contiguous run of at
  // least 64 rows
  int64_t grid = std::min<int64_t>(max_partials, std::max<int64_t>(8, ceil_div(H.n, 64)));
  grid = std::max<int64_t>(8, grid / 8 * 8);
  const int64_t chunk = ceil_div(H.n, grid);
#define BBL_REST(VT, L)                                                                       \
  hipLaunchKernelGGL((k_residual_t<VT, L, NV>), dim3((unsigned)grid), dim3(256), 0, s, H.n,    \
                     H.row_ptr, H.col, static_cast<const VT *>(H.val), X, theta, chunk, partial)
  if (H.val_dtype == BBL_F32) {
    if (lpr == 16) BBL_REST(float, 16);
    else if (lpr == 32) BBL_REST(float, 32);
    else BBL_REST(float, 64);
  } else {
    if (lpr == 16) BBL_REST(double, 16);
    else if (lpr == 32) BBL_REST(double, 32);
    else BBL_REST(double, 64);
  }
#undef BBL_REST
  check_launch("k_residual_t");
  return (int)grid;
}

int launch_residual_spmm(const bbl_csr &H, const double *X, int nvec, const double *theta,
                         double *partial, int max_partials, hipStream_t s) {
  const int lpr = pick_lpr(H);
  if (max_partials >= 8) {
    switch (nvec) {
      case 4: return residual_t<4>(H, X, theta, partial, max_partials, lpr, s);
      case 8: return residual_t<8>(H, X, theta, partial, max_partials, lpr, s);
      case 10: return residual_t<10>(H, X, theta, partial, max_partials, lpr, s);
      case 16: return residual_t<16>(H, X, theta, partial, max_partials, lpr, s);
      default: break;
    }
  }
  const int rows_per_wg = (256 / kWave) * (kWave / lpr);
  int grid = (int)std::min<int64_t>(ceil_div(H.n, rows_per_wg), max_partials);
  if (grid < 1) grid = 1;
#define BBL_RES(VT, L)                                                                        \
  hipLaunchKernelGGL((k_residual<VT, L>), dim3(grid), dim3(256), 0, s, H.n, H.row_ptr, H.col, \
                     static_cast<const VT *>(H.val), X, nvec, theta, partial)
  if (H.val_dtype == BBL_F32) {
    if (lpr == 16) BBL_RES(float, 16);
    else if (lpr == 32) BBL_RES(float, 32);
    else BBL_RES(float, 64);
  } else {
    if (lpr == 16) BBL_RES(double, 16);
    else if (lpr == 32) BBL_RES(double, 32);
    else BBL_RES(double, 64);
  }
#undef BBL_RES
  check_launch("k_residual");
  return grid;
}


// LDS row indices slot*G + offset all fit in 16 bits
bool plan_local16(const bbl_csr &H, int slots) {
  return (int64_t)slots * H.block_rows <= 65536;
}

// per-row 32-bit entry offsets from the group's first entry
bool plan_desc(const bbl_csr &H) { return H.nnz < ((int64_t)1 << 31) - 64; }

// Multi-set layout: float32 values and vectors at 4, 8, 10 or 16 vectors
// (16 as 16-wide rows read by lane pairs where a block of them fits in LDS,
// else as two halves of 8), when fewer than three column blocks fit in LDS
// per set or the entries need 64-bit offsets.  *slots blocks per set,
// *nsets sets covering the busiest kMsBlocks blocks of each group.
constexpr int kMsBlocks = 10;
bool plan_multi(const bbl_csr &H, int nvec, int vec_dtype, int *slots, int *nsets) {
  if (H.block_rows <= 0 || H.val_dtype != BBL_F32 || vec_dtype != BBL_F32) return false;
  if (!(nvec == 4 || nvec == 8 || nvec == 10 || nvec == 16)) return false;
  // 16 vectors: sets of 16-wide rows (one pass, lane pairs) when one block
  // fits in LDS with the zero row, else 8-column halves
  const bool w16 = nvec == 16 && ((int64_t)H.block_rows + 1) * 64 <= (int64_t)kPlanLds;
  const int BK = nvec == 16 && !w16 ? 8 : nvec;
  const int64_t s = std::min<int64_t>(kPlanMaxSlots,
                                      ((int64_t)kPlanLds / (BK * 4) - 1) / H.block_rows);
  if (s < 1 || s * H.block_rows > 65536) return false;
  if (s >= 3 && plan_desc(H)) return false;
  *slots = (int)s;
  *nsets = (int)std::min<int64_t>(kMsMaxWidth / s, ceil_div(kMsBlocks, s));
  return true;
}

int spmm_plan_slots(const bbl_csr &H, int nvec, int vec_dtype) {
  if (H.block_rows <= 0) return 0;
  int ms, mn;
  if (plan_multi(H, nvec, vec_dtype, &ms, &mn)) return ms;
  if (!(nvec == 1 || nvec == 2 || nvec == 4 || nvec == 8 || nvec == 10 || nvec == 16 ||
        (nvec == 12 && vec_dtype == BBL_F32)))
    return 0;
  if (nvec == 16 && vec_dtype == BBL_F32 && H.val_dtype == BBL_F32 && plan_desc(H)) {
    // FP32, 16 vectors: the pipelined kernels take the columns in two halves
    // of 8, so a slot holds 8 columns of a block (beside the all-zero row)
    const int s8 = (int)std::min<int64_t>(kPlanMaxSlots, ((int64_t)kPlanLds / 32 - 1) / H.block_rows);
    if (s8 >= 1 && plan_pipe_ok(plan_local16(H, s8), true, s8, H.block_rows, 8)) return s8;
  }
  const size_t per = (size_t)H.block_rows * nvec * (vec_dtype == BBL_F32 ? 4 : 8);
  return (int)std::min<size_t>(kPlanMaxSlots, kPlanLds / per);
}

// Regions of a multi-set plan, in order (byte sizes; each 256-aligned).
struct MsLayout {
  size_t blocks, sgroup, srow, rcnt, rpre, rtot, rpos, rgroup, rlist, vals, idx;
};
MsLayout ms_layout(const bbl_csr &H, int slots, int nsets) {
  const int64_t groups = ceil_div(H.n, H.block_rows);
  MsLayout L;
  L.blocks = (size_t)groups * nsets * slots * 4;
  L.sgroup = (size_t)nsets * (groups + 1) * 8;
  L.srow = (size_t)nsets * H.n * 8;
  L.rcnt = L.rpre = L.rpos = (size_t)H.n * 4;
  L.rtot = L.rgroup = (size_t)(groups + 1) * 8;
  L.rlist = (size_t)H.n * 16;
  L.vals = L.idx = (size_t)(H.nnz + 16) * 4;
  return L;
}
size_t ms_bytes(const MsLayout &L) {
  return align_up(L.blocks) + align_up(L.sgroup) + align_up(L.srow) + align_up(L.rcnt) +
         align_up(L.rpre) + align_up(L.rtot) + align_up(L.rpos) + align_up(L.rgroup) +
         align_up(L.rlist) + align_up(L.vals) + align_up(L.idx) + 256;
}

size_t spmm_plan_bytes(const bbl_csr &H, int nvec, int vec_dtype) {
  int ms, mn;
  if (plan_multi(H, nvec, vec_dtype, &ms, &mn)) return ms_bytes(ms_layout(H, ms, mn));
  const int slots = spmm_plan_slots(H, nvec, vec_dtype);
  if (slots < 1) return 0;
  const int64_t groups = ceil_div(H.n, H.block_rows);
  const size_t sv = H.val_dtype == BBL_F32 ? 4 : 8;
  // index and value arrays padded by 16 entries for the chunk loads
  const int width = plan_local16(H, slots) && plan_desc(H) ? 2 * slots : slots;
  return align_up((size_t)groups * width * 4) + align_up((size_t)H.n * 4) +
         align_up((size_t)(H.nnz + 16) * 4) + align_up((size_t)(H.nnz + 16) * sv) +
         (plan_local16(H, slots) ? align_up((size_t)(H.nnz + 16) * 2) : 0) +
         (plan_local16(H, slots) && plan_desc(H)
              ? align_up((size_t)H.n * 16) + align_up((size_t)H.n * 8) +
                    align_up((size_t)(groups + 1) * 8) + align_up((size_t)(H.nnz + 16) * 2) +
                    align_up((size_t)(H.nnz + 16) * sv) + align_up((size_t)H.n * 4) +
                    align_up((size_t)(groups + 1) * 8) + align_up((size_t)H.n * 16) +
                    align_up((size_t)H.n * 8) + align_up((size_t)(groups + 1) * 8) +
                    align_up((size_t)(H.nnz + 16) * 2) + align_up((size_t)(H.nnz + 16) * sv)
              : 0) +
         256;
}

__global__ void k_add_base(int64_t *a, int64_t m, int64_t base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) a[i] += base;
}

// Multi-set plan: block choice, per-row counts, per-group offsets, their scan
// over groups, the set bases (the copies lie set after set), then the fill.
// Reads the totals back to the host once (synchronises the stream).
void build_ms_plan(const bbl_csr &H, int nvec, int vec_dtype, int slots, int nsets, void *mem,
                   size_t bytes, bbl_spmm_plan *P, hipStream_t s) {
  const MsLayout L = ms_layout(H, slots, nsets);
  if (bytes < ms_bytes(L)) throw Error{BBL_E_NOMEM, "plan memory too small"};
  const int64_t groups = ceil_div(H.n, H.block_rows), G = H.block_rows;
  const int width = nsets * slots;
  char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(mem), 256));
  size_t off = 0;
  auto take = [&](size_t b) {
    char *p = base + off;
    off += align_up(b);
    return p;
  };
  int32_t *blocks = reinterpret_cast<int32_t *>(take(L.blocks));
  int64_t *sgroup = reinterpret_cast<int64_t *>(take(L.sgroup));
  int32_t *srow = reinterpret_cast<int32_t *>(take(L.srow));
  int32_t *rcnt = reinterpret_cast<int32_t *>(take(L.rcnt));
  int32_t *rpre = reinterpret_cast<int32_t *>(take(L.rpre));
  int64_t *rtot = reinterpret_cast<int64_t *>(take(L.rtot));
  int32_t *rpos = reinterpret_cast<int32_t *>(take(L.rpos));
  int64_t *rgroup = reinterpret_cast<int64_t *>(take(L.rgroup));
  int32_t *rlist = reinterpret_cast<int32_t *>(take(L.rlist));
  float *vals = reinterpret_cast<float *>(take(L.vals));
  char *idx = take(L.idx);
  hipLaunchKernelGGL(k_plan_blocks, dim3((unsigned)groups), dim3(256), 0, s, H.n, G, width,
                     H.row_ptr, H.col, blocks);
  // one wave per row, runs of kMsRowsPerWave rows per wave
  const unsigned grid = capped_grid(ceil_div(H.n, 4 * kMsRowsPerWave), 256);
  hipLaunchKernelGGL(k_ms_count, dim3(grid), dim3(256), 0, s, H.n, G, slots, width, H.row_ptr,
                     H.col, blocks, srow, rcnt);
  hipLaunchKernelGGL(k_ms_group, dim3((unsigned)groups), dim3(256), 0, s, H.n, G, nsets, groups,
                     srow, sgroup, rcnt, rpre, rtot, rpos, rgroup);
  for (int k = 0; k < nsets; ++k)
    hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, sgroup + k * (groups + 1), groups);
  hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, rtot, groups);
  hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, rgroup, groups);
  check_launch("multi-set plan counts");
  std::vector<int64_t> tot(nsets + 1);
  for (int k = 0; k < nsets; ++k)
    BBL_HIP(hipMemcpyAsync(&tot[k], sgroup + k * (groups + 1) + groups, 8, hipMemcpyDeviceToHost,
                           s));
  BBL_HIP(hipMemcpyAsync(&tot[nsets], rtot + groups, 8, hipMemcpyDeviceToHost, s));
  BBL_HIP(hipStreamSynchronize(s));
  int64_t run = 0;
  for (int k = 0; k < nsets; ++k) {
    if (run > 0)
      hipLaunchKernelGGL(k_add_base, dim3((unsigned)ceil_div(groups + 1, 256)), dim3(256), 0, s,
                         sgroup + k * (groups + 1), groups + 1, run);
    run += tot[k];
  }
  const int64_t rest = tot[nsets];
  BBL_REQUIRE(run + rest == H.nnz, "multi-set plan: entry counts do not add up");
  uint16_t *slcol = reinterpret_cast<uint16_t *>(idx);
  int32_t *rcol = reinterpret_cast<int32_t *>(idx + L.idx) - rest;  // from the back
  float *rval = vals + (H.nnz + 16) - rest;
  hipLaunchKernelGGL((k_ms_fill<float>), dim3(grid), dim3(256), 0, s, H.n, G, slots, width,
                     groups, H.row_ptr, H.col, static_cast<const float *>(H.val), blocks, srow,
                     sgroup, slcol, vals, rcnt, rpre, rtot, rpos, rgroup, rcol, rval,
                     reinterpret_cast<int4 *>(rlist));
  check_launch("multi-set plan fill");
  *P = bbl_spmm_plan{};
  P->n = H.n;
  P->nnz = H.nnz;
  P->block_rows = H.block_rows;
  P->slots = slots;
  P->nvec = nvec;
  P->vec_dtype = vec_dtype;
  P->val_dtype = H.val_dtype;
  P->local16 = 1;
  P->row_ptr = H.row_ptr;
  P->blocks = blocks;
  P->rgroup = rgroup;
  P->rlist = rlist;
  P->nsets = nsets;
  P->sgroup = sgroup;
  P->srow = srow;
  P->slcol = slcol;
  P->sval = vals;
  P->rcol = rcol;
  P->rval = rval;
}

void build_spmm_plan(const bbl_csr &H, int nvec, int vec_dtype, void *mem, size_t bytes,
                     bbl_spmm_plan *P, hipStream_t s) {
  {
    int ms, mn;
    if (plan_multi(H, nvec, vec_dtype, &ms, &mn))
      return build_ms_plan(H, nvec, vec_dtype, ms, mn, mem, bytes, P, s);
  }
  const int slots = spmm_plan_slots(H, nvec, vec_dtype);
  if (slots < 1)
    throw Error{BBL_E_INVALID, "no plan: block_rows must be > 0, nvec in {1,2,4,8,10,16} and "
                               "one block of V must fit in 160 KB of LDS"};
  if (bytes < spmm_plan_bytes(H, nvec, vec_dtype)) throw Error{BBL_E_NOMEM, "plan memory too small"};
  const int64_t groups = ceil_div(H.n, H.block_rows);
  const size_t sv = H.val_dtype == BBL_F32 ? 4 : 8;
  char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(mem), 256));
  size_t off = 0;
  auto take = [&](size_t b) {
    char *p = base + off;
    off += align_up(b);
    return p;
  };
  const int width = plan_local16(H, slots) && plan_desc(H) ? 2 * slots : slots;
  int32_t *blocks = reinterpret_cast<int32_t *>(take((size_t)groups * width * 4));
  int32_t *n_local = reinterpret_cast<int32_t *>(take((size_t)H.n * 4));
  int32_t *col2 = reinterpret_cast<int32_t *>(take((size_t)(H.nnz + 16) * 4));
  void *val2 = take((size_t)(H.nnz + 16) * sv);
  const bool l16 = plan_local16(H, slots);
  uint16_t *lcol = l16 ? reinterpret_cast<uint16_t *>(take((size_t)(H.nnz + 16) * 2)) : nullptr;
  const bool two = l16 && plan_desc(H);
  int32_t *rdesc = two ? reinterpret_cast<int32_t *>(take((size_t)H.n * 16)) : nullptr;
  int32_t *arow = two ? reinterpret_cast<int32_t *>(take((size_t)H.n * 8)) : nullptr;
  int64_t *agroup = two ? reinterpret_cast<int64_t *>(take((size_t)(groups + 1) * 8)) : nullptr;
  uint16_t *alcol = two ? reinterpret_cast<uint16_t *>(take((size_t)(H.nnz + 16) * 2)) : nullptr;
  void *aval = two ? take((size_t)(H.nnz + 16) * sv) : nullptr;
  int32_t *brow = two ? reinterpret_cast<int32_t *>(take((size_t)H.n * 8)) : nullptr;
  int64_t *bgroup = two ? reinterpret_cast<int64_t *>(take((size_t)(groups + 1) * 8)) : nullptr;
  uint16_t *blcol = two ? reinterpret_cast<uint16_t *>(take((size_t)(H.nnz + 16) * 2)) : nullptr;
  void *bval = two ? take((size_t)(H.nnz + 16) * sv) : nullptr;
  int32_t *rpos = two ? reinterpret_cast<int32_t *>(take((size_t)H.n * 4)) : nullptr;
  int64_t *rgroup = two ? reinterpret_cast<int64_t *>(take((size_t)(groups + 1) * 8)) : nullptr;
  int32_t *rlist = two ? reinterpret_cast<int32_t *>(take((size_t)H.n * 16)) : nullptr;
  hipLaunchKernelGGL(k_plan_blocks, dim3((unsigned)groups), dim3(256), 0, s, H.n,
                     (int64_t)H.block_rows, width, H.row_ptr, H.col, blocks);
  const unsigned grid = capped_grid(ceil_div(H.n, 4), 256);  // one wave per row, strided
  if (H.val_dtype == BBL_F32)
    hipLaunchKernelGGL((k_plan_rows<float>), dim3(grid), dim3(256), 0, s, H.n,
                       (int64_t)H.block_rows, slots, width, H.row_ptr, H.col,
                       static_cast<const float *>(H.val), blocks, n_local, col2,
                       static_cast<float *>(val2), lcol, rdesc, brow);
  else
    hipLaunchKernelGGL((k_plan_rows<double>), dim3(grid), dim3(256), 0, s, H.n,
                       (int64_t)H.block_rows, slots, width, H.row_ptr, H.col,
                       static_cast<const double *>(H.val), blocks, n_local, col2,
                       static_cast<double *>(val2), lcol, rdesc, brow);
  if (two) {
    hipLaunchKernelGGL(k_plan_bgroup, dim3((unsigned)groups), dim3(256), 0, s, H.n,
                       (int64_t)H.block_rows, rdesc, n_local, arow, agroup, brow, bgroup, rpos,
                       rgroup);
    hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, agroup, groups);
    hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, bgroup, groups);
    hipLaunchKernelGGL(k_plan_gscan, dim3(1), dim3(1024), 0, s, rgroup, groups);
    if (H.val_dtype == BBL_F32)
      hipLaunchKernelGGL((k_plan_bfill<float>), dim3(grid), dim3(256), 0, s, H.n,
                         (int64_t)H.block_rows, H.row_ptr, n_local, lcol,
                         static_cast<const float *>(val2), agroup, arow, alcol,
                         static_cast<float *>(aval), bgroup, brow, blcol,
                         static_cast<float *>(bval), rdesc, rpos, rgroup,
                         reinterpret_cast<int4 *>(rlist));
    else
      hipLaunchKernelGGL((k_plan_bfill<double>), dim3(grid), dim3(256), 0, s, H.n,
                         (int64_t)H.block_rows, H.row_ptr, n_local, lcol,
                         static_cast<const double *>(val2), agroup, arow, alcol,
                         static_cast<double *>(aval), bgroup, brow, blcol,
                         static_cast<double *>(bval), rdesc, rpos, rgroup,
                         reinterpret_cast<int4 *>(rlist));
  }
  check_launch("spmm plan");
  *P = bbl_spmm_plan{};
  P->n = H.n;
  P->nnz = H.nnz;
  P->block_rows = H.block_rows;
  P->slots = slots;
  P->nvec = nvec;
  P->vec_dtype = vec_dtype;
  P->val_dtype = H.val_dtype;
  P->local16 = l16 ? 1 : 0;
  P->row_ptr = H.row_ptr;
  P->blocks = blocks;
  P->n_local = n_local;
  P->col = col2;
  P->val = val2;
  P->lcol = lcol;
  P->rdesc = rdesc;
  P->agroup = agroup;
  P->arow = arow;
  P->alcol = alcol;
  P->aval = aval;
  P->bgroup = bgroup;
  P->brow = brow;
  P->blcol = blcol;
  P->bval = bval;
  P->rgroup = rgroup;
  P->rlist = rlist;
}

void launch_spmm_planned(const bbl_spmm_plan &P, const void *X, void *Y, hipStream_t s) {
  if (P.n == 0) return;
  if (P.val_dtype == BBL_F32 && P.vec_dtype == BBL_F32)
    planned_dispatch<float, float>(P, static_cast<const float *>(X), static_cast<float *>(Y), s);
  else if (P.val_dtype == BBL_F64 && P.vec_dtype == BBL_F64)
    planned_dispatch<double, double>(P, static_cast<const double *>(X), static_cast<double *>(Y),
                                     s);
  else
    throw Error{BBL_E_INVALID, "planned SpMM: values and vectors must share float32 or float64"};
}

}  // namespace bbl
