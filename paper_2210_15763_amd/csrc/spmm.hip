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

// Sector-staged variant for matrices whose rows come in aligned groups of G
// rows holding most of their columns (bbl_csr.block_rows): one workgroup per
// group copies the group's G rows of V into LDS with full-line loads, then
// gathers in-group columns from LDS and the rest from HBM.  The random 32-byte
// gathers otherwise each pull a 128-byte line through L2; staging turns the
// in-group share of them into one streaming read of V.
template <typename VT, typename XT, typename AT, typename YT, int B, int LPR>
__global__ __launch_bounds__(512) void k_spmm_blk(int64_t n, int64_t G,
                                                  const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const VT *__restrict__ val,
                                                  const XT *__restrict__ X, YT *__restrict__ Y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  XT *sX = reinterpret_cast<XT *>(smem_raw);
  const int64_t r0 = xcd_block(blockIdx.x) * G;
  if (r0 >= n) return;  // grid padding: the whole workgroup leaves
  const int64_t r1 = min(n, r0 + G);
  const uint64_t W = (uint64_t)(r1 - r0);
  {
    constexpr int bytes = (int)sizeof(XT) * B;
    const unsigned char *src = reinterpret_cast<const unsigned char *>(X + r0 * B);
    const int64_t total = (int64_t)W * bytes;
    if constexpr (bytes % 16 == 0) {
      for (int64_t i = threadIdx.x; i < total / 16; i += blockDim.x)
        reinterpret_cast<uint4 *>(smem_raw)[i] = reinterpret_cast<const uint4 *>(src)[i];
    } else if constexpr (bytes % 8 == 0) {
      for (int64_t i = threadIdx.x; i < total / 8; i += blockDim.x)
        reinterpret_cast<uint2 *>(smem_raw)[i] = reinterpret_cast<const uint2 *>(src)[i];
    } else {
      for (int64_t i = threadIdx.x; i < total / 4; i += blockDim.x)
        reinterpret_cast<uint32_t *>(smem_raw)[i] = reinterpret_cast<const uint32_t *>(src)[i];
    }
  }
  __syncthreads();
  constexpr int RPW = kWave / LPR;
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPR - 1);
  const int wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  // the loop bound is uniform per wave, so every lane joins the butterfly
  for (int64_t base = r0 + (int64_t)wave * RPW; base < r1; base += (int64_t)nwaves * RPW) {
    const int64_t row = base + lane / LPR;
    AT acc[B];
#pragma unroll
    for (int a = 0; a < B; ++a) acc[a] = AT(0);
    if (row < r1) {
      const int64_t p0 = rp[row], p1 = rp[row + 1];
      int64_t p = p0 + sub;
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
        for (int u = 0; u < UNR; ++u) {
          const uint64_t off = (uint64_t)((int64_t)c[u] - r0);
          if (off < W) RowIO<XT, B>::load(sX + off * B, x[u]);
          else RowIO<XT, B>::load(X + (int64_t)c[u] * B, x[u]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int a = 0; a < B; ++a) acc[a] = fma(h[u], (AT)x[u][a], acc[a]);
      }
      for (; p < p1; p += LPR) {
        const int c0 = ldg_stream(col + p);
        const AT h0 = (AT)ldg_stream(val + p);
        XT x0[B];
        const uint64_t off = (uint64_t)((int64_t)c0 - r0);
        if (off < W) RowIO<XT, B>::load(sX + off * B, x0);
        else RowIO<XT, B>::load(X + (int64_t)c0 * B, x0);
#pragma unroll
        for (int a = 0; a < B; ++a) acc[a] = fma(h0, (AT)x0[a], acc[a]);
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

constexpr size_t kBlkMaxLds = 128 * 1024;   // LDS bytes a staged group may use
constexpr int kBlkThreads = 512;

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
  const VT *valp = static_cast<const VT *>(H.val);
  const size_t lds = (size_t)H.block_rows * nvec * sizeof(XT);
  if (H.block_rows > 0 && lds <= kBlkMaxLds &&
      (nvec == 1 || nvec == 2 || nvec == 4 || nvec == 8 || nvec == 10 || nvec == 16)) {
    const int64_t groups = ceil_div(H.n, H.block_rows);
    const int64_t grid = ceil_div(groups, kXcds) * kXcds;
#define BBL_BLK_CASE(BV)                                                                      \
  case BV: {                                                                                  \
    auto kern = k_spmm_blk<VT, XT, AT, YT, BV, LPR>;                                          \
    if (lds > 65536) {                                                                        \
      static bool attr_set = false;                                                           \
      if (!attr_set) {                                                                        \
        BBL_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),                     \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,               \
                                    (int)kBlkMaxLds));                                        \
        attr_set = true;                                                                      \
      }                                                                                       \
    }                                                                                         \
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kBlkThreads), lds, s, H.n,            \
                       (int64_t)H.block_rows, H.row_ptr, H.col, valp, X, Y);                  \
    break;                                                                                    \
  }
    switch (nvec) {
      BBL_BLK_CASE(1)
      BBL_BLK_CASE(2)
      BBL_BLK_CASE(4)
      BBL_BLK_CASE(8)
      BBL_BLK_CASE(10)
      BBL_BLK_CASE(16)
      default: break;
    }
#undef BBL_BLK_CASE
    check_launch("k_spmm_blk");
    return;
  }
  const int rows_per_wg = (256 / kWave) * (kWave / LPR);
  const int64_t grid = ceil_div(ceil_div(H.n, rows_per_wg), kXcds) * kXcds;
  const VT *val = static_cast<const VT *>(H.val);
#define BBL_SPMM_CASE(BV)                                                                        \
  case BV:                                                                                       \
    hipLaunchKernelGGL((k_spmm<VT, XT, AT, YT, BV, LPR>), dim3(grid), dim3(256), 0, s, H.n,     \
                       H.row_ptr, H.col, val, X, Y);                                             \
    break;
  switch (nvec) {
    BBL_SPMM_CASE(1)
    BBL_SPMM_CASE(2)
    BBL_SPMM_CASE(4)
    BBL_SPMM_CASE(8)
    BBL_SPMM_CASE(10)
    BBL_SPMM_CASE(16)
    default:
      hipLaunchKernelGGL((k_spmm_generic<VT, XT, AT, YT, LPR>), dim3(grid), dim3(256), 0, s, H.n,
                         H.row_ptr, H.col, val, X, Y, nvec);
  }
#undef BBL_SPMM_CASE
  check_launch("k_spmm");
}

template <typename VT, typename XT, typename AT, typename YT>
void spmm_dispatch(const bbl_csr &H, const XT *X, YT *Y, int nvec, hipStream_t s) {
  switch (pick_lpr(H)) {
    case 16: spmm_dispatch_b<VT, XT, AT, YT, 16>(H, X, Y, nvec, s); break;
    case 32: spmm_dispatch_b<VT, XT, AT, YT, 32>(H, X, Y, nvec, s); break;
    default: spmm_dispatch_b<VT, XT, AT, YT, 64>(H, X, Y, nvec, s); break;
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

int launch_residual_spmm(const bbl_csr &H, const double *X, int nvec, const double *theta,
                         double *partial, int max_partials, hipStream_t s) {
  const int lpr = pick_lpr(H);
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

}  // namespace bbl
