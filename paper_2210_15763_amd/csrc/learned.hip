// Learned pivot proposer.  The paper builds the pivot block from eigenvectors
// of a truncated leading block and observes that such a pivot misses target
// states whose weight lies outside the truncation (Methods, last paragraphs;
// Results, bootstrapped runs).  It does not describe a learned proposer; this
// file implements one on the GPU:
//
//   features  per row: standardised diagonal, a fixed 16-value Fourier
//             encoding of the row's sector, the degree, and sqrt(n) times the
//             row of P_D -- the 10 lowest Ritz vectors of H on the one-hop
//             extension of the 20 lowest truncated eigenvectors
//             (y_ia = (H P)_ia / (theta_a - H_ii) outside the truncation);
//   network   residual form: the 10 P_D amplitudes of the row plus a
//             correction by 28 -> 128 -> 128 -> 128 -> 10 with ReLU, BF16
//             operands on v_mfma_f32_16x16x16bf16_1k, FP32 accumulation, FP32
//             master weights (output layer initialised to zero, so training
//             starts from P_D itself); one fused kernel for inference, one for
//             the gradient;
//   training  Adam on FP32 master weights; targets are converged eigenvectors
//             aligned to P_D by orthogonal Procrustes and scaled by sqrt(n);
//   fallback  the plain bootstrap block replaces the learned one when the
//             learned block has a non-finite entry, a Cholesky pivot of its
//             Gram matrix below 1e-8 of the largest diagonal entry, or a sum
//             of k lowest Rayleigh-Ritz values not below the bootstrap's.
//
// MFMA layout (16x16x16 bf16, wave64): A[i][k] at lane i + 16 (k / 4),
// element k % 4; B[k][j] at lane j + 16 (k / 4), element k % 4; D[i][j] at
// lane j + 16 (i / 4), element i % 4.
#include <chrono>
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "driver.h"
#include "philox.h"
#include "small.h"

namespace bbl {
namespace {

constexpr int kIn = 28, kInPad = 32, kHid = 128, kOut = 10, kOutPad = 16;
constexpr int kParams = 38026;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid * kHid, oW4 = oB3 + kHid,
              oB4 = oW4 + kOut * kHid;
static_assert(oB4 + kOut == kParams, "parameter layout");
constexpr int kTrunc = 2 * kOut;      // default count of truncated eigenvectors extended one hop
// truncated eigenvectors of the feature block: opts->feature_vectors, else 2 * 10
inline int trunc_vectors(const Opts &o) { return o.feature_vectors > 0 ? o.feature_vectors : kTrunc; }
constexpr int kTruncMax = kMaxBlock;  // the workspaces hold this many
constexpr int kSkip = 18;             // first P_D amplitude among the inputs (residual form)
constexpr int SA = kInPad + 8;        // LDS row strides (bf16 elements), padded
constexpr int SH = kHid + 8;          //   against bank conflicts
constexpr int SO = kOutPad + 8;
constexpr int kFwdRows = 64;          // rows per tile, inference
constexpr int kGradRows = 32;         // rows per tile, gradient
constexpr int kGradSlots = 256;       // workgroups (partial gradients) at most
constexpr int kMaxPartialRows = 4096;

typedef uint16_t bf16;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even; NaN stays a (quiet) NaN
__device__ inline bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (bf16)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ inline float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }
// ReLU that keeps NaN (so broken weights reach the output and the fallback)
__device__ inline float relu(float v) { return v > 0.f ? v : (v == v ? 0.f : v); }

__device__ inline f4 mma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline s4 ld4(const bf16 *p) { return *reinterpret_cast<const s4 *>(p); }
__device__ inline s4 ld4s(const bf16 *p, int stride) {
  s4 r;
  r[0] = (short)p[0];
  r[1] = (short)p[stride];
  r[2] = (short)p[2 * stride];
  r[3] = (short)p[3 * stride];
  return r;
}

// Network weights in LDS as bf16 (zero padded), biases as FP32.
struct SWeights {
  bf16 w1[kHid * SA], w2[kHid * SH], w3[kHid * SH], w4[kOutPad * SH];
  float b1[kHid], b2[kHid], b3[kHid], b4[kOutPad];
};

__device__ void load_weights(const float *__restrict__ p, SWeights &w) {
  for (int i = threadIdx.x; i < kHid * SA; i += blockDim.x) {
    const int r = i / SA, c = i % SA;
    w.w1[i] = c < kIn ? f2bf(p[oW1 + r * kIn + c]) : (bf16)0;
  }
  for (int i = threadIdx.x; i < kHid * SH; i += blockDim.x) {
    const int r = i / SH, c = i % SH;
    w.w2[i] = c < kHid ? f2bf(p[oW2 + r * kHid + c]) : (bf16)0;
    w.w3[i] = c < kHid ? f2bf(p[oW3 + r * kHid + c]) : (bf16)0;
  }
  for (int i = threadIdx.x; i < kOutPad * SH; i += blockDim.x) {
    const int r = i / SH, c = i % SH;
    w.w4[i] = (r < kOut && c < kHid) ? f2bf(p[oW4 + r * kHid + c]) : (bf16)0;
  }
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    w.b1[i] = p[oB1 + i];
    w.b2[i] = p[oB2 + i];
    w.b3[i] = p[oB3 + i];
  }
  for (int i = threadIdx.x; i < kOutPad; i += blockDim.x) w.b4[i] = i < kOut ? p[oB4 + i] : 0.f;
}

// out[r][j] = relu(sum_k in[r][k] W[j][k] + b[j]) for r < TR, j < N, as bf16.
// 16x16 output tiles are split evenly over the four waves.
template <int TR, int K, int N>
__device__ void layer_fwd(const bf16 *in, int sin, const bf16 *W, int sw, const float *bias,
                          bf16 *out, int sout) {
  constexpr int RT = TR / 16, T = RT * (N / 16), PER = (T + 3) / 4;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = 4 * (l >> 4);
  f4 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = w * PER + u;
      if (t < T) {
        const int rt = t % RT, ct = t / RT;
        acc[u] = mma(ld4(in + (rt * 16 + li) * sin + k0 + lk),
                     ld4(W + (ct * 16 + li) * sw + k0 + lk), acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = w * PER + u;
    if (t < T) {
      const int rt = t % RT, ct = t / RT;
      const int col = ct * 16 + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rt * 16 + lk + q;
        out[row * sout + col] = f2bf(relu(acc[u][q] + bias[col]));
      }
    }
  }
}

// Output layer: calls f(row, col, value) for the 16-wide padded output.
template <int TR, typename F>
__device__ void layer_out(const bf16 *in, const SWeights &w, F &&f) {
  constexpr int RT = TR / 16;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = l & 15, lk = 4 * (l >> 4);
  for (int rt = wv; rt < RT; rt += 4) {
    f4 acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < kHid; k0 += 16)
      acc = mma(ld4(in + (rt * 16 + li) * SH + k0 + lk), ld4(w.w4 + li * SH + k0 + lk), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) f(rt * 16 + lk + q, li, acc[q] + w.b4[li]);
  }
}

// Loads rows [r0, r0 + TR) of the features (or the rows idx[r0..]) into LDS.
template <int TR>
__device__ void load_rows(const bf16 *__restrict__ X, int64_t rows, int64_t r0,
                          const int64_t *__restrict__ idx, bf16 *dst) {
  for (int i = threadIdx.x; i < TR * SA; i += blockDim.x) {
    const int r = i / SA, c = i % SA;
    const int64_t g = r0 + r;
    bf16 v = 0;
    if (g < rows && c < kIn) v = X[(idx ? idx[g] : g) * kIn + c];
    dst[i] = v;
  }
}

// Inference: out[r][0..10) for all rows; persistent workgroups, weights staged
// once per workgroup.
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ params,
                                                     const bf16 *__restrict__ X, int64_t rows,
                                                     float *__restrict__ out) {
  __shared__ SWeights w;
  __shared__ bf16 sX[kFwdRows * SA], sA[kFwdRows * SH], sB[kFwdRows * SH];
  load_weights(params, w);
  for (int64_t r0 = (int64_t)blockIdx.x * kFwdRows; r0 < rows;
       r0 += (int64_t)gridDim.x * kFwdRows) {
    __syncthreads();
    load_rows<kFwdRows>(X, rows, r0, nullptr, sX);
    __syncthreads();
    layer_fwd<kFwdRows, kInPad, kHid>(sX, SA, w.w1, SA, w.b1, sA, SH);
    __syncthreads();
    layer_fwd<kFwdRows, kHid, kHid>(sA, SH, w.w2, SH, w.b2, sB, SH);
    __syncthreads();
    layer_fwd<kFwdRows, kHid, kHid>(sB, SH, w.w3, SH, w.b3, sA, SH);
    __syncthreads();
    // residual form: the P_D amplitudes (inputs 18..27) plus the network
    layer_out<kFwdRows>(sA, w, [&](int r, int c, float v) {
      if (c < kOut && r0 + r < rows) out[(r0 + r) * kOut + c] = v + bf2f(sX[r * SA + kSkip + c]);
    });
  }
}

// G[i][j] += sum_r D[r][i] X[r][j] over the TR rows of a tile, i < NI, j < NJ
// (tiles of 16); accumulated into this workgroup's FP32 partial (row stride
// ldg, only i < ni, j < nj stored).  Every element has one owning lane, so the
// read-modify-write needs no atomics and is deterministic.
template <int TR, int NI, int NJ>
__device__ void wgrad(const bf16 *D, int sd, const bf16 *X, int sx, float *__restrict__ g,
                      int ldg, int ni, int nj) {
  constexpr int IT = NI / 16, T = IT * (NJ / 16), PER = (T + 3) / 4;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = 4 * (l >> 4);
  f4 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < TR; k0 += 16) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = w * PER + u;
      if (t < T) {
        const int it = t % IT, jt = t / IT;
        acc[u] = mma(ld4s(D + (k0 + lk) * sd + it * 16 + li, sd),
                     ld4s(X + (k0 + lk) * sx + jt * 16 + li, sx), acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = w * PER + u;
    if (t < T) {
      const int it = t % IT, jt = t / IT;
      const int j = jt * 16 + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = it * 16 + lk + q;
        if (i < ni && j < nj) g[i * ldg + j] += acc[u][q];
      }
    }
  }
}

// out[r][j] = (sum_i D[r][i] W[i][j]) * (H[r][j] > 0), i < NI, j < NJ, bf16.
template <int TR, int NI, int NJ>
__device__ void backprop(const bf16 *D, int sd, const bf16 *W, int sw, const bf16 *H, int sh,
                         bf16 *out, int sout) {
  constexpr int RT = TR / 16, T = RT * (NJ / 16), PER = (T + 3) / 4;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = 4 * (l >> 4);
  f4 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < NI; k0 += 16) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = w * PER + u;
      if (t < T) {
        const int rt = t % RT, jt = t / RT;
        acc[u] = mma(ld4(D + (rt * 16 + li) * sd + k0 + lk),
                     ld4s(W + (k0 + lk) * sw + jt * 16 + li, sw), acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = w * PER + u;
    if (t < T) {
      const int rt = t % RT, jt = t / RT;
      const int j = jt * 16 + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rt * 16 + lk + q;
        out[r * sout + j] = bf2f(H[r * sh + j]) > 0.f ? f2bf(acc[u][q]) : (bf16)0;
      }
    }
  }
}

// bias gradient: g[j] += sum_r D[r][j] for j < n (one owning thread per j)
template <int TR>
__device__ void bgrad(const bf16 *D, int sd, float *__restrict__ g, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    float s = 0.f;
    for (int r = 0; r < TR; ++r) s += bf2f(D[r * sd + j]);
    g[j] += s;
  }
}

// Gradient of the mean squared error over `rows` rows (features X, or the
// rows idx[] of X when idx is given) into per-workgroup partials.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ params,
                                                  const bf16 *__restrict__ X,
                                                  const float *__restrict__ T, int64_t rows,
                                                  const int64_t *__restrict__ idx, float scale,
                                                  float *__restrict__ partial,
                                                  double *__restrict__ loss_part) {
  __shared__ SWeights w;
  __shared__ bf16 s0[kGradRows * SA], s1[kGradRows * SH], s2[kGradRows * SH], s3[kGradRows * SH];
  __shared__ bf16 sD[kGradRows * SH], sE[kGradRows * SH];
  __shared__ double sl[256];
  float *g = partial + (int64_t)blockIdx.x * kParams;
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) g[i] = 0.f;
  load_weights(params, w);
  double lsum = 0.0;
  for (int64_t r0 = (int64_t)blockIdx.x * kGradRows; r0 < rows;
       r0 += (int64_t)gridDim.x * kGradRows) {
    __syncthreads();
    load_rows<kGradRows>(X, rows, r0, idx, s0);
    __syncthreads();
    layer_fwd<kGradRows, kInPad, kHid>(s0, SA, w.w1, SA, w.b1, s1, SH);
    __syncthreads();
    layer_fwd<kGradRows, kHid, kHid>(s1, SH, w.w2, SH, w.b2, s2, SH);
    __syncthreads();
    layer_fwd<kGradRows, kHid, kHid>(s2, SH, w.w3, SH, w.b3, s3, SH);
    __syncthreads();
    // output layer and d loss / d out = scale * (out - target)
    layer_out<kGradRows>(s3, w, [&](int r, int c, float v) {
      const int64_t gr = r0 + r;
      float d = 0.f;
      if (c < kOut && gr < rows) {
        const float diff = v + bf2f(s0[r * SA + kSkip + c]) - T[(idx ? idx[gr] : gr) * kOut + c];
        lsum += (double)diff * diff;
        d = scale * diff;
      }
      sD[r * SO + c] = f2bf(d);
    });
    __syncthreads();
    wgrad<kGradRows, kOutPad, kHid>(sD, SO, s3, SH, g + oW4, kHid, kOut, kHid);
    bgrad<kGradRows>(sD, SO, g + oB4, kOut);
    backprop<kGradRows, kOutPad, kHid>(sD, SO, w.w4, SH, s3, SH, sE, SH);
    __syncthreads();
    wgrad<kGradRows, kHid, kHid>(sE, SH, s2, SH, g + oW3, kHid, kHid, kHid);
    bgrad<kGradRows>(sE, SH, g + oB3, kHid);
    backprop<kGradRows, kHid, kHid>(sE, SH, w.w3, SH, s2, SH, sD, SH);
    __syncthreads();
    wgrad<kGradRows, kHid, kHid>(sD, SH, s1, SH, g + oW2, kHid, kHid, kHid);
    bgrad<kGradRows>(sD, SH, g + oB2, kHid);
    backprop<kGradRows, kHid, kHid>(sD, SH, w.w2, SH, s1, SH, sE, SH);
    __syncthreads();
    wgrad<kGradRows, kHid, kInPad>(sE, SH, s0, SA, g + oW1, kIn, kHid, kIn);
    bgrad<kGradRows>(sE, SH, g + oB1, kHid);
  }
  sl[threadIdx.x] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) s += sl[i];
    loss_part[blockIdx.x] = s;
  }
}

// grad[p] = sum over slots (fixed order); loss = sum of loss partials / count
__global__ void k_mlp_grad_reduce(const float *__restrict__ partial, int slots,
                                  const double *__restrict__ loss_part, double inv_count,
                                  float *__restrict__ grad, float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) {
    float s = 0.f;
    for (int k = 0; k < slots; ++k) s += partial[(int64_t)k * kParams + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    double s = 0.0;
    for (int k = 0; k < slots; ++k) s += loss_part[k];
    *loss = (float)(s * inv_count);
  }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// He-uniform weights (bound sqrt(6 / fan_in)), zero biases; Philox counter
// (index, 0, 0, 11) under the caller's key.
__global__ void k_mlp_init(float *__restrict__ p, uint64_t key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  // hidden layers He-uniform; the output layer (and every bias) zero, so an
  // untrained network returns the P_D amplitudes unchanged
  int fan = 0;
  if (i < oB1) fan = kIn;
  else if (i >= oW2 && i < oB2) fan = kHid;
  else if (i >= oW3 && i < oB3) fan = kHid;
  if (fan == 0) {
    p[i] = 0.f;
    return;
  }
  U4 c;
  c.v[0] = (uint32_t)i;
  c.v[1] = 0;
  c.v[2] = 0;
  c.v[3] = 11;
  const U4 r = philox4x32_10(c, (uint32_t)key, (uint32_t)(key >> 32));
  const double u = u53(r.v[0], r.v[1]);
  p[i] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan));
}

// Uniform row sample with replacement: idx[r] from Philox counter
// (r, step, 0, 12), reduced modulo the dataset size.
__global__ void k_sample(int64_t batch, int64_t total, uint64_t key, uint32_t step,
                         int64_t *__restrict__ idx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= batch) return;
  U4 c;
  c.v[0] = (uint32_t)r;
  c.v[1] = (uint32_t)((uint64_t)r >> 32);
  c.v[2] = step;
  c.v[3] = 12;
  const U4 o = philox4x32_10(c, (uint32_t)key, (uint32_t)(key >> 32));
  const uint64_t x = ((uint64_t)o.v[0] << 32) | o.v[1];
  idx[r] = (int64_t)(x % (uint64_t)total);
}

// ------------------------------------------------------------- features
__global__ void k_diag(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                       const void *__restrict__ val, int f32, double *__restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = rp[i], hi = rp[i + 1];
    double v = 0.0;
    while (lo < hi) {  // first position with col >= i
      const int64_t mid = (lo + hi) >> 1;
      if (col[mid] < i) lo = mid + 1;
      else hi = mid;
    }
    if (lo < rp[i + 1] && col[lo] == i)
      v = f32 ? (double)static_cast<const float *>(val)[lo] : static_cast<const double *>(val)[lo];
    d[i] = v;
  }
}

// mode 0: partial sums of d; mode 1: of (d - mean)^2.  Contiguous row ranges
// per workgroup, fixed-order tree inside it.
__global__ __launch_bounds__(256) void k_stat_partial(int64_t n, const double *__restrict__ d,
                                                      int mode, const double *__restrict__ mean,
                                                      double *__restrict__ partial) {
  __shared__ double sh[256];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = blockIdx.x * per, b = min(n, a + per);
  const double mu = mode ? *mean : 0.0;
  double s = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    const double x = d[i] - mu;
    s += mode ? x * x : x;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// out = sum(partial) / n  (mode 0: mean) or sqrt(sum / n) (mode 1: std)
__global__ void k_stat_final(const double *__restrict__ partial, int P, int64_t n, int mode,
                             double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < P; ++i) s += partial[i];
  s /= (double)n;
  *out = mode ? sqrt(s) : s;
}

// Y = [P; (H P)_out / clamp(theta - H_ii)] for the m columns (row-major n x m)
__global__ void k_extend(int64_t n, int64_t n_t, int m, const double *__restrict__ P,
                         const double *__restrict__ HP, const double *__restrict__ theta,
                         const double *__restrict__ d, double *__restrict__ Y) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * m;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / m;
    const int a = (int)(idx - i * m);
    if (i < n_t) {
      Y[idx] = P[idx];
      continue;
    }
    double den = theta[a] - d[i];
    if (fabs(den) < 1.0) den = den < 0.0 ? -1.0 : 1.0;
    Y[idx] = HP[idx] / den;
  }
}

__global__ void k_features(int64_t n, int64_t R, const int64_t *__restrict__ rp, double zbar,
                           const double *__restrict__ d, const double *__restrict__ stats,
                           const double *__restrict__ PD, bf16 *__restrict__ F,
                           float *__restrict__ F32) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float f[kIn];
    f[0] = (float)((d[i] - stats[0]) / stats[1]);
    const int64_t S = (n + R - 1) / R;
    const double base = 6.283185307179586476925 * (double)(i / R) / (double)S;
#pragma unroll
    for (int q = 1; q <= 8; ++q) {
      double sn, cs;
      sincos(base * q, &sn, &cs);
      f[2 * q - 1] = (float)sn;
      f[2 * q] = (float)cs;
    }
    f[17] = (float)((double)(rp[i + 1] - rp[i]) / zbar);
    const double sq = sqrt((double)n);
#pragma unroll
    for (int a = 0; a < kOut; ++a) f[18 + a] = (float)(sq * PD[i * kOut + a]);
#pragma unroll
    for (int c = 0; c < kIn; ++c) F[i * kIn + c] = f2bf(f[c]);
    if (F32)
#pragma unroll
      for (int c = 0; c < kIn; ++c) F32[i * kIn + c] = f[c];
  }
}

// dst[i][a] = src[i][a] for a < mc (src row stride ms, dst row stride md)
template <typename S, typename D>
__global__ void k_copy_cols(int64_t n, int mc, const S *__restrict__ src, int ms,
                            D *__restrict__ dst, int md) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * mc;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / mc;
    const int a = (int)(idx - i * mc);
    dst[i * md + a] = (D)src[i * ms + a];
  }
}

// Rayleigh-Ritz on span(Y) from G = Y^T Y and K = Y^T H Y (m <= 32): whitening
// Sw = U Lambda^{-1/2} (G = U Lambda U^T), eig(Sw^T K Sw) = Z Theta Z^T,
// C = Sw Z.  theta[0..m) ascending, C[0..m)[0..keep) row-major; flag[0] = 1
// if G is not positive definite.
__global__ __launch_bounds__(64) void k_rr_small(const double *__restrict__ Gin,
                                                 const double *__restrict__ Kin, int m, int keep,
                                                 double *__restrict__ theta,
                                                 double *__restrict__ C, int *__restrict__ flag) {
  __shared__ double G[32 * 32], K[32 * 32], U[32 * 32], A[32 * 32], Z[32 * 32];
  __shared__ double lg[32], lt[32], cs[4];
  const int t = threadIdx.x;
  for (int i = t; i < m * m; i += blockDim.x) {
    const int r = i / m, c = i % m;
    G[i] = 0.5 * (Gin[r * m + c] + Gin[c * m + r]);
    K[i] = 0.5 * (Kin[r * m + c] + Kin[c * m + r]);
  }
  __syncthreads();
  wg_jacobi_eig(G, U, lg, m, cs);
  __syncthreads();
  const bool bad = !(lg[0] > 1e-300 * fabs(lg[m - 1])) || !(lg[0] > 0.0);
  if (t == 0 && flag) flag[0] = bad ? 1 : 0;
  // Sw in U (scale columns), then A = Sw^T K Sw via Z as scratch
  for (int i = t; i < m * m; i += blockDim.x) U[i] /= sqrt(fmax(lg[i % m], 1e-300));
  __syncthreads();
  for (int i = t; i < m * m; i += blockDim.x) {  // Z = K Sw
    const int r = i / m, c = i % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += K[r * m + k] * U[k * m + c];
    Z[i] = s;
  }
  __syncthreads();
  for (int i = t; i < m * m; i += blockDim.x) {  // A = Sw^T Z
    const int r = i / m, c = i % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += U[k * m + r] * Z[k * m + c];
    A[i] = s;
  }
  __syncthreads();
  for (int i = t; i < m * m; i += blockDim.x) {
    const int r = i / m, c = i % m;
    G[i] = 0.5 * (A[r * m + c] + A[c * m + r]);
  }
  __syncthreads();
  wg_jacobi_eig(G, Z, lt, m, cs);
  __syncthreads();
  for (int i = t; i < m * keep; i += blockDim.x) {  // C = Sw Z[:, :keep]
    const int r = i / keep, c = i % keep;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += U[r * m + k] * Z[k * m + c];
    C[i] = s;
  }
  for (int i = t; i < m; i += blockDim.x) theta[i] = lt[i];
}

// Fallback checks on a pivot block P (n x b) from G = P^T P, K = P^T H P:
// out[0] = 1 if a non-finite entry, out[1] = 1 if a squared Cholesky pivot of G
// is not above 1e-8 max_i G_ii, out[2] = sum of the k lowest Ritz values.
__global__ __launch_bounds__(64) void k_pivot_check(const double *__restrict__ Gin,
                                                    const double *__restrict__ Kin, int b, int k,
                                                    double *__restrict__ out) {
  __shared__ double G[32 * 32], K[32 * 32], U[32 * 32], A[32 * 32], Z[32 * 32];
  __shared__ double lg[32], lt[32], cs[4];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) {
    int nf = 0;
    for (int i = 0; i < b * b; ++i) nf |= !isfinite(Gin[i]) || !isfinite(Kin[i]);
    int cf = 0;
    if (!nf) {
      double *L = A;  // Cholesky factor, row stride 32
      double gmax = 0.0;
      for (int i = 0; i < b; ++i) gmax = fmax(gmax, Gin[i * b + i]);
      for (int j = 0; j < b && !cf; ++j) {
        double piv = Gin[j * b + j];
        for (int q = 0; q < j; ++q) piv -= L[j * 32 + q] * L[j * 32 + q];
        if (!(piv > 1e-8 * gmax)) {
          cf = 1;
          break;
        }
        L[j * 32 + j] = sqrt(piv);
        for (int i = j + 1; i < b; ++i) {
          double s = Gin[i * b + j];
          for (int q = 0; q < j; ++q) s -= L[i * 32 + q] * L[j * 32 + q];
          L[i * 32 + j] = s / L[j * 32 + j];
        }
      }
    }
    out[0] = nf;
    out[1] = cf;
    out[2] = NAN;
    bad = nf | cf;
  }
  __syncthreads();
  if (bad) return;
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    G[i] = 0.5 * (Gin[r * b + c] + Gin[c * b + r]);
    K[i] = 0.5 * (Kin[r * b + c] + Kin[c * b + r]);
  }
  __syncthreads();
  wg_jacobi_eig(G, U, lg, b, cs);
  __syncthreads();
  for (int i = t; i < b * b; i += blockDim.x) U[i] /= sqrt(lg[i % b]);
  __syncthreads();
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    double s = 0.0;
    for (int q = 0; q < b; ++q) s += K[r * b + q] * U[q * b + c];
    Z[i] = s;
  }
  __syncthreads();
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    double s = 0.0;
    for (int q = 0; q < b; ++q) s += U[q * b + r] * Z[q * b + c];
    A[i] = s;
  }
  __syncthreads();
  for (int i = t; i < b * b; i += blockDim.x) {
    const int r = i / b, c = i % b;
    G[i] = 0.5 * (A[r * b + c] + A[c * b + r]);
  }
  __syncthreads();
  wg_jacobi_eig(G, Z, lt, b, cs);
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int i = 0; i < min(k, b); ++i) s += lt[i];
    out[2] = s;
  }
}

// Orthogonal polar factor Q = M (M^T M)^{-1/2} of an m x m matrix (m <= 32).
__global__ __launch_bounds__(64) void k_polar(const double *__restrict__ Min, int m,
                                              double *__restrict__ Q, int *__restrict__ flag) {
  __shared__ double M[32 * 32], A[32 * 32], U[32 * 32], Z[32 * 32];
  __shared__ double lam[32], cs[4];
  const int t = threadIdx.x;
  for (int i = t; i < m * m; i += blockDim.x) M[i] = Min[i];
  __syncthreads();
  for (int i = t; i < m * m; i += blockDim.x) {
    const int r = i / m, c = i % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += M[k * m + r] * M[k * m + c];
    A[i] = s;
  }
  __syncthreads();
  wg_jacobi_eig(A, U, lam, m, cs);
  __syncthreads();
  if (t == 0 && flag) flag[0] = (lam[0] > 0.0) ? 0 : 1;
  for (int i = t; i < m * m; i += blockDim.x) {  // Z = U Lambda^{-1/2} U^T
    const int r = i / m, c = i % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += U[r * m + k] * U[c * m + k] / sqrt(fmax(lam[k], 1e-300));
    Z[i] = s;
  }
  __syncthreads();
  for (int i = t; i < m * m; i += blockDim.x) {
    const int r = i / m, c = i % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += M[r * m + k] * Z[k * m + c];
    Q[i] = s;
  }
}

// ------------------------------------------------------------- host side
// kernels launched on grid_for(n ...) stride over their work
unsigned grid_for(int64_t work, int threads = 256) {
  return capped_grid(ceil_div(work, threads), threads);
}

// Workspace carve-up helper.
struct Arena {
  char *base;
  size_t off = 0, cap;
  Arena(void *ws, size_t bytes) : cap(bytes) {
    base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    cap = bytes > 256 ? bytes - 256 : 0;
  }
  template <typename T>
  T *take(size_t count) {
    const size_t o = off;
    off += align_up(count * sizeof(T));
    if (base && off > cap) throw Error{BBL_E_NOMEM, "workspace too small"};
    return reinterpret_cast<T *>(base + o);
  }
};

// partial-sum capacity for the small grams here (<= 32 x 32 results)
size_t gram_ws_doubles() { return (size_t)4096 * kMaxBlock * kMaxBlock * 9 / 8 + 65536; }

// C = X^T Y (M x ny, X n x M, Y n x ny, both FP64 row-major)
void gram64(int64_t n, const double *X, int M, const double *Y, int ny, double *partial,
            double *C, hipStream_t s) {
  const int mp = gram_max_partials(gram_ws_doubles(), M, ny);
  const int P = launch_gram(n, X, BBL_F64, M, 1, (int64_t)n * M, Y, BBL_F64, ny, partial, mp, s);
  launch_reduce(partial, P, M, ny, C, s);
}

struct FeatBufs {
  double *Ppad, *HP, *Y, *PD, *d, *small, *partial;
  int *flag;
  void *trunc;
  size_t trunc_bytes;
};

int check_trunc_vectors(const Opts &o, int64_t n_trunc, int64_t n) {
  const int mt = trunc_vectors(o);
  BBL_REQUIRE(mt >= kOut && mt <= kTruncMax, "feature_vectors must be 0 or in 10..32");
  BBL_REQUIRE(n_trunc >= mt && n_trunc <= n, "n_trunc must be in feature_vectors..n");
  return mt;
}

size_t feature_bytes(const bbl_csr &H, int64_t n_t, const Opts &o, hipStream_t s, FeatBufs *fb,
                     void *ws, size_t ws_bytes) {
  const int64_t n = H.n;
  const int mt = kTruncMax;  // room for any feature_vectors setting
  const size_t tb = truncated_ws_bytes(H, n_t, kOut, mt, o, s);
  Arena a(ws, ws ? ws_bytes : 0);
  if (!ws) a.base = nullptr;
  FeatBufs b{};
  b.Ppad = a.take<double>((size_t)n * mt);
  b.HP = a.take<double>((size_t)n * mt);
  b.Y = a.take<double>((size_t)n * mt);
  b.PD = a.take<double>((size_t)n * kOut);
  b.d = a.take<double>((size_t)n);
  b.small = a.take<double>(4096);
  b.flag = a.take<int>(64);
  b.partial = a.take<double>(std::max(gram_ws_doubles(), normalize_scratch_bytes(kOut, kMaxPartialRows) / 8 + 1));
  b.trunc = a.take<char>(tb);
  b.trunc_bytes = tb;
  if (fb) *fb = b;
  return a.off + 256;
}

// Builds P_D (and optionally the features) for H; returns the Ritz values of
// P_D on the host.  Ppad keeps the 20 truncated eigenvectors, zero padded.
void build_features(const bbl_csr &H, int64_t n_t, int64_t R, double tol, const Opts &o,
                    const FeatBufs &b, bf16 *F, float *F32, double *theta_d, bbl_stats *stats,
                    hipStream_t s) {
  const int64_t n = H.n;
  const int mt = trunc_vectors(o);
  std::vector<double> th(mt);
  const int st = truncated_solve(H, n_t, kOut, mt, tol, o, b.trunc, b.trunc_bytes, b.Ppad,
                                 th.data(), stats, s);
  if (st != BBL_OK && st != BBL_E_NOT_CONVERGED)
    throw Error{st, "truncated solve failed: " + std::string(bbl_last_error())};
  // the truncated solve's products, then H P and H Y at width 2 * 10
  if (stats) stats->pivot_spmm_calls = stats->spmm_calls + 2 * (mt / kOut);
  if (n > n_t) launch_fill(b.Ppad + (size_t)n_t * mt, (n - n_t) * mt, 0.0, s);
  double *dtheta = b.small;           // [0, 32): truncated eigenvalues
  double *G = b.small + 64;           // [64, 64 + 1024)
  double *K = b.small + 64 + 1024;    // [1088, 2112)
  double *C = b.small + 2112;         // [2112, 3136)
  double *thd = b.small + 3136;       // [3136, 3168)
  double *mean = b.small + 3200, *stats2 = b.small + 3200;  // mean, std
  double *spart = b.small + 3264;     // 256 partials
  BBL_HIP(hipMemcpyAsync(dtheta, th.data(), mt * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_diag, dim3(grid_for(n)), dim3(256), 0, s, n, H.row_ptr, H.col, H.val,
                     H.val_dtype == BBL_F32 ? 1 : 0, b.d);
  launch_spmm(H, b.Ppad, BBL_F64, b.HP, BBL_F64, mt, s);
  hipLaunchKernelGGL(k_extend, dim3(grid_for(n * mt)), dim3(256), 0, s, n, n_t, mt,
                     b.Ppad, b.HP, dtheta, b.d, b.Y);
  launch_spmm(H, b.Y, BBL_F64, b.HP, BBL_F64, mt, s);  // HP <- H Y
  gram64(n, b.Y, mt, b.Y, mt, b.partial, G, s);
  gram64(n, b.Y, mt, b.HP, mt, b.partial, K, s);
  hipLaunchKernelGGL(k_rr_small, dim3(1), dim3(64), 0, s, G, K, mt, kOut, thd, C, b.flag);
  launch_update(n, b.Y, BBL_F64, mt, 1, (int64_t)n * mt, C, kOut, 1.0, nullptr, BBL_F64,
                0.0, b.PD, BBL_F64, s);
  launch_normalize_columns(n, kOut, b.PD, b.partial, kMaxPartialRows, s);
  int flag = 0;
  std::vector<double> thh(mt);
  BBL_HIP(hipMemcpyAsync(&flag, b.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BBL_HIP(hipMemcpyAsync(thh.data(), thd, kOut * sizeof(double), hipMemcpyDeviceToHost, s));
  BBL_HIP(hipStreamSynchronize(s));
  if (flag) throw Error{BBL_E_BREAKDOWN, "extended truncated block is rank deficient"};
  if (theta_d)
    for (int i = 0; i < kOut; ++i) theta_d[i] = thh[i];
  if (F) {
    const int P = 256;
    hipLaunchKernelGGL(k_stat_partial, dim3(P), dim3(256), 0, s, n, b.d, 0, nullptr, spart);
    hipLaunchKernelGGL(k_stat_final, dim3(1), dim3(64), 0, s, spart, P, n, 0, mean);
    hipLaunchKernelGGL(k_stat_partial, dim3(P), dim3(256), 0, s, n, b.d, 1, mean, spart);
    hipLaunchKernelGGL(k_stat_final, dim3(1), dim3(64), 0, s, spart, P, n, 1, stats2 + 1);
    const double zbar = (double)H.nnz / (double)n;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n)), dim3(256), 0, s, n, R, H.row_ptr, zbar, b.d,
                       stats2, b.PD, F, F32);
  }
  check_launch("features");
}

void mlp_forward(const float *params, const bf16 *F, int64_t rows, float *out, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, kFwdRows), 1024));
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, s, params, F, rows, out);
  check_launch("k_mlp_forward");
}

size_t grad_bytes(int64_t rows) {
  const int slots = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, kGradRows), kGradSlots));
  return align_up((size_t)slots * kParams * 4) + align_up((size_t)slots * 8) + 256;
}

void mlp_grad(const float *params, const bf16 *F, const float *T, int64_t rows,
              const int64_t *idx, void *ws, float *grad, float *loss, hipStream_t s) {
  const int slots = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, kGradRows), kGradSlots));
  char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
  float *partial = reinterpret_cast<float *>(base);
  double *lp = reinterpret_cast<double *>(base + align_up((size_t)slots * kParams * 4));
  const float scale = (float)(2.0 / ((double)rows * kOut));
  hipLaunchKernelGGL(k_mlp_grad, dim3(slots), dim3(256), 0, s, params, F, T, rows, idx, scale,
                     partial, lp);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3(grid_for(kParams)), dim3(256), 0, s, partial, slots,
                     lp, 1.0 / ((double)rows * kOut), grad, loss);
  check_launch("k_mlp_grad");
}

void adam(float *p, float *m, float *v, const float *g, int64_t count, int step, float lr,
          float b1, float b2, float eps, hipStream_t s) {
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(count)), dim3(256), 0, s, p, m, v, g, count, lr, b1,
                     b2, eps, c1, c2);
  check_launch("k_adam");
}

}  // namespace
}  // namespace bbl

using namespace bbl;

extern "C" {

size_t bbl_features_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t m_max,
                                   int32_t basis_dtype, void *stream) {
  size_t r = 0;
  const int st = guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(n_trunc >= kTrunc && n_trunc <= H->n, "n_trunc must be in 20..n");
    BBL_REQUIRE(m_max >= 2, "m_max must be >= 2");
    Opts o;
    o.m_max = m_max;
    o.basis_dtype = basis_dtype;
    r = feature_bytes(*H, n_trunc, o, static_cast<hipStream_t>(stream), nullptr, nullptr, 0);
    return (int)BBL_OK;
  });
  return st == BBL_OK ? r : 0;
}

int bbl_pivot_features(const bbl_csr *H, int64_t n_trunc, int64_t sector_size, double tol,
                       void *ws, size_t ws_bytes, const bbl_opts *opts, uint16_t *feats,
                       float *feats32, double *p_d, double *p_boot, double *theta_d,
                       bbl_stats *stats, void *stream) {
  return guarded([&] {
    validate_csr(H);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BBL_REQUIRE(sector_size >= 1, "sector_size must be >= 1");
    BBL_REQUIRE(feats && ws, "feats/workspace is NULL");
    BBL_REQUIRE(tol > 0.0, "tol must be > 0");
    const auto t0 = std::chrono::steady_clock::now();
    const Opts o = read_opts(opts, H->val_dtype);
    const int mt = check_trunc_vectors(o, n_trunc, H->n);
    FeatBufs b{};
    const size_t need = feature_bytes(*H, n_trunc, o, s, &b, ws, ws_bytes);
    if (ws_bytes < need) throw Error{BBL_E_NOMEM, "features workspace too small"};
    build_features(*H, n_trunc, sector_size, tol, o, b, feats, feats32, theta_d, stats, s);
    const int64_t n = H->n;
    if (p_d)
      BBL_HIP(hipMemcpyAsync(p_d, b.PD, (size_t)n * kOut * 8, hipMemcpyDeviceToDevice, s));
    if (p_boot)
      hipLaunchKernelGGL((k_copy_cols<double, double>), dim3(grid_for(n * kOut)), dim3(256), 0, s,
                         n, kOut, b.Ppad, mt, p_boot, kOut);
    BBL_HIP(hipStreamSynchronize(s));
    if (stats)
      stats->t_pivot_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return (int)BBL_OK;
  });
}

size_t bbl_procrustes_workspace_size(int64_t n, int32_t m) {
  if (n < 1 || m < 1 || m > kMaxBlock) return 0;
  return (gram_ws_doubles() + 4096) * 8 + 1024;
}

int bbl_procrustes_targets(const double *X, const double *P, int64_t n, int32_t m, void *ws,
                           size_t ws_bytes, float *targets, void *stream) {
  return guarded([&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    BBL_REQUIRE(X && P && targets && ws, "NULL argument");
    BBL_REQUIRE(n >= 1 && m >= 1 && m <= kMaxBlock, "bad n/m");
    if (ws_bytes < bbl_procrustes_workspace_size(n, m))
      throw Error{BBL_E_NOMEM, "procrustes workspace too small"};
    char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    double *Mt = reinterpret_cast<double *>(base);
    double *Q = Mt + 1024;
    int *flag = reinterpret_cast<int *>(Q + 1024);
    double *partial = Mt + 4096;
    gram64(n, X, m, P, m, partial, Mt, s);
    hipLaunchKernelGGL(k_polar, dim3(1), dim3(64), 0, s, Mt, m, Q, flag);
    launch_update(n, X, BBL_F64, m, 1, (int64_t)n * m, Q, m, std::sqrt((double)n), nullptr,
                  BBL_F64, 0.0, targets, BBL_F32, s);
    int f = 0;
    BBL_HIP(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    BBL_HIP(hipStreamSynchronize(s));
    if (f) throw Error{BBL_E_BREAKDOWN, "X^T P is singular"};
    return (int)BBL_OK;
  });
}

int bbl_mlp_init(float *params, uint64_t seed, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(params != nullptr, "params is NULL");
    hipLaunchKernelGGL(k_mlp_init, dim3(grid_for(kParams)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, seed);
    check_launch("k_mlp_init");
    return (int)BBL_OK;
  });
}

int bbl_mlp_forward(const float *params, const uint16_t *feats, int64_t rows, float *out,
                    void *stream) {
  return guarded([&] {
    BBL_REQUIRE(params && feats && out, "NULL argument");
    BBL_REQUIRE(rows >= 0, "rows must be >= 0");
    if (rows > 0) mlp_forward(params, feats, rows, out, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_mlp_grad_workspace_size(int64_t rows) {
  if (rows < 1) return 0;
  return grad_bytes(rows);
}

int bbl_mlp_grad(const float *params, const uint16_t *feats, const float *targets, int64_t rows,
                 void *ws, size_t ws_bytes, float *grad, float *loss, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(params && feats && targets && ws && grad, "NULL argument");
    BBL_REQUIRE(rows >= 1, "rows must be >= 1");
    if (ws_bytes < grad_bytes(rows)) throw Error{BBL_E_NOMEM, "gradient workspace too small"};
    mlp_grad(params, feats, targets, rows, nullptr, ws, grad, loss,
             static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

int bbl_adam_step(float *params, float *m, float *v, const float *grad, int64_t count,
                  int32_t step, float lr, float beta1, float beta2, float eps, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(params && m && v && grad, "NULL argument");
    BBL_REQUIRE(count >= 1 && step >= 1, "count and step must be >= 1");
    adam(params, m, v, grad, count, step, lr, beta1, beta2, eps,
         static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_mlp_train_workspace_size(int64_t batch) {
  if (batch < 1) return 0;
  return grad_bytes(batch) + align_up((size_t)batch * 8) + align_up((size_t)kParams * 4) + 512;
}

int bbl_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                       const uint16_t *feats, const float *targets, int64_t dataset_rows,
                       int64_t batch, uint64_t sample_key, void *ws, size_t ws_bytes,
                       float *loss, void *stream) {
  return guarded([&] {
    hipStream_t s = static_cast<hipStream_t>(stream);
    BBL_REQUIRE(params && adam_m && adam_v && feats && targets && ws, "NULL argument");
    BBL_REQUIRE(dataset_rows >= 1 && batch >= 1 && step >= 1, "bad sizes");
    if (ws_bytes < bbl_mlp_train_workspace_size(batch))
      throw Error{BBL_E_NOMEM, "training workspace too small"};
    char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    int64_t *idx = reinterpret_cast<int64_t *>(base);
    float *grad = reinterpret_cast<float *>(base + align_up((size_t)batch * 8));
    char *gws = base + align_up((size_t)batch * 8) + align_up((size_t)kParams * 4);
    hipLaunchKernelGGL(k_sample, dim3(grid_for(batch)), dim3(256), 0, s, batch, dataset_rows,
                       sample_key, (uint32_t)step, idx);
    mlp_grad(params, feats, targets, batch, idx, gws, grad, loss, s);
    adam(params, adam_m, adam_v, grad, kParams, step, lr, 0.9f, 0.999f, 1e-8f, s);
    return (int)BBL_OK;
  });
}

size_t bbl_learned_pivot_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t nvec,
                                        int32_t m_max, int32_t basis_dtype, void *stream) {
  size_t r = 0;
  const int st = guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(nvec >= 1 && nvec <= kOut, "nvec must be in 1..10");
    BBL_REQUIRE(n_trunc >= kTrunc && n_trunc <= H->n, "n_trunc must be in 20..n");
    Opts o;
    o.m_max = m_max;
    o.basis_dtype = basis_dtype;
    const int64_t n = H->n;
    r = feature_bytes(*H, n_trunc, o, static_cast<hipStream_t>(stream), nullptr, nullptr, 0) +
        align_up((size_t)n * kIn * 2) + align_up((size_t)n * kOut * 4) +
        3 * align_up((size_t)n * nvec * 8) + 8192;
    return (int)BBL_OK;
  });
  return st == BBL_OK ? r : 0;
}

int bbl_learned_pivot(const bbl_csr *H, const float *params, int64_t n_trunc, int64_t sector_size,
                      int32_t nvec, int32_t k, double tol, void *ws, size_t ws_bytes,
                      const bbl_opts *opts, double *pivot, int32_t *used_fallback,
                      double *rr_sums, bbl_stats *stats, void *stream) {
  return guarded([&] {
    validate_csr(H);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BBL_REQUIRE(params && pivot && ws, "NULL argument");
    BBL_REQUIRE(nvec >= 1 && nvec <= kOut, "nvec must be in 1..10");
    BBL_REQUIRE(k >= 1, "k must be >= 1");
    BBL_REQUIRE(sector_size >= 1, "sector_size must be >= 1");
    const auto t0 = std::chrono::steady_clock::now();
    const Opts o = read_opts(opts, H->val_dtype);
    const int mt = check_trunc_vectors(o, n_trunc, H->n);
    const int64_t n = H->n;
    FeatBufs b{};
    const size_t fb = feature_bytes(*H, n_trunc, o, s, &b, ws, ws_bytes);
    Arena a(reinterpret_cast<char *>(ws) + fb, ws_bytes > fb ? ws_bytes - fb : 0);
    bf16 *F = a.take<bf16>((size_t)n * kIn);
    float *out = a.take<float>((size_t)n * kOut);
    double *Pl = a.take<double>((size_t)n * nvec);
    double *Pb = a.take<double>((size_t)n * nvec);
    double *HPx = a.take<double>((size_t)n * nvec);
    double *chk = a.take<double>(512);
    double thd[kOut];
    build_features(*H, n_trunc, sector_size, tol, o, b, F, nullptr, thd, stats, s);
    mlp_forward(params, F, n, out, s);
    hipLaunchKernelGGL((k_copy_cols<float, double>), dim3(grid_for(n * nvec)), dim3(256), 0, s, n,
                       nvec, out, kOut, Pl, nvec);
    hipLaunchKernelGGL((k_copy_cols<double, double>), dim3(grid_for(n * nvec)), dim3(256), 0, s,
                       n, nvec, b.Ppad, mt, Pb, nvec);
    // Rayleigh-Ritz checks of both blocks: chk[0..3) learned, chk[3..6) bootstrap
    double *G = chk + 8, *K = chk + 8 + 128;
    const double *blocks[2] = {Pl, Pb};
    for (int q = 0; q < 2; ++q) {
      launch_spmm(*H, blocks[q], BBL_F64, HPx, BBL_F64, nvec, s);
      gram64(n, blocks[q], nvec, blocks[q], nvec, b.partial, G, s);
      gram64(n, blocks[q], nvec, HPx, nvec, b.partial, K, s);
      hipLaunchKernelGGL(k_pivot_check, dim3(1), dim3(64), 0, s, G, K, nvec, k, chk + 3 * q);
    }
    double h[6];
    BBL_HIP(hipMemcpyAsync(h, chk, sizeof(h), hipMemcpyDeviceToHost, s));
    BBL_HIP(hipStreamSynchronize(s));
    // P_D's columns are Ritz vectors of H: on their span H is diagonal, so the
    // sum of its k lowest Rayleigh-Ritz values is the sum of its own
    double sd = 0.0;
    for (int i = 0; i < std::min(k, nvec); ++i) sd += thd[i];
    const bool learn_ok = h[0] == 0.0 && h[1] == 0.0;
    int choice;  // 0 learned, 1 bootstrap, 2 P_D
    if (learn_ok && h[2] < h[5] && h[2] < sd) choice = 0;
    else if (sd < h[5]) choice = 2;
    else choice = 1;
    if (choice == 2)
      hipLaunchKernelGGL((k_copy_cols<double, double>), dim3(grid_for(n * nvec)), dim3(256), 0, s,
                         n, nvec, b.PD, kOut, pivot, nvec);
    else
      BBL_HIP(hipMemcpyAsync(pivot, choice == 1 ? Pb : Pl, (size_t)n * nvec * 8,
                             hipMemcpyDeviceToDevice, s));
    BBL_HIP(hipStreamSynchronize(s));
    if (used_fallback) *used_fallback = choice;
    if (rr_sums) {
      rr_sums[0] = h[2];
      rr_sums[1] = h[5];
      rr_sums[2] = sd;
    }
    if (stats) {
      stats->pivot_spmm_calls += 2;  // H P_learn and H P_boot of the selection
      stats->used_fallback = choice;
      stats->t_pivot_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return (int)BBL_OK;
  });
}

}  // extern "C"
