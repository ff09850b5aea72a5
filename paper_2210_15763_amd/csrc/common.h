// Shared declarations of the bbl HIP library (kernels + host driver).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/bbl.h"

namespace bbl {

// ------------------------------------------------------------- error state
void set_error(const std::string &msg);

struct Error {
  int code;
  std::string msg;
};

#define BBL_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::bbl::Error{BBL_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define BBL_REQUIRE(cond, msg)                               \
  do {                                                       \
    if (!(cond)) throw ::bbl::Error{BBL_E_INVALID, (msg)};   \
  } while (0)

inline void check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{BBL_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

constexpr int kMaxBlock = 32;    // largest supported block size / k
constexpr int kWave = 64;
constexpr int kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2

// Capacity (doubles) of a partial-sum buffer for gram products with at most
// Mmax columns of X and ny <= nyw columns of Y, including the reduction's
// second-stage scratch.
inline size_t gram_partial_doubles(int64_t Mmax, int nyw) {
  return ((size_t)524288 + 4 * (size_t)Mmax + 8192) * nyw * 9 / 8 + 65536;
}
// Largest partial count a gram over M x ny may produce in such a buffer.
inline int gram_max_partials(size_t cap_doubles, int M, int ny) {
  const size_t per = (size_t)M * ny;
  const size_t p = cap_doubles * 8 / 9 / per;
  return (int)(p > 1 ? p - 1 : 1);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// The dispatch packet holds a launch's size per dimension in work-items
// (grid x workgroup) as a 32-bit count.  Launches whose grid grows with n stay
// at or below this many work-items: their kernels stride over the rows, or
// the rows are split over several launches.
constexpr int64_t kMaxLaunchItems = (int64_t)1 << 31;
inline unsigned capped_grid(int64_t blocks, int threads) {
  const int64_t cap = kMaxLaunchItems / threads;
  return (unsigned)(blocks < 1 ? 1 : blocks < cap ? blocks : cap);
}

// ---------------------------------------------------------- kernel launchers
// SpMM: Y = H X (templated on value/vector/accumulator types inside).
void launch_spmm(const bbl_csr &H, const void *X, int xdtype, void *Y, int ydtype, int nvec,
                 hipStream_t s);
// Planned SpMM (rows reordered per aligned group, partner blocks staged in LDS).
constexpr int kPlanMaxSlots = 5;                 // column blocks staged per group
constexpr size_t kPlanLds = 160 * 1024;          // LDS bytes they may take (all of it)
int spmm_plan_slots(const bbl_csr &H, int nvec, int vec_dtype);
size_t spmm_plan_bytes(const bbl_csr &H, int nvec, int vec_dtype);
void build_spmm_plan(const bbl_csr &H, int nvec, int vec_dtype, void *mem, size_t bytes,
                     bbl_spmm_plan *P, hipStream_t s);
void launch_spmm_planned(const bbl_spmm_plan &P, const void *X, void *Y, hipStream_t s);
// Explicit residual: partial[g][c] = sum over the rows of group g of
// ((H X)_{r,c} - theta_c X_{r,c})^2, float64 accumulation.  Returns the number
// of partial rows written.
int launch_residual_spmm(const bbl_csr &H, const double *X, int nvec, const double *theta,
                         double *partial, int max_partials, hipStream_t s);

// Tall-skinny products on FP64 MFMA.
//   X: nblk column blocks of width bx, block b at X + b * xstride (row-major
//      n x bx each), element type xdtype.  M = nblk * bx columns in total.
//   Y: n x ny row-major, element type ydtype.
// gram: partial[p][m][c] = sum over chunk p of X[r][m] * Y[r][c]; returns P.
int launch_gram(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                const void *Y, int ydtype, int ny, double *partial, int max_partials,
                hipStream_t s);
// out[m][c] = scale * sum_p partial[p][m][c]   (M x ny)
void launch_reduce(const double *partial, int P, int M, int ny, double *out, hipStream_t s);
// Yout = beta * Yin + alpha * X C   (C: M x ny float64, Yout type ydtype)
void launch_update(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                   const double *C, int ny, double alpha, const void *Yin, int yindtype,
                   double beta, void *Yout, int youtdtype, hipStream_t s);

// Small dense kernels (one workgroup).
void launch_fill(double *p, int64_t count, double v, hipStream_t s);
// *p = v (one lane; a kernel, so it may be recorded into a graph)
void launch_store_int(int *p, int v, hipStream_t s);
// *dd = *ds and *id = *is in one launch (a one-thread kernel)
void launch_copy_pair(double *dd, const double *ds, int *id, const int *is, hipStream_t s);

// Random normal block (Philox4x32-10 + Box-Muller), entry (i, a) from counter
// (i, a + col0, tag).
void launch_gauss(int64_t n, int nvec, int ld, int col0, uint64_t key, uint32_t tag,
                  double *out, const int32_t *colmask, const int *when, hipStream_t s);

// Variants whose kernels return at once when *when == 0 (device flag), so a
// data-dependent branch needs no host round trip.
int launch_gram_when(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                     const void *Y, int ydtype, int ny, double *partial, int max_partials,
                     const int *when, hipStream_t s);
void launch_reduce_when(const double *partial, int P, int M, int ny, double *out,
                        const int *when, hipStream_t s);
void launch_update_when(int64_t n, const void *X, int xdtype, int bx, int nblk, int64_t xstride,
                        const double *C, int ny, double alpha, const void *Yin, int yindtype,
                        double beta, void *Yout, int youtdtype, const int *when, hipStream_t s);
// The update above, also leaving the Gram partials of Yout (as stored) in
// gpart[p][a][c], p < the returned count, for launch_reduce_when(.., ny, ny);
// returns 0 when this shape has no fused Gram or gcap_doubles is too small
// (then only the update ran).
int launch_update_gram_when(int64_t n, const void *X, int xdtype, int bx, int nblk,
                            int64_t xstride, const double *C, int ny, double alpha,
                            const void *Yin, int yindtype, double beta, void *Yout, int youtdtype,
                            double *gpart, size_t gcap_doubles, const int *when, hipStream_t s);

}  // namespace bbl
