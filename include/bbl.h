/*
 * bbl.h -- C ABI of libbbl.so: bootstrapped block Lanczos on one AMD MI355X.
 *
 * The library finds the lowest k eigenpairs of a real symmetric sparse matrix H
 * with the block Lanczos method of Zbikowski & Johnson, "Bootstrapped Block
 * Lanczos for large-dimension eigenvalue problems" (arXiv 2210.15763), Methods
 * section, started either from a random pivot block or from a "bootstrapped"
 * pivot block made of eigenvectors of a truncated leading block of H.
 *
 * Conventions shared by every entry point
 *  - Every call returns a bbl_status; nothing throws across the ABI.  On a
 *    non-OK status bbl_last_error() returns a thread-local message.
 *  - "device" pointers are HIP device memory owned by the caller (allocated,
 *    e.g., by PyTorch); the library never frees them and never allocates device
 *    memory on the solve path: all scratch comes from a caller-provided
 *    workspace whose size is given by the matching *_workspace_size() call.
 *  - "host" pointers are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Device outputs are ordered on it; a call returns after its host outputs
 *    are written.
 *  - Blocks of vectors are row-major n x nvec arrays: the nvec entries of one
 *    row are contiguous (the paper's v(a, j) with the block index fastest,
 *    equivalently the transposed block W^T it stores row-wise).
 *  - A CSR matrix has int64 row pointers, int32 column indices ascending within
 *    each row, and float32 or float64 values; it must be exactly symmetric.
 */
#ifndef BBL_H
#define BBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BBL_OK = 0,
  BBL_E_INVALID = -1,       /* an argument is out of range or inconsistent */
  BBL_E_NOMEM = -2,         /* workspace smaller than the size query returned */
  BBL_E_HIP = -3,           /* a HIP runtime call failed */
  BBL_E_NOT_CONVERGED = -4, /* block cap reached; outputs hold current Ritz pairs */
  BBL_E_BREAKDOWN = -5      /* unrecoverable loss of rank in the block QR */
} bbl_status;

typedef enum { BBL_F32 = 1, BBL_F64 = 2 } bbl_dtype;

/* Symmetric CSR matrix resident on the device. */
typedef struct {
  int64_t n;              /* dimension, >= 1 */
  int64_t nnz;            /* number of stored entries (row_ptr[n]) */
  const int64_t *row_ptr; /* device, n + 1 entries, row_ptr[0] = 0 */
  const int32_t *col;     /* device, nnz entries, ascending within each row */
  const void *val;        /* device, nnz entries of type val_dtype */
  int32_t val_dtype;      /* BBL_F32 or BBL_F64 */
  int32_t reserved;       /* must be 0 */
} bbl_csr;

/* Solver options; a NULL pointer selects the defaults shown. */
typedef struct {
  int32_t m_max;        /* block iteration cap (default 200) */
  int32_t basis_dtype;  /* storage and SpMM precision of the Krylov basis:
                           BBL_F32 (default for float32 H) or BBL_F64 */
  int32_t check_every;  /* solve the band matrix every this many blocks; 0 = auto */
  int32_t flags;        /* bitwise OR of BBL_FLAG_* (default 0) */
  double defl_tau;      /* deflation threshold on singular values of the
                           residual block relative to max(sigma_max, ||H||)
                           (default 1e-12) */
  uint64_t seed;        /* key of random replacement directions (default 0) */
} bbl_opts;

/* Option flags.  BBL_FLAG_TIME_SPMM records a pair of HIP events on the
   solver's stream around every product H V_j of the block recurrence and
   reports their summed duration in bbl_stats.spmm_ms (costs two event
   records per block). */
#define BBL_FLAG_TIME_SPMM 1

/* Counters of one solve and its wall time (host clock around the call). */
typedef struct {
  int32_t iters;        /* block iterations (products H V_j) */
  int32_t spmm_calls;   /* all products with H, explicit residual checks included */
  int32_t deflations;   /* columns replaced because of (near) rank loss */
  int32_t converged;    /* 1 if every wanted pair met the tolerance */
  int32_t checks;       /* band-matrix eigensolves */
  int32_t reorth_second_passes; /* blocks that needed a second Gram-Schmidt sweep */
  double hnorm_est;     /* largest |Ritz value| of the final band matrix */
  double t_total_ms;    /* wall time of the call */
  double spmm_ms;       /* summed device time of the recurrence's products H V_j
                           (BBL_FLAG_TIME_SPMM only, else 0) */
  int32_t spmm_timed;   /* number of products in spmm_ms */
  int32_t reserved;
} bbl_stats;

/* Message describing the last non-OK status on the calling thread. */
const char *bbl_last_error(void);

/* Library version string. */
const char *bbl_version(void);

/*
 * W = H V  -- the block sparse product w_{a,i} = sum_j H_ij v_{a,j} (Methods,
 * "Block Lanczos algorithm"), every matrix element loaded once per block.
 *   H        device CSR (float32 or float64 values)
 *   V, W     device n x nvec row-major blocks of vec_dtype; must not overlap
 *   nvec     1..32
 *   vec_dtype BBL_F32: float32 values and vectors required, float32
 *            accumulation.  BBL_F64: float64 vectors, float64 accumulation
 *            (float32 values are promoted).
 * Errors: BBL_E_INVALID for a bad shape/dtype/NULL pointer, BBL_E_HIP.
 */
int bbl_spmm(const bbl_csr *H, const void *V, void *W, int32_t nvec, int32_t vec_dtype,
             void *stream);

/*
 * Workspace bytes needed by bbl_block_lanczos for dimension n, block size
 * nvec, k_eig wanted pairs, block cap m_max and basis precision basis_dtype.
 * Returns 0 for invalid arguments.
 */
size_t bbl_lanczos_workspace_size(int64_t n, int32_t nvec, int32_t k_eig, int32_t m_max,
                                  int32_t basis_dtype);

/*
 * Lowest k_eig eigenpairs of H by non-restarted block Lanczos (Methods): the
 * block recurrence H V_j = V_{j-1} B_{j-1}^T + V_j A_j + V_{j+1} B_j with
 * A_j = V_j^T H V_j, full reorthogonalisation of every new block against all
 * stored blocks, a block QR of the residual block giving B_j and V_{j+1}, and
 * the block-tridiagonal band matrix of the A's and B's solved for its lowest
 * Ritz pairs.
 *   pivot    device n x nvec float64 starting block (any full-rank block;
 *            rank loss is repaired by deflation)
 *   nvec     block size, 1..32;  k_eig 1..min(n, 32, nvec * m_max)
 *   tol      convergence: ||H x_i - theta_i x_i||_2 <= tol * ||H||_est for all
 *            i < k_eig, ||H||_est = max |Ritz value| of the band matrix
 *   ws       device workspace of ws_bytes >= bbl_lanczos_workspace_size(...)
 *   eigvals  host, k_eig ascending Ritz values
 *   eigvecs  device n x k_eig float64 row-major; columns of unit 2-norm whose
 *            largest-magnitude entry is positive (may be NULL)
 *   residuals host, k_eig explicit residual norms in float64 (may be NULL)
 *   stats    host (may be NULL)
 * Returns BBL_OK on convergence, BBL_E_NOT_CONVERGED at the cap (outputs hold
 * the current Ritz pairs and their true residuals), or an error.
 */
int bbl_block_lanczos(const bbl_csr *H, const double *pivot, int32_t nvec, int32_t k_eig,
                      double tol, void *ws, size_t ws_bytes, const bbl_opts *opts,
                      double *eigvals, double *eigvecs, double *residuals, bbl_stats *stats,
                      void *stream);

/*
 * Workspace bytes for bbl_bootstrap_pivot (reads row_ptr[n_trunc] from the
 * device, hence the stream).  Returns 0 for invalid arguments.
 */
size_t bbl_bootstrap_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t nvec,
                                    int32_t m_max, int32_t basis_dtype, void *stream);

/*
 * Bootstrapped pivot block (Methods, last paragraphs): approximate lowest
 * eigenvectors computed in a much smaller space and carried into the full one.
 * The smaller space is the leading principal block H[0:n_trunc, 0:n_trunc];
 * its lowest nvec eigenvectors are found by block Lanczos from a random pivot
 * (key opts->seed + 1) to the same tolerance, then zero-padded to n rows.
 *   n_trunc  nvec..n;  tol as in bbl_block_lanczos
 *   pivot    device n x nvec float64 output, orthonormal columns
 *   stats    host, statistics of the truncated solve (may be NULL)
 */
int bbl_bootstrap_pivot(const bbl_csr *H, int64_t n_trunc, int32_t nvec, double tol, void *ws,
                        size_t ws_bytes, const bbl_opts *opts, double *pivot, bbl_stats *stats,
                        void *stream);

/*
 * Random pivot block: n x nvec float64 N(0,1) entries, entry (i, a) from
 * Philox4x32-10 counter (i, a, tag 6) under the 64-bit key, Box-Muller
 * (cosine branch).  The conventional block Lanczos start the paper compares
 * against.  Device output; no workspace.
 */
int bbl_random_pivot(int64_t n, int32_t nvec, uint64_t key, double *pivot, void *stream);

/*
 * Eigenpairs of a symmetric band matrix (diagnostic entry point for the
 * band-matrix solve used inside bbl_block_lanczos).
 *   band     device N x (kd+1) float64, band[i*(kd+1)+d] = T[i][i-d]
 *   k        number of lowest eigenpairs, 1..min(N, 32)
 *   theta    host k ascending eigenvalues;  S device N x k eigenvectors
 *   top      host, largest eigenvalue (may be NULL)
 *   ws       device workspace of ws_bytes >= bbl_band_eig_workspace_size(N, kd, k)
 */
size_t bbl_band_eig_workspace_size(int32_t N, int32_t kd, int32_t k);
int bbl_band_eig(const double *band, int32_t N, int32_t kd, int32_t k, void *ws, size_t ws_bytes,
                 double *theta, double *S, double *top, void *stream);

/*
 * Tall-skinny products of the block recurrence on FP64 matrix cores
 * (diagnostic entry points for the kernels bbl_block_lanczos uses for
 * A_n = V_n^T W_n, the reorthogonalisation coefficients and the overlap
 * O = W'^T W' of the Methods section, and for W' = W - V_n A_n - ...).
 *   X     device: nblk blocks of width bx, block i a row-major n x bx array at
 *         X + i*n*bx elements (the Krylov-basis layout), type xdtype
 *   Y     device n x ny row-major, type ydtype (ny 1..32)
 * bbl_gram:   C (device, (nblk*bx) x ny float64) = X^T Y, summed in a fixed
 *             order; ws is scratch of ws_bytes >= bbl_gram_workspace_size(...)
 * bbl_block_update: Yout = beta*Yin + alpha*X*C, C device (nblk*bx) x ny
 *             float64; Yout may equal Yin (and may equal X when nblk == 1).
 */
size_t bbl_gram_workspace_size(int64_t n, int32_t bx, int32_t nblk, int32_t ny);
int bbl_gram(int64_t n, const void *X, int32_t xdtype, int32_t bx, int32_t nblk, const void *Y,
             int32_t ydtype, int32_t ny, double *C, void *ws, size_t ws_bytes, void *stream);
int bbl_block_update(int64_t n, const void *X, int32_t xdtype, int32_t bx, int32_t nblk,
                     const double *C, int32_t ny, double alpha, const void *Yin, int32_t yindtype,
                     double beta, void *Yout, int32_t youtdtype, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BBL_H */
