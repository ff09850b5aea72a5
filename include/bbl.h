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

/* Symmetric CSR matrix resident on the device.
 * block_rows is an optional locality hint: when > 0, the rows come in aligned
 * groups [g*block_rows, (g+1)*block_rows) (sectors of the basis, e.g. blocks of
 * fixed quantum numbers) and most of a row's columns fall inside a few column
 * blocks of the same size.  Only the planned SpMM uses it (bbl_spmm_plan_size,
 * bbl_spmm_plan_build, bbl_spmm_planned: column blocks staged in the 160 KB
 * of LDS); bbl_spmm and the solver's plain kernel ignore it, and the result
 * does not depend on it beyond rounding.  0 = no hint. */
typedef struct {
  int64_t n;              /* dimension, >= 1 */
  int64_t nnz;            /* number of stored entries (row_ptr[n]) */
  const int64_t *row_ptr; /* device, n + 1 entries, row_ptr[0] = 0 */
  const int32_t *col;     /* device, nnz entries, ascending within each row */
  const void *val;        /* device, nnz entries of type val_dtype */
  int32_t val_dtype;      /* BBL_F32 or BBL_F64 */
  int32_t block_rows;     /* locality hint (see above), >= 0 */
} bbl_csr;

/* Prepared form of a matrix with a block_rows hint for the SpMM of the block
 * recurrence (built by bbl_spmm_plan_build; all pointers are device memory
 * inside the caller's plan buffer, except row_ptr, which is H's).  For every
 * aligned row group the plan names up to five column blocks of block_rows
 * columns (set A) -- the group's own and the partner blocks holding most of
 * its other entries -- and every row's entries are reordered: entries inside
 * those blocks first, stored as an LDS row index slot*block_rows + offset,
 * then the others with their global column.  When every LDS row index fits
 * in 16 bits and nnz < 2^31 the plan also names the next busiest blocks (set
 * B, as many as set A), places each row's set-B entries right after its set-A
 * entries, keeps the LDS index of set-A and set-B entries within their set as
 * uint16 (lcol), per-row entry ranges (rdesc), dense copies of the set-A and
 * set-B entries and the list of rows with entries outside both sets.  The
 * FP32 planned SpMM at nvec 4, 8 or 10 then runs one workgroup per group
 * over set A and then set B, each staged in LDS, and a last pass over the
 * listed rows that gathers the rows of V their remaining entries need; at
 * nvec 16 it does so twice, for columns 0-7 and 8-15 (the slot count is
 * then sized for 8 columns).  Otherwise one pass stages set A and gathers
 * the rest.  The same sums are
 * formed in a different order, so results agree with bbl_spmm to rounding,
 * not bitwise. */
typedef struct {
  int64_t n, nnz;
  int32_t block_rows;     /* rows (and columns) per group */
  int32_t slots;          /* column blocks staged per group, 1..5 */
  int32_t nvec;           /* block width the plan serves */
  int32_t vec_dtype;      /* vector element type it serves */
  int32_t val_dtype;      /* matrix value type */
  int32_t local16;        /* 1 if lcol is present (slots*block_rows <= 65536) */
  const int64_t *row_ptr; /* H.row_ptr (not copied; H must outlive the plan) */
  const int32_t *blocks;  /* [groups][slots] staged block ids (set A), or
                             [groups][2 slots] (set A, then set B) when lcol
                             and rdesc are present; -1 = none */
  const int32_t *n_local; /* [n] entries of the row inside staged blocks */
  const int32_t *col;     /* [nnz] reordered column / LDS row indices */
  const void *val;        /* [nnz] reordered values */
  const uint16_t *lcol;   /* [nnz] LDS row index within its set of every set-A
                             and set-B entry (others unspecified), or NULL */
  const int32_t *rdesc;   /* [n][4] per row: first entry, first set-B entry,
                             first remaining entry and end, as offsets from the
                             group's first entry rounded down to a multiple of 8;
                             present with lcol when nnz < 2^31, else NULL */
  /* Dense copies of the set-A and set-B entries (present with rdesc, else
   * NULL), read by the first and second passes of the FP32 SpMM: each
   * group's rows in order with no gaps. */
  const int64_t *agroup;  /* [groups + 1] first set-A copy entry of each group's rows */
  const int32_t *arow;    /* [n][2] first and end set-A copy entry of each row, relative
                             to its group's first rounded down to a multiple of 8 */
  const uint16_t *alcol;  /* [nnz + 16] LDS index within set A of each copied entry */
  const void *aval;       /* [nnz + 16] its value (val_dtype) */
  const int64_t *bgroup;  /* [groups + 1] first set-B copy entry of each group's rows */
  const int32_t *brow;    /* [n][2] first and end copy entry of each row, relative
                             to its group's first rounded down to a multiple of 8 */
  const uint16_t *blcol;  /* [nnz + 16] LDS index within set B of each copied entry */
  const void *bval;       /* [nnz + 16] its value (val_dtype) */
  /* The rows with entries outside both sets (present with rdesc): group g's
   * are rlist[rgroup[g] .. rgroup[g + 1]), each {row, count, first entry as
   * two 32-bit words (low, high)}; their entries are the row's last. */
  const int64_t *rgroup;  /* [groups + 1] */
  const int32_t *rlist;   /* [n][4] */
  /* Multi-set layout (nsets > 0; the fields from n_local to brow are then
   * NULL): when fewer than three column blocks fit in LDS per set (e.g.
   * 2000-row groups at 8 float32 columns; at 16 columns, blocks of 16-wide
   * rows where one fits beside the all-zero row, else of 8-column halves) or
   * the entries need 64-bit offsets, the group's busiest blocks form nsets
   * sets of `slots` blocks
   * (blocks: [groups][nsets * slots]), staged in LDS one set after the other.
   * Each set keeps a dense copy of its entries (16-bit LDS index within the
   * set, value; the copies lie set after set, group after group, rows in
   * order); the entries outside every set are kept compactly (global
   * column, value) and listed per row in rgroup / rlist, whose first-entry
   * field indexes rcol / rval.  The plan takes 8 (nnz + 16) bytes for the
   * entries, about as much as H's own arrays, plus per-row descriptors. */
  int32_t nsets;
  int32_t reserved;
  const int64_t *sgroup;  /* [nsets][groups + 1] first copy entry of each group's set-s entries */
  const int32_t *srow;    /* [nsets][n][2] first and end copy entry of each row, relative to
                             its group's first rounded down to a multiple of 8 */
  const uint16_t *slcol;  /* LDS index within its set of every copied entry */
  const void *sval;       /* its value (float32) */
  const int32_t *rcol;    /* global column of every entry outside the sets */
  const void *rval;       /* its value */
} bbl_spmm_plan;

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
  const bbl_spmm_plan *spmm_plan; /* optional plan of H for the recurrence's SpMM
                           (its nvec and vec_dtype must equal the solve's block
                           width and basis type); NULL = plain CSR kernel */
  int32_t restart_keep; /* thick restart (see bbl_block_lanczos): Ritz vectors
                           kept when the basis reaches m_max blocks, a multiple
                           of nvec in [max(k_eig, nvec), min(32, nvec*(m_max-2))];
                           0 (default) = no restart, stop at m_max.  The pivot
                           calls raise it to cover their own pair count. */
  int32_t max_restarts; /* restarts before giving up (0 = default 100) */
  int32_t fault_block;  /* testing only, 0 (default) = off.  f > 0 forces the
                           failure-handling path from the host: block f-1 is
                           marked as having lost rank beyond repair, and block
                           f as needing the second Gram-Schmidt sweep (so it is
                           redone); the solve must then return BBL_E_BREAKDOWN */
  int32_t feature_vectors; /* learned-pivot features: lowest truncated eigenvectors
                           extended one hop before the Rayleigh-Ritz step that
                           selects P_D, 10..32 (0 = default 20) */
  int32_t reserved;
} bbl_opts;

/* Option flags.  BBL_FLAG_TIME_SPMM records a pair of HIP events on the
   solver's stream around every product H V_j of the block recurrence and
   reports their summed duration in bbl_stats.spmm_ms (costs two event
   records per block).  BBL_FLAG_TIME_PHASES also times the three-term step,
   the reorthogonalisation, the block QR, the band eigensolves of the
   convergence checks (on their own stream, concurrent with the recurrence)
   and the thick restarts, filling the t_*_ms fields of bbl_stats. */
#define BBL_FLAG_TIME_SPMM 1
#define BBL_FLAG_TIME_PHASES 2

/* Counters of one solve and its wall time (host clock around the call). */
typedef struct {
  int32_t iters;        /* block iterations (products H V_j of the recurrence)
                           that built the space the returned pairs come from,
                           over all thick-restart cycles (the recurrence may
                           have built a few more while the last check ran
                           beside it: up to two, or four when n < 2^19, whose
                           blocks are short next to the check's band
                           eigensolve) */
  int32_t spmm_calls;   /* all products with H, explicit residual checks and
                           the blocks built beside the last check included */
  int32_t deflations;   /* columns replaced because of (near) rank loss */
  int32_t converged;    /* 1 if every wanted pair met the tolerance */
  int32_t checks;       /* band-matrix eigensolves */
  int32_t reorth_second_passes; /* blocks that needed a second Gram-Schmidt sweep */
  double hnorm_est;     /* largest |Ritz value| of the final band matrix */
  double t_total_ms;    /* wall time of the call */
  double spmm_ms;       /* summed device time of the recurrence's products H V_j
                           (BBL_FLAG_TIME_SPMM or _PHASES, else 0) */
  int32_t spmm_timed;   /* number of products in spmm_ms */
  int32_t restarts;     /* thick restarts performed */
  /* Device time per phase (BBL_FLAG_TIME_PHASES, else 0), summed over every
   * block instance the recurrence ran, redone and discarded ones included. */
  double t_threeterm_ms; /* A_j = V_j^T W and W - V_j A_j - V_{j-1} B_{j-1}^T */
  double t_reorth_ms;    /* full reorthogonalisation against the stored blocks */
  double t_qr_ms;        /* block QR: B_j and V_{j+1} */
  double t_eig_ms;       /* band eigensolves (concurrent with the recurrence) */
  double t_restart_ms;   /* thick restarts: Ritz vectors and the new band matrix */
  /* Pivot calls (bbl_bootstrap_pivot, bbl_pivot_features, bbl_learned_pivot)
   * fill these; a solve sets them to 0. */
  double t_pivot_ms;     /* wall time of the pivot call */
  int32_t pivot_spmm_calls; /* products with H or its leading block the pivot
                           needed, in units of one nvec-wide product */
  int32_t used_fallback; /* learned pivot: 1 if the bootstrap block was returned */
  int32_t basis_blocks;  /* blocks of the basis the returned pairs come from
                            (= iters without restart; see the workspace views) */
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
 * Planned SpMM: the same product for a matrix with the block_rows locality
 * hint, from its prepared form.  bbl_spmm_plan_size returns the device bytes
 * a plan of (H, nvec, vec_dtype) needs, or 0 when no plan can be made
 * (block_rows == 0; nvec not in {1, 2, 4, 8, 10, 16} and not 12 with
 * float32 vectors; or one column block of
 * V -- block_rows * nvec elements; block_rows * 8 floats plus one row for
 * 16 float32 vectors on float32 values -- larger than the 160 KB of LDS).
 * bbl_spmm_plan_build fills `mem` (device, caller-owned, `bytes` >= the size)
 * with two kernels on the stream and the host struct *plan; H must stay
 * unchanged while the plan is used.  bbl_spmm_planned: W = H V for row-major
 * n x plan->nvec blocks of plan->vec_dtype (no overlap); float32 values need
 * float32 vectors, float64 values float64 vectors.
 * Errors: BBL_E_INVALID (no plan possible, NULL pointers, mismatched types),
 * BBL_E_NOMEM (bytes too small), BBL_E_HIP.
 */
size_t bbl_spmm_plan_size(const bbl_csr *H, int32_t nvec, int32_t vec_dtype);
int bbl_spmm_plan_build(const bbl_csr *H, int32_t nvec, int32_t vec_dtype, void *mem,
                        size_t bytes, bbl_spmm_plan *plan, void *stream);
int bbl_spmm_planned(const bbl_spmm_plan *plan, const void *V, void *W, void *stream);

/*
 * Workspace bytes needed by bbl_block_lanczos for dimension n, block size
 * nvec, k_eig wanted pairs, block cap m_max and basis precision basis_dtype,
 * without restart; the _restart form for opts->restart_keep kept Ritz vectors
 * (restart_keep / nvec more basis blocks).  Returns 0 for invalid arguments.
 */
size_t bbl_lanczos_workspace_size(int64_t n, int32_t nvec, int32_t k_eig, int32_t m_max,
                                  int32_t basis_dtype);
size_t bbl_lanczos_workspace_size_restart(int64_t n, int32_t nvec, int32_t k_eig, int32_t m_max,
                                          int32_t basis_dtype, int32_t restart_keep);

/*
 * Lowest k_eig eigenpairs of H by block Lanczos (Methods): the block
 * recurrence H V_j = V_{j-1} B_{j-1}^T + V_j A_j + V_{j+1} B_j with
 * A_j = V_j^T H V_j, full reorthogonalisation of every new block against all
 * stored blocks, a block QR of the residual block giving B_j and V_{j+1}, and
 * the block-tridiagonal band matrix of the A's and B's solved for its lowest
 * Ritz pairs.  Non-restarted by default (the paper's runs); with
 * opts->restart_keep = p > 0, thick restart (the restarted method the paper's
 * introduction and base-Lanczos subsection cite, Wu & Simon): when the basis
 * holds m_max blocks and the pairs have not converged, the p lowest Ritz
 * vectors and the next Lanczos block are kept and the recurrence continues
 * from that block; the projected matrix on the kept vectors is brought back
 * to band form by rotating them (Householder reflectors on the small
 * matrix), so every cycle runs the same kernels as a non-restarted solve.
 * The workspace then comes from bbl_lanczos_workspace_size_restart.
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
 * Returns BBL_OK on convergence, BBL_E_NOT_CONVERGED at the cap (after
 * max_restarts restarts with restart; outputs hold the current Ritz pairs
 * and their true residuals), or an error.
 */
int bbl_block_lanczos(const bbl_csr *H, const double *pivot, int32_t nvec, int32_t k_eig,
                      double tol, void *ws, size_t ws_bytes, const bbl_opts *opts,
                      double *eigvals, double *eigvecs, double *residuals, bbl_stats *stats,
                      void *stream);

/*
 * Diagnostic view of the state a bbl_block_lanczos call left in its workspace
 * (pure pointer arithmetic on ws; nothing is read or launched).  With the same
 * (n, nvec, k_eig, m_max, basis_dtype, restart_keep) as the solve:
 *   basis  receives the device address of the stored Krylov basis: block j
 *          (the paper's V_{j+1}) is a row-major n x nvec array of basis_dtype
 *          at basis + j*n*nvec elements, j = 0..m_max
 *   band   receives the device address of the band matrix of the block
 *          recurrence, (m_max + 1)*nvec rows of nvec + 1 float64:
 *          band[i*(nvec+1) + d] = T[i][i-d] (A blocks on the diagonal, B
 *          blocks below it; the matrix is symmetric)
 * After a solve that reported stats.basis_blocks = m, blocks 0..m-1 and the
 * leading m*nvec rows of the band are V_{1:m} and T_m of the Methods section
 * (after a thick restart: of the final cycle, whose leading restart_keep/nvec
 * blocks hold the kept Ritz vectors in a rotated basis that makes the
 * projected matrix a band matrix again).  Valid until ws is reused.
 */
int bbl_lanczos_workspace_views(const void *ws, int64_t n, int32_t nvec, int32_t k_eig,
                                int32_t m_max, int32_t basis_dtype, int32_t restart_keep,
                                void **basis, double **band);

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
 * Pivot-overlap diagnostic (the Results discussion of why a bootstrapped
 * pivot helps or not: target states missing from the truncated space,
 * "intruders", leave no overlap with the pivot).  For k unit vectors X
 * (e.g. converged eigenvectors) and an n x nvec pivot block P:
 *   cosines   host [k]: cosines of the principal angles between span(X) and
 *             span(P), descending (singular values of X^T Q for an
 *             orthonormal basis Q of span(P); zeros beyond rank)
 *   captured  host [k] or NULL: ||Q^T x_i||^2, the weight of each x_i in span(P)
 * X device n x k float64, P device n x nvec float64 (any full-rank block;
 * directions of P^T P below 1e-12 of its largest eigenvalue are dropped);
 * k, nvec in 1..32; ws device >= bbl_pivot_overlap_workspace_size(n, k, nvec).
 */
size_t bbl_pivot_overlap_workspace_size(int64_t n, int32_t k, int32_t nvec);
int bbl_pivot_overlap(int64_t n, const double *X, int32_t k, const double *P, int32_t nvec,
                      void *ws, size_t ws_bytes, double *cosines, double *captured, void *stream);

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
 * bbl_band_eig without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as bbl_band_eig; the
 * scratch is a 24 MiB array the library holds in device memory on every GPU
 * it runs on until the process ends, so the call allocates nothing (its
 * device address is looked up on the first call on each device).  Sizes
 * whose bbl_band_eig_workspace_size exceeds 24 MiB are rejected with
 * BBL_E_INVALID (N <= 8192 with kd, k <= 16 always fit).  All calls on one
 * GPU share that scratch: calls that overlap in time on one GPU (different
 * streams or threads) race and must be serialised by the caller; nothing
 * needs clearing between calls.
 */
int bbl_band_eig_noalloc(const double *band, int32_t N, int32_t kd, int32_t k, double *theta,
                         double *S, double *top, void *stream);

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

/* ------------------------------------------------------------------------
 * Learned pivot proposer.  The paper's bootstrapped pivot comes from
 * eigenvectors of a truncated leading block, and the Results discussion shows
 * such a pivot can miss target states that live outside the truncation.  The
 * paper does not describe a learned proposer; these entry points implement
 * one (a per-row network fed by truncation-derived features), with the plain
 * bootstrap block as the fallback.  Layouts: features bf16 [rows][28]
 * (bfloat16 bit patterns), network outputs and targets float32 [rows][10],
 * parameters float32 [38026] in the order W1 (128 x 28, row = output unit),
 * b1, W2 (128 x 128), b2, W3 (128 x 128), b3, W4 (10 x 128), b4.  All
 * pointers are device memory unless marked host; the caller owns them.
 * ------------------------------------------------------------------------ */
#define BBL_MLP_IN 28
#define BBL_MLP_OUT 10
#define BBL_MLP_PARAMS 38026

/*
 * Per-row features of H.  The lowest 20 eigenpairs of the leading block
 * H[0:n_trunc, 0:n_trunc] (block Lanczos, block size 10, random pivot of key
 * (opts->seed + 1) ^ 0x9E3779B97F4A7C15, tolerance tol) are extended one hop
 * outside the truncation by first-order perturbation theory,
 * y_ia = (H P)_ia / (theta_a - H_ii) with |denominator| clamped to >= 1; the
 * 10 lowest Rayleigh-Ritz vectors of H on their span form P_D (unit columns,
 * largest-magnitude entry positive).  Row i of the features holds
 *   [0] (H_ii - mean) / std over the diagonal (population std),
 *   [1..16] sin, cos of 2 pi f s / S, f = 1..8, sector s = i / sector_size of
 *       S = ceil(n / sector_size),
 *   [17] nnz of row i / (nnz / n),
 *   [18..27] sqrt(n) P_D[i][0..10).
 *   feats    device n x 28 bfloat16 (round to nearest even)
 *   feats32  optional device n x 28 float32 (the values before rounding)
 *   p_d      optional device n x 10 float64: P_D
 *   p_boot   optional device n x 10 float64: the lowest 10 truncated
 *            eigenvectors, zero padded (the plain bootstrap block)
 *   theta_d  optional host [10]: Ritz values of P_D
 *   stats    optional host: statistics of the truncated solve
 * n_trunc must be in 20..n; BBL_E_BREAKDOWN if the extended block is rank
 * deficient.
 */
size_t bbl_features_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t m_max,
                                   int32_t basis_dtype, void *stream);
int bbl_pivot_features(const bbl_csr *H, int64_t n_trunc, int64_t sector_size, double tol,
                       void *ws, size_t ws_bytes, const bbl_opts *opts, uint16_t *feats,
                       float *feats32, double *p_d, double *p_boot, double *theta_d,
                       bbl_stats *stats, void *stream);

/*
 * Training targets: T = sqrt(n) X Q in float32, Q the orthogonal polar factor
 * of X^T P (the Procrustes rotation taking X closest to P; Schoenemann 1966).
 * X, P device n x m float64 (m <= 32).  BBL_E_BREAKDOWN if X^T P is singular.
 */
size_t bbl_procrustes_workspace_size(int64_t n, int32_t m);
int bbl_procrustes_targets(const double *X, const double *P, int64_t n, int32_t m, void *ws,
                           size_t ws_bytes, float *targets, void *stream);

/*
 * Network 28 -> 128 -> 128 -> 128 -> 10 with ReLU after the first three
 * layers; bfloat16 operands on matrix cores, float32 accumulation, float32
 * parameters (rounded to bfloat16 on load), bfloat16 hidden activations.
 * bbl_mlp_init: He-uniform weights (bound sqrt(6 / fan_in)) from Philox
 *   counter (index, 0, 0, 11) under key `seed`, zero biases.
 * bbl_mlp_forward: out = network(feats) for `rows` rows.
 * bbl_mlp_grad: grad = d loss / d params and *loss (device float, may be
 *   NULL) of loss = mean over rows x 10 outputs of (out - targets)^2;
 *   deterministic (fixed-order partial sums).
 * bbl_adam_step: Adam with bias correction at step >= 1 on `count` values.
 * bbl_mlp_train_step: samples `batch` rows uniformly with replacement
 *   (Philox counter (r, step, 0, 12) under sample_key, modulo dataset_rows),
 *   computes the gradient on them and applies one Adam step (beta1 0.9,
 *   beta2 0.999, eps 1e-8); *loss is the batch loss before the step.
 */
int bbl_mlp_init(float *params, uint64_t seed, void *stream);
int bbl_mlp_forward(const float *params, const uint16_t *feats, int64_t rows, float *out,
                    void *stream);
size_t bbl_mlp_grad_workspace_size(int64_t rows);
int bbl_mlp_grad(const float *params, const uint16_t *feats, const float *targets, int64_t rows,
                 void *ws, size_t ws_bytes, float *grad, float *loss, void *stream);
int bbl_adam_step(float *params, float *m, float *v, const float *grad, int64_t count,
                  int32_t step, float lr, float beta1, float beta2, float eps, void *stream);
size_t bbl_mlp_train_workspace_size(int64_t batch);
int bbl_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                       const uint16_t *feats, const float *targets, int64_t dataset_rows,
                       int64_t batch, uint64_t sample_key, void *ws, size_t ws_bytes,
                       float *loss, void *stream);

/*
 * Learned pivot block: features of H (as bbl_pivot_features), the network's
 * first nvec outputs as the n x nvec block, then the selection: of the
 * learned block, P_D (the network's own input block, the first nvec of its
 * columns) and the plain bootstrap block (lowest nvec truncated
 * eigenvectors, zero padded), the one whose k lowest Rayleigh-Ritz values
 * sum lowest is returned.  The learned block takes part only if its entries
 * are finite and every squared pivot of the Cholesky factor of its Gram
 * matrix is above 1e-8 of the largest diagonal entry; P_D's sum is that of
 * its own Ritz values; ties go to the bootstrap block, then to P_D.
 *   nvec          1..10;  k  number of Ritz values compared (min(k, nvec))
 *   pivot         device n x nvec float64 output (not orthonormalised)
 *   used_fallback host: 0 the learned block, 1 the bootstrap block, 2 P_D
 *   rr_sums       host [3]: the sums (learned, bootstrap, P_D); the learned
 *                 one is NaN when that block failed the finite/Cholesky test
 */
size_t bbl_learned_pivot_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t nvec,
                                        int32_t m_max, int32_t basis_dtype, void *stream);
int bbl_learned_pivot(const bbl_csr *H, const float *params, int64_t n_trunc, int64_t sector_size,
                      int32_t nvec, int32_t k, double tol, void *ws, size_t ws_bytes,
                      const bbl_opts *opts, double *pivot, int32_t *used_fallback,
                      double *rr_sums, bbl_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BBL_H */
