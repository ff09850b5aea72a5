// Host-side pieces of the solver shared by the C ABI entry points: options,
// argument checks, the block-Lanczos driver and the truncated-block solve
// used by the bootstrapped and learned pivots.
#pragma once

#include <cstdint>

#include "common.h"

namespace bbl {

struct Opts {
  int m_max = 200;
  int basis_dtype = 0;  // 0: from H
  int check_every = 0;
  int flags = 0;
  double tau = 1e-12;
  uint64_t seed = 0;
  const bbl_spmm_plan *plan = nullptr;
  int restart_keep = 0;  // thick restart: Ritz vectors kept (0 = off)
  int max_restarts = 100;
  int fault_block = 0;   // testing: host-forced breakdown + redo (0 = off)
  int feature_vectors = 0;  // learned pivot: truncated eigenvectors of P_D (0 = 20)
};

Opts read_opts(const bbl_opts *o, int val_dtype);
void validate_csr(const bbl_csr *H);
// row_ptr[i] read back to the host (synchronises the stream)
int64_t read_row_ptr(const bbl_csr &H, int64_t i, hipStream_t s);

// Lowest k eigenpairs of H from the n x nvec pivot (see bbl_block_lanczos).
int solve_impl(const bbl_csr *H, const double *pivot, int32_t nvec, int32_t k, double tol,
               void *ws, size_t ws_bytes, const Opts &o, double *eigvals, double *eigvecs,
               double *residuals, bbl_stats *stats, hipStream_t s);

// Lowest k eigenpairs of the leading block H[0:n_t, 0:n_t]: the block is
// sliced out of H into the workspace, then solved by block Lanczos with block
// size b from the Gaussian pivot of key (seed + 1) ^ 0x9E3779B97F4A7C15 and
// deflation seed seed + 1.  eigvecs_t: device [n_t][k]; theta: host [k].
size_t truncated_ws_bytes(const bbl_csr &H, int64_t n_t, int b, int k, const Opts &o,
                          hipStream_t s);
int truncated_solve(const bbl_csr &H, int64_t n_t, int b, int k, double tol, const Opts &o,
                    void *ws, size_t ws_bytes, double *eigvecs_t, double *theta,
                    bbl_stats *stats, hipStream_t s);

// Runs f, turning exceptions into a status code and the thread's last error.
template <typename F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception &e) {
    set_error(e.what());
    return BBL_E_INVALID;
  } catch (...) {
    set_error("unknown error");
    return BBL_E_INVALID;
  }
}

}  // namespace bbl
