// Pivot-block kernels (see pivot.hip).
#pragma once

#include "common.h"

namespace bbl {

// Leading principal block H[0:n_t, 0:n_t] into (rp_t[n_t+1], col_t, val_t).
// The caller sizes col_t/val_t for row_ptr[n_t] entries (an upper bound).
void launch_slice_leading(const bbl_csr &H, int64_t n_t, int64_t *rp_t, int32_t *col_t,
                          void *val_t, hipStream_t s);

// Principal-angle cosines (out[0..k), descending) and per-vector captured
// weights (out[k..2k)) from M = X^T P (k x b) and G = P^T P (b x b).
void launch_overlap(const double *M, const double *G, int k, int b, double *out, hipStream_t s);

}  // namespace bbl
