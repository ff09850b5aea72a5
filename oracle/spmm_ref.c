/* CPU FP64 oracle -- test infrastructure only (see oracle/__init__.py).
 *
 * Block sparse-matrix product of the paper's block Lanczos section:
 *     w_{a,i} = sum_j H_ij v_{a,j}
 * written as the plain loop over matrix elements with the loop over the block
 * index a innermost.  H is CSR (int64 row pointers, int32 columns, float64 or
 * float32 values, the latter promoted exactly to float64); V and W are
 * row-major n x b float64 blocks.  Each w_{a,i} is accumulated serially in
 * ascending element order.  Rows are independent, so OpenMP splits them.
 */
#include <stdint.h>

void oracle_spmm_f64(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *V, int32_t b, double *W) {
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < n; ++i) {
    double *w = W + i * b;
    for (int32_t a = 0; a < b; ++a) w[a] = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const double h = val[p];
      const double *v = V + (int64_t)col[p] * b;
      for (int32_t a = 0; a < b; ++a) w[a] += h * v[a];
    }
  }
}

void oracle_spmm_f32val(int64_t n, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *V, int32_t b, double *W) {
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < n; ++i) {
    double *w = W + i * b;
    for (int32_t a = 0; a < b; ++a) w[a] = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const double h = (double)val[p];
      const double *v = V + (int64_t)col[p] * b;
      for (int32_t a = 0; a < b; ++a) w[a] += h * v[a];
    }
  }
}

/* Absolute-value companion: sum_j |H_ij| |v_{a,j}|, the scale in the standard
 * forward-error bound of a floating-point dot product. */
void oracle_spmm_abs(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *V, int32_t b, double *W) {
#pragma omp parallel for schedule(dynamic, 512)
  for (int64_t i = 0; i < n; ++i) {
    double *w = W + i * b;
    for (int32_t a = 0; a < b; ++a) w[a] = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      const double h = val[p] < 0 ? -val[p] : val[p];
      const double *v = V + (int64_t)col[p] * b;
      for (int32_t a = 0; a < b; ++a) w[a] += h * (v[a] < 0 ? -v[a] : v[a]);
    }
  }
}
