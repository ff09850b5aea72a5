/* Host-sanitizer driver for the C part of the oracle (test infrastructure).
 * Built with -fsanitize=address,undefined next to oracle/spmm_ref.c and run
 * on the CPU: every oracle product on small CSR matrices with empty rows, a
 * single row, a last row reaching the end of the arrays and block widths 1..32,
 * checked against a dense recomputation.  Exit status 0 = all checks passed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_spmm_f64(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *V, int32_t b, double *W);
void oracle_spmm_f32val(int64_t n, const int64_t *row_ptr, const int32_t *col, const float *val,
                        const double *V, int32_t b, double *W);
void oracle_spmm_abs(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *V, int32_t b, double *W);

static uint64_t lcg = 88172645463325252ull;
static double urand(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) / 9007199254740992.0 - 0.5;
}

/* one case: n rows, each row i has (i * 7 + s) % (m + 1) entries (some empty),
 * columns ascending, exactly allocated arrays (no padding) */
static int run_case(int64_t n, int m, int s, int b) {
  int64_t *rp = malloc((size_t)(n + 1) * sizeof(int64_t));
  rp[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t cnt = (i * 7 + s) % (m + 1);
    if (cnt > n) cnt = n;
    rp[i + 1] = rp[i] + cnt;
  }
  const int64_t nnz = rp[n];
  int32_t *col = malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
  double *val = malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
  float *val32 = malloc((size_t)(nnz ? nnz : 1) * sizeof(float));
  for (int64_t i = 0; i < n; ++i) {
    const int64_t cnt = rp[i + 1] - rp[i];
    for (int64_t t = 0; t < cnt; ++t) {
      col[rp[i] + t] = (int32_t)((t * n) / cnt);  /* ascending, distinct */
      val[rp[i] + t] = urand();
      val32[rp[i] + t] = (float)val[rp[i] + t];
    }
  }
  double *V = malloc((size_t)n * b * sizeof(double));
  for (int64_t k = 0; k < n * b; ++k) V[k] = urand();
  double *W = malloc((size_t)n * b * sizeof(double));
  int bad = 0;
  for (int kind = 0; kind < 3; ++kind) {
    if (kind == 0) oracle_spmm_f64(n, rp, col, val, V, b, W);
    if (kind == 1) oracle_spmm_f32val(n, rp, col, val32, V, b, W);
    if (kind == 2) oracle_spmm_abs(n, rp, col, val, V, b, W);
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < b; ++a) {
        double ref = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
          const double h = kind == 1 ? (double)val32[p] : val[p];
          const double v = V[(int64_t)col[p] * b + a];
          ref += kind == 2 ? fabs(h) * fabs(v) : h * v;
        }
        if (W[i * b + a] != ref) ++bad;  /* same summation order: bit-equal */
      }
  }
  free(rp); free(col); free(val); free(val32); free(V); free(W);
  if (bad) fprintf(stderr, "case n=%lld m=%d s=%d b=%d: %d mismatches\n", (long long)n, m, s, b, bad);
  return bad;
}

int main(void) {
  int bad = 0;
  const int widths[] = {1, 2, 3, 4, 8, 10, 16, 32};
  for (int w = 0; w < 8; ++w) {
    bad += run_case(1, 1, 0, widths[w]);     /* one row, possibly empty */
    bad += run_case(1, 1, 1, widths[w]);
    bad += run_case(37, 5, 3, widths[w]);    /* ragged, some empty rows */
    bad += run_case(1000, 40, 11, widths[w]);
  }
  bad += run_case(5, 0, 0, 4);               /* no entries at all */
  printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
