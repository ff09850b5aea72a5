/* Host-sanitizer driver for the C ABI (include/bbl.h), linked against a build
 * of the library whose host code carries -fsanitize=address,undefined.  No
 * GPU is needed: it calls only what returns before any device work -- the
 * argument validation of every kind of entry point (NULL and out-of-range
 * arguments, inconsistent types, a workspace smaller than its query), the
 * size queries, and the workspace views (pointer arithmetic).  Exit status
 * 0 = every call returned what the header promises. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "bbl.h"

static int fails = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      fprintf(stderr, "line %d: %s (last error: %s)\n", __LINE__, #cond, \
              bbl_last_error());                                          \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

int main(void) {
  /* fake device addresses: never dereferenced by the calls below */
  const int64_t *rp = (const int64_t *)(uintptr_t)0x1000;
  const int32_t *col = (const int32_t *)(uintptr_t)0x2000;
  const void *val = (const void *)(uintptr_t)0x3000;
  void *V = (void *)(uintptr_t)0x4000, *W = (void *)(uintptr_t)0x5000;
  double ev[8];
  bbl_opts o;
  bbl_csr H;

  EXPECT(bbl_version() != NULL && strlen(bbl_version()) > 0);
  /* workspace queries */
  EXPECT(bbl_lanczos_workspace_size(0, 4, 4, 10, BBL_F64) == 0);
  EXPECT(bbl_lanczos_workspace_size(100, 0, 4, 10, BBL_F64) == 0);
  EXPECT(bbl_lanczos_workspace_size(100, 33, 4, 10, BBL_F64) == 0);
  EXPECT(bbl_lanczos_workspace_size(100, 4, 4, 10, 7) == 0);
  EXPECT(bbl_lanczos_workspace_size(20000, 4, 4, 200, BBL_F64) >
         bbl_lanczos_workspace_size(20000, 4, 4, 200, BBL_F32));
  EXPECT(bbl_lanczos_workspace_size_restart(1000, 4, 4, 20, BBL_F64, 6) == 0);
  EXPECT(bbl_band_eig_workspace_size(100, 4, 200) == 0);
  EXPECT(bbl_gram_workspace_size(100, 8, 2, 33) == 0);
  EXPECT(bbl_gram_workspace_size(100, 16, 3, 16) > 0);

  /* SpMM */
  EXPECT(bbl_spmm(NULL, NULL, NULL, 4, BBL_F64, NULL) == BBL_E_INVALID);
  memset(&H, 0, sizeof H);
  EXPECT(bbl_spmm(&H, V, W, 4, BBL_F64, NULL) == BBL_E_INVALID);       /* n = 0 */
  H.n = 10; H.nnz = 5; H.row_ptr = rp; H.col = col; H.val = val; H.val_dtype = 9;
  EXPECT(bbl_spmm(&H, V, W, 4, BBL_F64, NULL) == BBL_E_INVALID);       /* bad dtype */
  H.val_dtype = BBL_F64;
  EXPECT(bbl_spmm(&H, V, W, 4, BBL_F32, NULL) == BBL_E_INVALID);       /* f32 vectors, f64 H */
  EXPECT(bbl_spmm(&H, V, W, 40, BBL_F64, NULL) == BBL_E_INVALID);      /* nvec > 32 */
  EXPECT(bbl_spmm(&H, NULL, W, 4, BBL_F64, NULL) == BBL_E_INVALID);    /* NULL V */

  /* plan sizes (host-only arithmetic) */
  H.n = 20000; H.nnz = 2000000; H.val_dtype = BBL_F32; H.block_rows = 0;
  EXPECT(bbl_spmm_plan_size(&H, 8, BBL_F32) == 0);                     /* no hint */
  H.block_rows = 1000;
  EXPECT(bbl_spmm_plan_size(&H, 3, BBL_F32) == 0);                     /* width 3 */
  EXPECT(bbl_spmm_plan_size(&H, 8, BBL_F32) > 0);
  EXPECT(bbl_spmm_plan_size(&H, 12, BBL_F32) > 0);
  EXPECT(bbl_spmm_plan_size(&H, 32, BBL_F32) == 0);
  H.val_dtype = BBL_F64;
  EXPECT(bbl_spmm_plan_size(&H, 8, BBL_F64) > 0);
  EXPECT(bbl_spmm_plan_size(&H, 12, BBL_F64) == 0);

  /* block Lanczos: validation before any launch */
  H.n = 10; H.nnz = 5; H.val_dtype = BBL_F64; H.block_rows = 0;
  memset(&o, 0, sizeof o);
  o.m_max = 1; o.basis_dtype = BBL_F64; o.defl_tau = 1e-12;
  EXPECT(bbl_block_lanczos(&H, (const double *)V, 2, 4, 1e-8, W, (size_t)1 << 30, &o, ev, NULL,
                           NULL, NULL, NULL) == BBL_E_INVALID);        /* k > nvec * m_max */
  o.m_max = 10; o.basis_dtype = BBL_F32;
  EXPECT(bbl_block_lanczos(&H, (const double *)V, 2, 2, 1e-8, W, (size_t)1 << 30, &o, ev, NULL,
                           NULL, NULL, NULL) == BBL_E_INVALID);        /* f32 basis, f64 H */
  o.basis_dtype = BBL_F64;
  EXPECT(bbl_block_lanczos(&H, (const double *)V, 2, 2, 1e-8, W, 16, &o, ev, NULL, NULL, NULL,
                           NULL) == BBL_E_NOMEM);                      /* workspace too small */
  EXPECT(bbl_block_lanczos(NULL, (const double *)V, 2, 2, 1e-8, W, (size_t)1 << 30, &o, ev, NULL,
                           NULL, NULL, NULL) == BBL_E_INVALID);
  {
    const int keeps[5] = {0, -2, 3, 2, 18}, faults[5] = {-1, 0, 0, 0, 0};
    for (int t = 0; t < 5; ++t) {
      o.restart_keep = keeps[t]; o.fault_block = faults[t];
      EXPECT(bbl_block_lanczos(&H, (const double *)V, 2, 4, 1e-8, W, (size_t)1 << 30, &o, ev,
                               NULL, NULL, NULL, NULL) == BBL_E_INVALID);
    }
    o.restart_keep = 0; o.fault_block = 0;
  }

  /* pivots, products, band eigensolve, no-allocation entry point */
  EXPECT(bbl_random_pivot(0, 4, 1, (double *)V, NULL) == BBL_E_INVALID);
  EXPECT(bbl_block_update(10, NULL, 2, 4, 1, NULL, 4, 1.0, NULL, 2, 0.0, NULL, 2, NULL) ==
         BBL_E_INVALID);
  EXPECT(bbl_gram(10, NULL, 2, 4, 1, NULL, 2, 4, NULL, NULL, 0, NULL) == BBL_E_INVALID);
  EXPECT(bbl_band_eig_noalloc(NULL, 100, 4, 4, ev, NULL, NULL, NULL) == BBL_E_INVALID);
  EXPECT(bbl_band_eig_noalloc((const double *)V, 8192, 32, 32, ev, NULL, NULL, NULL) ==
         BBL_E_INVALID);
  EXPECT(bbl_bootstrap_pivot(NULL, 10, 4, 1e-8, W, 0, NULL, NULL, NULL, NULL) == BBL_E_INVALID);

  /* workspace views: pointer arithmetic only */
  {
    void *basis = NULL;
    double *band = NULL;
    const uintptr_t base = 0x10000000u;
    EXPECT(bbl_lanczos_workspace_views((const void *)(base + 8), 1000, 4, 4, 20, BBL_F64, 0,
                                       &basis, &band) == BBL_OK);
    EXPECT((uintptr_t)basis == base + 256);
    EXPECT((uintptr_t)band % 256 == 0 && (uintptr_t)band >= (uintptr_t)basis + 21u * 1000 * 4 * 8);
    EXPECT(bbl_lanczos_workspace_views((const void *)base, 0, 4, 4, 20, BBL_F64, 0, &basis,
                                       &band) == BBL_E_INVALID);
  }
  printf("abi driver: %s\n", fails ? "FAILED" : "ok");
  return fails ? 1 : 0;
}
