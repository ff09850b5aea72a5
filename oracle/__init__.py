"""CPU FP64 oracle for bootstrapped block Lanczos -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of what the HIP path computes,
written from Zbikowski & Johnson, "Bootstrapped Block Lanczos for
large-dimension eigenvalue problems" (arXiv 2210.15763):

* ``spmm``            -- the block product w_{a,i} = sum_j H_ij v_{a,j}
                         (Methods, "Block Lanczos algorithm"), a C loop.
* ``block_lanczos``   -- the block three-term recurrence with the diagonal
                         block A_n, the residual block W', the overlap O and
                         its spectral factorisation B_n, V_{n+1}, full
                         reorthogonalisation, and the band matrix solved by a
                         dense symmetric eigensolver (Methods).
* ``block_lanczos_restarted`` -- the same recurrence with thick restart: at
                         the block cap the lowest Ritz vectors and the
                         residual block are kept and the recurrence
                         continues on the arrowhead-bordered band matrix
                         (the restarted method the paper cites, Wu & Simon).
* ``scalar_lanczos``  -- the single-vector method (Algorithm "Lanczos method").
* ``bootstrap_pivot`` -- the pivot block built from eigenvectors of a
                         truncated leading block (Methods, last paragraphs).
* ``pivot``           -- a float64 reference of the learned pivot proposer:
                         its per-row features (one-hop extension of truncated
                         eigenvectors plus Rayleigh-Ritz), the network's
                         forward/backward pass, Adam, Procrustes targets and
                         the fallback rule (not in the paper; see that module).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the HIP path; the only
common dependency is the seeded input generator ``synthgen``.
"""
from .spmm import spmm, spmm_abs, build_native  # noqa: F401
from .lanczos import (block_lanczos, scalar_lanczos, bootstrap_pivot, svqb,  # noqa: F401
                      ritz_residuals, LanczosResult, block_lanczos_restarted)
