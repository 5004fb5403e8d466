"""MI355X (gfx950) implementation of the N log N hierarchical direct solver for
regularized Gaussian-kernel systems (lambda I + K) x = b of Yu, March & Biros,
arXiv:1701.02324: tree, sampled-ID skeletons, recursive Sherman-Morrison-
Woodbury factorization and solves, in hand-written HIP kernels behind a C ABI
(include/askit.h).  This package holds the HIP sources (csrc/), the build
script and the ctypes binding."""
from .askit import (ASKIT_FP64, ASKIT_MIXED, AskitError, Batch, Factor, Tree, askit_batch_check, askit_batch_create,
                    askit_batch_destroy, askit_batch_factor, askit_batch_factorize, askit_batch_solve,
                    askit_skeletonize_batched, askit_build_tree,  # noqa: F401
                    askit_factor_destroy, askit_factor_pivot_ratio, askit_factorize, askit_get_stats,
                    askit_last_solve_info, askit_matvec, askit_profile_enable, askit_profile_report, askit_release_cached_memory,
                    askit_set_refinement, askit_skeletonize,
                    askit_skeletons_export, askit_skeletons_import, askit_solve, askit_solve_transpose,
                    askit_tree_depth, askit_tree_destroy, askit_tree_perm, askit_tree_set_bandwidth, askit_adjoint_scalars,
                    load)
from .autograd import KernelSolve, kernel_solve  # noqa: E402,F401
