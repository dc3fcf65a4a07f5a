"""FFT-based block-Toeplitz parameter-to-observable operator for MI355X (gfx950).

Applies the p2o map F of a linear time-invariant system, its adjoint F^*,
the data-space products F F^* and the data-misfit gradient, and on top of
them the data-space matrix K, its Cholesky factor, the real-time MAP point
and posterior-covariance actions, with hand-written HIP kernels behind a C
ABI (include/p2o.h, libp2o.so).  Importing the
package loads the library and fails if it has not been built.
"""
from ._lib import P2OError, LIB_PATH, PRECISIONS, lib, status_name, last_error
from .ops import (P2OOperator, P2O, P2OT, misfit, SCALE_BLOCK, bandwidth_probe, gemm_tiles, cholesky,
                  cholesky_solve, d2q_apply, assemble_K_from_blocks)

__all__ = ["bandwidth_probe", "gemm_tiles", "P2OOperator", "P2O", "P2OT", "misfit", "cholesky", "cholesky_solve", "d2q_apply",
           "assemble_K_from_blocks", "P2OError", "PRECISIONS", "SCALE_BLOCK", "lib", "LIB_PATH", "status_name", "last_error"]
