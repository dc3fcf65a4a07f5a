"""FP64 CPU oracle (test infrastructure only; never on the product path).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.
"""
from .toeplitz import (apply_F, apply_Ft, misfit_and_grad, data_space_hessian,
                       spectrum, rel_l2)

__all__ = ["apply_F", "apply_Ft", "misfit_and_grad", "data_space_hessian",
           "spectrum", "rel_l2"]
