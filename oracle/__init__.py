"""FP64 CPU oracle for the KS loop-space adjoint step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. It shares no code with the HIP path.
"""
from . import ks_loop, brute  # noqa: F401
from .ks_loop import (EXPLICIT, IMEX, adjoint_grad, autograd_grad, canonical, cost, dJdT,  # noqa: F401
                      residual, step)
