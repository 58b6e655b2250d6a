"""MI355X-native hot path of the adjoint-based variational method for periodic orbits of the
Kuramoto-Sivashinsky equation (Azimi, Ashtari & Schneider, arXiv:2007.06427).

The kernels live in liblooporbit.so (HIP, gfx950) behind the C ABI of include/looporbit.h.
This package binds that ABI and adds a torch.autograd.Function whose backward is the adjoint
kernel. There is no CPU fallback: the functions raise if the library is missing.
"""
from ._lib import EXPLICIT, IMEX, LoopOrbitError, status_string  # noqa: F401

__all__ = ["EXPLICIT", "IMEX", "LoopOrbitError", "status_string"]


def __getattr__(name):
    # the tensor-level API needs torch; import it lazily so that the ctypes layer loads without it
    if name in ("api", "autograd", "initial_loops"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
