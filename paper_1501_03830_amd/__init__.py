"""gfx950 (MI355X) structure-preserving eigensolver for Bethe-Salpeter
Hamiltonians (arXiv:1501.03830, Algorithms 1 and 3).

The solver lives in libbse.so (HIP kernels behind the C ABI of
include/bse.h); this package only loads it and marshals torch tensors.
Importing the package does not load the library; `Context` does, and fails
loudly when the library has not been built.
"""

from ._lib import (BSE_OK, BSE_ENOMEM, BSE_EDEVICE, BSE_PREC_FP64, BSE_WANT_VECTORS,  # noqa: F401
                   BSE_WANT_WEIGHTS, BseError, load, LIB_PATH, STAGE_NAMES)


def Context(*args, **kwargs):
    from .api import Context as _Ctx
    return _Ctx(*args, **kwargs)


def footprint_bytes(n: int, prec: int = BSE_PREC_FP64, flags: int = 0) -> int:
    from .api import footprint_bytes as _fb
    return _fb(n, prec, flags)
