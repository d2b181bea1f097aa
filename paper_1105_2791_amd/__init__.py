"""MI355X-native modal bispectrum estimator hot path (Fergusson & Shellard,
"Optimal Polyspectra Estimation").

The computation lives in libmodal.so (hand-written HIP for gfx950) behind the C
ABI in include/modal.h; this package is its Python binding.  Importing
``ModalContext`` loads the library and fails if it has not been built.
"""
from __future__ import annotations

__all__ = ["ModalContext", "ModalError", "ModalBeta"]


def __getattr__(name):
    if name in ("ModalContext",):
        from .api import ModalContext
        return ModalContext
    if name == "ModalError":
        from ._lib import ModalError
        return ModalError
    if name == "ModalBeta":
        from .autograd import ModalBeta
        return ModalBeta
    raise AttributeError(name)
