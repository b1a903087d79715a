"""MI355X-native assembly of the explicit LES momentum residual.

The compute path lives in a C-ABI shared library (``csrc/``, HIP for gfx950);
``lesasm`` is its thin ctypes binding.  ``meshgen`` builds seeded synthetic
inputs.  Submodules are imported lazily so that input generation never loads
the GPU library.
"""
import importlib

__all__ = ["meshgen", "lesasm"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
