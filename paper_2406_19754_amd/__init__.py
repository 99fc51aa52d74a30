"""MI355X-native AMG-preconditioned CG (solve phase of arXiv 2406.19754).

Importing the package loads nothing native. ``paper_2406_19754_amd.psc``
is the thin ctypes binding over the C-ABI library ``libpsc.so`` (HIP for
gfx950); ``paper_2406_19754_amd.problems`` holds the seeded synthetic
inputs.
"""
import importlib

__all__ = ["problems", "psc"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
