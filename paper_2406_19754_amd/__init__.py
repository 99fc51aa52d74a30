"""MI355X-native AMG-preconditioned CG (solve phase of arXiv 2406.19754).

Importing the package loads nothing native. ``paper_2406_19754_amd.psc``
is the thin ctypes binding over the C-ABI library ``libpsc.so`` (HIP for
gfx950); ``paper_2406_19754_amd.problems`` holds the seeded synthetic
inputs.
"""
__all__ = ["problems", "psc"]


def __getattr__(name):
    if name == "psc":
        from . import psc
        return psc
    if name == "problems":
        from . import problems
        return problems
    raise AttributeError(name)
