"""MI355X-native path-compression Morse-Smale segmentation and connected
components (arXiv 2409.03771), behind the C-ABI library ``libmsc.so``.

The binding lives in ``paper_2409_03771_amd.msc``; it is loaded on first
attribute access so that ``paper_2409_03771_amd.synth`` can be used on
machines without the built library.
"""
import importlib

__all__ = ["msc", "synth"]


_SUBMODULES = ("msc", "synth", "build", "profsum")


def __getattr__(name):
    # Submodules import on their own: `build` in particular must not load
    # the library it is about to replace (a process keeps the first copy of
    # a shared object it opened under a given path).
    if name in _SUBMODULES:
        return importlib.import_module(f"{__name__}.{name}")
    mod = importlib.import_module(f"{__name__}.msc")
    return getattr(mod, name)
