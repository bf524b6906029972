"""MI355X (gfx950) low-rank splitting solver for differential Lyapunov and
Riccati equations (Mena, Pfurtscheller, Stillfjord 2018).

The compute path is the HIP library ``libdme.so`` (C ABI in include/dme.h);
this package only loads it and marshals arguments.  Importing the package does
not load the library; ``load()`` (or any attribute of ``_binding``) does, and
raises ImportError if it has not been built.
"""

__all__ = ["load", "build"]


def load():
    """Import and return the ctypes binding (raises ImportError if unbuilt)."""
    from . import _binding
    return _binding


def build(verbose: bool = False) -> str:
    from .build import build as _build
    return _build(verbose=verbose)
