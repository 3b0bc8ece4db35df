"""hloc: hierarchical L2 retrieval and 2-D candidate aggregation for indoor
localization on MI355X (gfx950).

Importing the package loads nothing native; `HlocDB` (in `.hloc`) loads the
HIP library on first use and raises if it has not been built.
"""
__all__ = ["HlocDB", "HlocError"]


def __getattr__(name):
    if name in ("HlocDB", "HlocError"):
        from . import hloc
        return getattr(hloc, name)
    raise AttributeError(name)
