"""MI355X (gfx950) neural-constitutive finite-element hot path.

The HIP library (libpa.so, C ABI in include/pa.h) is loaded lazily by the
binding in ``api``; importing this package does not touch the GPU.
"""

__version__ = "0.1.0"


def __getattr__(name):
    if name in ("api",):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
