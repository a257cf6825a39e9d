"""MI355X-native recursive Green's function (RGF) library for NEGF device
simulation: HIP kernels for gfx950 behind a C ABI (include/negf.h), a ctypes
binding (``negf``) and a thin host driver (``runtime``)."""

__all__ = ["negf", "runtime", "build"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
