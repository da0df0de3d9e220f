"""MI355X-native feature-field Gaussian rasterizer (GSFF-SLAM hot path).

The computation lives in ``libgsff.so`` (HIP, gfx950) behind the C ABI of
``include/gsff.h``; this package only marshals arguments.  Submodules are
imported lazily so ``scenegen`` can be used without touching the GPU library.
"""
import importlib

__all__ = ["rasterizer", "scenegen", "decoder", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
