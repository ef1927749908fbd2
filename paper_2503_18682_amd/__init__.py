"""MI355X (gfx950) ray-based Gaussian splatting: HIP kernels behind a C ABI
(include/raygs.h, libraygs.so) with a thin torch/ctypes binding.

The package import is light; the HIP library is loaded on first use and the
import of `Renderer` fails loudly if it has not been built.
"""
__all__ = ["Renderer", "BatchRenderer", "RenderFunction", "render", "load_library"]


def load_library():
    from . import _lib

    return _lib.load()


def __getattr__(name):
    if name in ("Renderer", "BatchRenderer", "RenderFunction", "render", "make_options", "DEFAULT_OPTIONS"):
        from . import renderer

        return getattr(renderer, name)
    raise AttributeError(name)
