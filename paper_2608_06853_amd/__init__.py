"""MI355X (gfx950) lens-aware differentiable beamforming.

``_lib``      ctypes binding of libaf.so (the C ABI in include/af.h);
``autofocus`` torch.autograd.Function over the library, the dynamic-grid sweep and
              the plain autofocus loop;
``build``     compiles libaf.so in-tree.

The binding is imported lazily so that ``build`` works before the library exists;
touching any other attribute loads libaf.so and raises if it is missing.
"""
__all__ = ["_lib", "autofocus", "build"]


def __getattr__(name):
    if name in ("_lib", "autofocus", "cnn"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
