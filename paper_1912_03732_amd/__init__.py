"""MI355X (gfx950) S-box Walsh spectrum and nonlinearity.

The compute path is the HIP library ``libsboxwalsh.so`` built from
``csrc/``; ``binding`` marshals arguments to its C ABI.  Submodules are
imported lazily so that ``inputs`` can be used without loading the library.
"""
import importlib

__all__ = ["binding", "inputs", "autotune", "serving", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
