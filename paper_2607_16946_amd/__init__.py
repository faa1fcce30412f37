"""MI355X-native pointwise signed distance to point clouds ("Points as Tori").

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``, declared in ``include/pts.h``).  ``binding`` marshals
arguments to it through ctypes; PyTorch supplies device memory and streams.
Submodules load lazily so that the workload generators (``synth``) can be
imported without a GPU or a built library.
"""

import importlib

_LAZY = {"binding", "synth", "autograd", "server", "build"}


def __getattr__(name):
    if name in _LAZY:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
