"""MI355X-native D3Q27 MRT pipe-flow stepper (arXiv:2405.12082 hot path).

The package holds the HIP library (``csrc/``, built into ``liblbm.so``), its
ctypes binding and a thin PyTorch front end.  Importing the package does not
touch the GPU; constructing a :class:`Pipe` needs the built library and a GPU.
"""
from ._lib import LbmConfig, LbmError, LbmLayout, describe, header_functions, lib, make_config

__all__ = ["LbmConfig", "LbmError", "LbmLayout", "describe", "header_functions", "lib", "make_config",
           "Pipe", "radial_profiles"]


def __getattr__(name):
    if name in ("Pipe", "radial_profiles"):
        from . import pipe
        return getattr(pipe, name)
    raise AttributeError(name)
