"""MI355X (gfx950) energy + force evaluation of a descriptor-based neural network
potential for the ML atoms of an MD system.

The computation lives in the HIP library ``libnnp.so`` (C ABI in include/nnp.h);
this package is its thin Python binding.
"""
from .nnp import *  # noqa: F401,F403  (the C ABI's calls under their own names, NNPModel, NNPEnergy)
from .nnp import __all__  # noqa: F401
from . import _lib  # noqa: F401

__version__ = "0.1.0"
