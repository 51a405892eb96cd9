"""MI355X (gfx950) energy + force evaluation of a descriptor-based neural network
potential for the ML atoms of an MD system.

The computation lives in the HIP library ``libnnp.so`` (C ABI in include/nnp.h);
this package is its thin Python binding.
"""
from .nnp import (NNPEnergy, NNPError, NNPModel, make_config, nnp_compute, nnp_compute_pairs, nnp_compute_batch,  # noqa: F401
                  nnp_create, nnp_destroy, nnp_get_status, nnp_autotune, nnp_set_variant, nnp_get_variants, nnp_me_coupling, nnp_set_links, nnp_profile_enable, nnp_profile_read, nnp_set_graph, nnp_last_error, nnp_read_buffer, nnp_reserve,
                  nnp_status_string, nnp_version)
from . import _lib  # noqa: F401

__version__ = "0.1.0"
