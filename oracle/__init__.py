"""FP64 CPU oracle -- test infrastructure only (tests, smoke check, CPU baseline).

The product package never imports this; the oracle never imports the product.
"""
from .nnp_oracle import *  # noqa: F401,F403
