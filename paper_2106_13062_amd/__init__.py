"""MI355X-native fast count sketch (arXiv 2106.13062): dense, COO and CP
sketches and sketched contractions behind the C ABI of include/fcs.h."""
from ._lib import FcsError, load  # noqa: F401
from .fcs import Batch, Plan, inner_median  # noqa: F401

__all__ = ["Plan", "Batch", "FcsError", "load", "inner_median"]
