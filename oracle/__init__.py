"""FP64 CPU oracle for fast count sketch.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  Nothing in the product package imports
it, and it imports nothing from the product package.
"""
from .fcs_oracle import *  # noqa: F401,F403
from .fcs_oracle import hash_tables, sketch_length  # noqa: F401
from .native import dense_rows, coo, build_native, tables_flat  # noqa: F401
