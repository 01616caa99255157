"""CPU FP64 oracle for random-features-preconditioned kernel ridge regression.

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it. The product path (the HIP library
and its Python binding) never imports, calls or links anything here, and nothing here
imports the product path.
"""
from .krr_oracle import *  # noqa: F401,F403
from . import sketch_oracle  # noqa: F401
