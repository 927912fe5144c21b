"""FP64 CPU oracle (test infrastructure only; see vit64.py).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product package never does.
"""
from . import vit64  # noqa: F401
