"""Plain FP64 CPU oracle (test infrastructure only).

Nothing in the product path may import this package: only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code with the HIP library.
"""
from .solver import *  # noqa: F401,F403
from .solver import __all__  # noqa: F401
