"""CPU oracle — test infrastructure only (see ``psi_oracle``).

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library.
"""
from .psi_oracle import *  # noqa: F401,F403
