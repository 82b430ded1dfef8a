"""FP64 CPU oracle for APPGA on the SHOITV Poisson PET model (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package.  It is independent of the GPU library:
it shares no source, header or helper with it and never imports it.
"""
from .oracle import *  # noqa: F401,F403
