"""FP64 CPU oracle for coherent dedispersion (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never does.
"""
from .cdd_oracle import *  # noqa: F401,F403
from .cdd_oracle import D_PAPER  # noqa: F401
