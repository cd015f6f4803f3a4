"""Float64 CPU oracle of the NU-FDS reconstruction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The GPU
library never uses it, and it shares no code with the GPU library.
"""
from .nufds_oracle import *  # noqa: F401,F403
from .nufds_oracle import __all__  # noqa: F401
