"""FP64 CPU oracle for pitch-by-pitch Katsevich helical FBP.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never calls it and shares no code with it.
"""
from .katsevich_oracle import *  # noqa: F401,F403
from . import data_oracle  # noqa: F401,E402
