"""FP64 CPU oracle (test infrastructure only; see ``oracle.kmeans``).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It imports nothing from the HIP
library package and the library imports nothing from it.
"""
from . import kmeans  # noqa: F401
