"""CPU complex128 oracle for the state-vector hot path.

TEST INFRASTRUCTURE ONLY: imported solely by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path (``paper_2406_17248_amd``)
never imports it, and it never imports the product path.
"""

from .statevector import *  # noqa: F401,F403
from . import statevector  # noqa: F401
