"""FP64 CPU oracle of the reconstruction hot path -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import this package.  The product library never does, and it
shares no code with the HIP path.
"""
from .utr import *  # noqa: F401,F403
from .utr import __all__  # noqa: F401
