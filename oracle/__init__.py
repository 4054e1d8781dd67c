"""FP64 CPU oracle of the reconstruction hot path -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import this package.  The product library never does, and it
shares no code with the HIP path.
"""
from .utr import *  # noqa: F401,F403
from .fourier import *  # noqa: F401,F403
from . import utr as _utr, fourier as _fourier

__all__ = list(_utr.__all__) + list(_fourier.__all__)
