"""FP64 CPU oracle (test infrastructure only; see oracle/hubbard.py)."""
from .hubbard import *  # noqa: F401,F403
from .hubbard import __all__  # noqa: F401
from . import hmc  # noqa: F401
