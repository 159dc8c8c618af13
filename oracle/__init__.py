"""FP64 CPU oracle (test infrastructure only; see claire_oracle.py)."""
from .claire_oracle import *  # noqa: F401,F403
from .claire_oracle import Grid, build_c  # noqa: F401
