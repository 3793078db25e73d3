"""FP64 CPU oracle (test infrastructure only; see fe_oracle.py)."""
from .fe_oracle import *  # noqa: F401,F403
