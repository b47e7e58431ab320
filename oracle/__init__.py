"""FP64 CPU oracle (test infrastructure only; see lt_oracle's header)."""
from .lt_oracle import *  # noqa: F401,F403
