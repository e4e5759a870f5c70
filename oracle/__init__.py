"""FP64 CPU oracle (test infrastructure only; see sb2_oracle's header)."""
from .sb2_oracle import *  # noqa: F401,F403
