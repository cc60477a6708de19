"""FP64 CPU oracle (test infrastructure only; see mdp_oracle.py)."""
from .mdp_oracle import *  # noqa: F401,F403
