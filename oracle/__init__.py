"""CPU FP64 oracle (test infrastructure only; see ipi_oracle.py)."""
from .ipi_oracle import *  # noqa: F401,F403
