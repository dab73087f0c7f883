"""CPU oracle (test infrastructure only; see prony_oracle)."""
from . import prony_oracle  # noqa: F401
