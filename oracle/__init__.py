"""FP64 CPU oracle (test infrastructure only; see wc4d_oracle's header)."""
from . import wc4d_oracle  # noqa: F401
