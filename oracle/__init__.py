"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from . import ptycho  # noqa: F401
