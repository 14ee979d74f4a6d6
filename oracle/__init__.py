"""FP64 CPU oracle (test infrastructure; never imported by the library)."""
from .powerflow import Oracle, Solved, solve  # noqa: F401
