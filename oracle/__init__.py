"""FP64 CPU oracle for the SHARP RAAR hot path (test infrastructure only:
imported by the tests, the smoke check and the benchmark's CPU-baseline leg,
never by the library)."""
from .sharp_oracle import *  # noqa: F401,F403
from . import sharp_oracle  # noqa: F401
