"""FP64 CPU oracle for the k-means Lloyd iteration and the applications that
reuse its building blocks (``oracle.ml``) -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library and imports nothing from it.
"""
from .oracle import (  # noqa: F401
    build, assign, update, lloyd, objective, near_tie_margin, num_threads, LIB_PATH,
)
from . import ml  # noqa: F401,E402


def build_all():
    """Compile every C oracle (gcc)."""
    build()
    ml.build()
