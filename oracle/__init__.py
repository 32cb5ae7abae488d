"""Plain FP64 CPU oracle of the grim method (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library and its Python binding never do.
"""
from .oracle import Oracle, OCfg, OStats, build, FLAGS  # noqa: F401
