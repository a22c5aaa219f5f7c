"""Serial CPU oracle of pdGRASS off-tree edge recovery (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library never uses it.
"""
from .oracle import (OracleResult, build, load, recover, MODE_INDEXED, MODE_BRUTE,  # noqa: F401
                     MODE_SUBTASK, STATUS, spanning_tree)
