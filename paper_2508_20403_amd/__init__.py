"""pdGRASS off-tree edge recovery on MI355X (gfx950): C-ABI library + thin binding."""
from . import synth  # noqa: F401  (seeded input generators, no method arithmetic)

__all__ = ["synth"]
