"""MI355X-native RD step of SpeedyGS's structural-formation stage.

The computation lives in ``libspeedygs.so`` (hand-written HIP for gfx950,
C ABI in ``include/speedygs.h``); this package is its Python binding.
Importing it does not load the library; ``Context`` does, and fails loudly
when the library has not been built.
"""
from ._lib import EXPORTS, NCH, RATE_GRAD_FLOATS, STATS_WORDS, Context, SgsError, lib  # noqa: F401

__all__ = ["Context", "SgsError", "lib", "EXPORTS", "NCH", "STATS_WORDS", "RATE_GRAD_FLOATS"]
