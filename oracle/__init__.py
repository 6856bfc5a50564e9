"""FP64 CPU oracle of WB-arSVD RZF precoding.

TEST INFRASTRUCTURE, not product code.  Only `tests/`, the smoke check in
`__graft_entry__.py` and the CPU-baseline leg of `bench.py` may import, call or
execute anything in this package.  The GPU library never routes through it.

Pinned functions and their pins are listed in `tests/test_oracle_*.py`; a
function without an independent pin says "parity unpinned" in its docstring.
"""
from .rzf import *  # noqa: F401,F403
from .rzf import (PATH_NOOP, PATH_WB, PATH_FULL_RANK, PATH_FULL_SINGULAR,  # noqa: F401
                  PATH_RESET, PATH_NAMES, OracleTrack, TrackParams, UpdateInfo)
from . import philox  # noqa: F401
