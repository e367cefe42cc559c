"""Reference parser for text edge lists (TEST INFRASTRUCTURE ONLY).

The paper streams graphs that it reads as text edge lists (Sec. 5, Table 2
reports the reading time separately).  This is the plain definition of the
format the device parser accepts, written out line by line: a line whose
first byte is '#' or '%' is a comment; on every other line each maximal run
of decimal digits is one vertex id; ids 2k and 2k+1 (in file order) form
edge k.  Any other bytes (spaces, tabs, commas, '\\r') separate ids.  Used only
by the tests; it shares no code with the device parser.
"""
from __future__ import annotations

import numpy as np


class ParseError(ValueError):
    """An odd number of ids, or an id above 2^32 - 1."""


def parse_edge_list(text: bytes) -> np.ndarray:
    """The edges of `text` in file order, as a (m, 2) uint64 array."""
    ids = []
    for line in text.split(b"\n"):
        if line[:1] in (b"#", b"%"):
            continue
        cur = None
        for ch in line + b" ":
            if 48 <= ch <= 57:
                cur = (cur or 0) * 10 + ch - 48
            elif cur is not None:
                if cur > 0xFFFFFFFF:
                    raise ParseError("an id above 2^32 - 1")
                ids.append(cur)
                cur = None
    if len(ids) % 2:
        raise ParseError("an odd number of ids")
    return np.array(ids, dtype=np.uint64).reshape(-1, 2)
