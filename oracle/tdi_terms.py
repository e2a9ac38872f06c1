"""Term lists of the Michelson TDI combinations (test infrastructure only).

X1 and X2 are written out from Sec. IV.C, eqs. (tdi1) and (tdi2); Y and Z
follow by the cyclic relabelling 1 -> 2 -> 3 -> 1 applied once and twice
(same section).  A term is sign * D_{path} y_{link}; a path of one spacecraft
is the undelayed sample; the delay of a path i1 i2 ... in is the sum of
L_{ik ik+1} taken at the output time.
"""
from __future__ import annotations

import dataclasses

# link l -> (receiver, emitter)
LINKS = ((1, 2), (2, 3), (3, 1), (1, 3), (3, 2), (2, 1))


@dataclasses.dataclass(frozen=True)
class Term:
    channel: int          # 0 = X, 1 = Y, 2 = Z
    sign: int
    link: int             # index into LINKS of the measured series
    path: tuple           # spacecraft of the delay chain, length >= 1


def _link(s):
    return LINKS.index((int(s[0]), int(s[1])))


# (sign, delay path, measured link) for X1, eq. (tdi1):
#   y13 + D13 y31 + D131 y12 + D1312 y21 - [y12 + D12 y21 + D121 y13 + D1213 y31]
_X1 = [
    (+1, "1", "13"), (+1, "13", "31"), (+1, "131", "12"), (+1, "1312", "21"),
    (-1, "1", "12"), (-1, "12", "21"), (-1, "121", "13"), (-1, "1213", "31"),
]
# additional terms of X2, eq. (tdi2):
#   + D13121 y12 + D131212 y21 + D1312121 y13 + D13121213 y31
#   - [D12131 y13 + D121313 y31 + D1213131 y12 + D12131312 y21]
_X2_EXTRA = [
    (+1, "13121", "12"), (+1, "131212", "21"), (+1, "1312121", "13"), (+1, "13121213", "31"),
    (-1, "12131", "13"), (-1, "121313", "31"), (-1, "1213131", "12"), (-1, "12131312", "21"),
]


def _rotate(s, times):
    out = s
    for _ in range(times):
        out = "".join(str(int(ch) % 3 + 1) for ch in out)
    return out


def michelson_terms(generation):
    if generation not in (1, 2):
        raise ValueError("generation must be 1 or 2")
    base = _X1 + (_X2_EXTRA if generation == 2 else [])
    terms = []
    for ch in range(3):
        for sign, path, link in base:
            p = _rotate(path, ch)
            terms.append(Term(ch, sign, _link(_rotate(link, ch)), tuple(int(c) for c in p)))
    return terms
