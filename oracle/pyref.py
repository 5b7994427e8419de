"""Pure-Python reference evaluations -- TEST INFRASTRUCTURE ONLY.

Small, slow and exact: rational arithmetic (fractions.Fraction), one point and
one ring at a time. Used to pin the C oracle on hand-made shapes.

* ``crossing_inside``: the crossing-number test of Sec. III-A written out
  literally -- intersect the boundary with the horizontal line through the
  point, keep the intersections strictly to the right, count them, odd means
  inside. An edge takes part when exactly one end lies strictly above the
  line (half-open rule; horizontal edges never take part).
* ``winding_number``: an independent formula (Sunday's winding number with the
  same half-open edge rules), nonzero exactly when a simple ring contains the
  point.
* ``quantize_lonlat``: longitude/latitude doubles (Sec. II) to integer fixed
  point; see the function for the reading of the unspecified constants.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def crossing_inside(ring, px: int, py: int) -> bool:
    """Exact crossing-number test; ring is a sequence of (x, y) integer vertices,
    implicitly closed from the last vertex to the first."""
    m = len(ring)
    count = 0
    for k in range(m):
        ax, ay = ring[k]
        bx, by = ring[(k + 1) % m]
        if (ay > py) == (by > py):
            continue
        x_int = Fraction(ax) + Fraction((py - ay) * (bx - ax), by - ay)
        if x_int > px:
            count += 1
    return count % 2 == 1


def winding_number(ring, px: int, py: int) -> int:
    """Signed number of turns of the ring around the point (half-open rules):
    an upward edge counts +1 when the point is strictly left of it, a downward
    edge -1 when the point is strictly right of it."""
    m = len(ring)
    wn = 0
    for k in range(m):
        ax, ay = ring[k]
        bx, by = ring[(k + 1) % m]
        side = (bx - ax) * (py - ay) - (px - ax) * (by - ay)  # > 0: point left of a->b
        if ay <= py:
            if by > py and side > 0:
                wn += 1
        elif by <= py and side < 0:
            wn -= 1
    return wn


def smallest_containing(rings, px: int, py: int) -> int:
    for b, r in enumerate(rings):
        if crossing_inside(r, px, py):
            return b
    return -1


# Quantiser. The paper stores locations as IEEE doubles (Sec. II) and gives no
# fixed-point encoding; the reading used here: q = rint(v * 2^22) + 2^30 per
# axis, rint rounding half to even, the offset added after rounding in integer
# arithmetic; NaN, infinities, |lon| > 180 and |lat| > 90 give (-1, -1).
QSCALE = 2 ** 22
QOFFSET = 2 ** 30


def quantize_lonlat(lonlat) -> np.ndarray:
    a = np.asarray(lonlat, dtype=np.float64).reshape(-1, 2)
    out = np.empty(a.shape, dtype=np.int32)
    for i, (lon, lat) in enumerate(a.tolist()):
        ok = (math.isfinite(lon) and math.isfinite(lat) and abs(lon) <= 180.0
              and abs(lat) <= 90.0)
        if ok:
            # Python's round() of a float is exact and ties to even
            out[i, 0] = round(lon * QSCALE) + QOFFSET
            out[i, 1] = round(lat * QSCALE) + QOFFSET
        else:
            out[i] = (-1, -1)
    return out
