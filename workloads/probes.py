"""Scalar sampling locations: the 24 wall and roof points of Table 1 and the
two points of the scalar-CDF figure (section 3), in the canyon coordinates of
this package.

The paper's coordinates are in units of h = H/2 with the canyon between
x = 2 and x = 4 and the roofs at y = 2; here H = 1, the canyon spans
[x_l, x_r] = [0.5, 1.5] and the domain is periodic over [0, 2).  A point
(x, y) of the paper maps to ((x - 2)/2 + 0.5 mod 2, y/2).  Points on a wall
are placed on that wall of the given geometry, which moves them onto the
stripped boundary (by y_p) for the wall-function mesh.

Reading of a garbled entry: Table 1 lists point 10 at x = 2.5, y = 0.5, in
the middle of a column of points on the wall x = 2 (y = 0.67, 0.5, 0.33) and
opposite point 15 at (4, 0.5); it is taken as (2, 0.5).
"""
from __future__ import annotations

from typing import List, Tuple

# Table 1, paper units (point 10 as read above)
TABLE1 = [(0.5, 2.0), (1.0, 2.0), (1.5, 2.0), (2.0, 2.0), (2.0, 1.93), (2.0, 1.5), (2.0, 1.33), (2.0, 1.0),
          (2.0, 0.67), (2.0, 0.5), (2.0, 0.33), (2.0, 0.17),
          (4.0, 0.17), (4.0, 0.33), (4.0, 0.5), (4.0, 0.67), (4.0, 1.0), (4.0, 1.33), (4.0, 1.5), (4.0, 1.93),
          (4.0, 2.0), (4.5, 2.0), (5.0, 2.0), (5.5, 2.0)]

# the scalar-CDF figure: above the street and at roof level, mid-canyon
CDF_POINTS = [(3.0, 0.2), (3.0, 2.0)]


def _map(x: float, y: float, geo) -> Tuple[float, float]:
    X = ((x - 2.0) / 2.0 + 0.5) % 2.0
    Y = y / 2.0
    if x == 2.0 and y <= 2.0:          # wall of the upstream building (and its corner)
        X = geo.x_l
    if x == 4.0 and y <= 2.0:          # wall of the downstream building
        X = geo.x_r
    if y == 2.0:                       # roof tops
        Y = geo.y_roof
    return X, Y


def table1_points(geo) -> List[Tuple[float, float]]:
    """The 24 Table 1 locations on the walls and roofs of the given geometry."""
    return [_map(x, y, geo) for x, y in TABLE1]


def cdf_points(geo) -> List[Tuple[float, float]]:
    """The two CDF locations (inside the flow, not on walls)."""
    return [(((x - 2.0) / 2.0 + 0.5) % 2.0, y / 2.0) for x, y in CDF_POINTS]
