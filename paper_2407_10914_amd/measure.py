"""Geometric observables read from an exported phase field (host side).

The paper reads the contact angle of a sessile drop from the base b and the
height h of the drop (Sec. III.B, Eqs. 45-46): with the cap radius
r = (4 h^2 + b^2) / (8 h), theta = arctan((b/2) / (r - h)); it is written here
with atan2 so that caps taller than a half disc (theta > 90 deg) keep their
angle.  The angle is the drop's own, measured through the drop's fluid; an
input angle given through the surrounding fluid is 180 deg minus it.  The
imbibition front of the capillary tube (Sec. IV.A) is where the phase field
on the tube axis changes sign, or, from volumes, the red volume divided by
the cross-section.  Interface points are the phi = 0 crossings of the
linearly interpolated field.  None of this is on the time step.
"""
from __future__ import annotations

import math

import numpy as np


def crossings(values, positions=None):
    """Positions where a 1D profile changes sign (linear interpolation).

    `positions` are the coordinates of the samples (default 0, 1, 2, ...)."""
    v = np.asarray(values, dtype=np.float64)
    x = np.arange(len(v), dtype=np.float64) if positions is None else np.asarray(positions, dtype=np.float64)
    out = []
    for k in range(len(v) - 1):
        a, b = v[k], v[k + 1]
        if a == 0.0:
            out.append(x[k])
        elif a * b < 0.0:
            out.append(x[k] + (x[k + 1] - x[k]) * a / (a - b))
    if len(v) and v[-1] == 0.0:
        out.append(x[-1])
    return out


def cap_angle(base: float, height: float) -> float:
    """Contact angle in degrees of a circular cap of base b and height h
    (Eqs. 45-46, through the cap's fluid)."""
    if not (base > 0.0 and height > 0.0):
        raise ValueError("base and height must be positive")
    r = (4.0 * height * height + base * base) / (8.0 * height)
    return math.degrees(math.atan2(base / 2.0, r - height))


def drop_base_height(phi2d, wall: float = 0.5, row: int | None = None, sign: float = 1.0):
    """Base and height of a drop (phi * sign > 0 inside) resting on a wall at
    y = `wall` (halfway bounce-back: the wall lies half a node below the first
    fluid row).  phi2d is indexed [y, x].  The base is the distance between the
    two interface points on the first fluid row (`row`, default the row just
    above the wall); the height is the interface point on the drop's axis (the
    midpoint of the base), measured from the wall."""
    ph = np.asarray(phi2d, dtype=np.float64) * sign
    ny, nx = ph.shape
    if row is None:
        row = int(math.floor(wall + 0.5))
    xs = crossings(ph[row])
    inside = ph[row] > 0
    if len(xs) < 2 or not inside.any():
        raise ValueError("no drop on the first fluid row")
    base = xs[-1] - xs[0]
    axis = 0.5 * (xs[0] + xs[-1])
    # profile along y on the axis, interpolated between the two nearest columns
    x0 = int(math.floor(axis))
    t = axis - x0
    col = (1.0 - t) * ph[:, x0] + t * ph[:, min(x0 + 1, nx - 1)]
    ys = [y for y in crossings(col[row:], np.arange(row, ny)) if y > row]
    if not ys:
        raise ValueError("no interface above the wall on the drop axis")
    height = ys[0] - wall
    return base, height


def drop_angle(phi2d, wall: float = 0.5, row: int | None = None, sign: float = 1.0) -> float:
    """Contact angle (degrees, through the drop) of a sessile drop, Eqs. 45-46."""
    b, h = drop_base_height(phi2d, wall=wall, row=row, sign=sign)
    return cap_angle(b, h)


def front_on_axis(phi, axis: int = 0, line=None):
    """Interface position along `axis` on one grid line (the tube axis): the
    first phi = 0 crossing from the low end.  `line` holds the indices of the
    other axes in their order (default: the middle of each)."""
    ph = np.moveaxis(np.asarray(phi, dtype=np.float64), axis, -1)
    if line is None:
        line = tuple(n // 2 for n in ph.shape[:-1])
    xs = crossings(ph[tuple(line)])
    return xs[0] if xs else float("nan")


def front_from_volume(phi, fluid, area: float, sign: float = 1.0) -> float:
    """Volume-based front position: the volume of the fluid with phi * sign > 0,
    sum over fluid nodes of (1 + sign phi)/2, divided by the cross-section."""
    ph = np.asarray(phi, dtype=np.float64) * sign
    m = np.asarray(fluid, dtype=bool)
    return float(np.sum((1.0 + ph[m]) * 0.5) / area)
