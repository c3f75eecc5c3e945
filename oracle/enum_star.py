"""Independent pure-Python enumerator of the octagonal star, for tiny inputs.

TEST INFRASTRUCTURE ONLY.  It pins the C oracle by building the star's two
pixel sets explicitly (Sec. "Rotation Invariance", Fig. os: a square and a
45-degree diamond of the same size, superimposed) rather than by evaluating
a weight predicate, and by deriving the square's half-width geometrically
as the integer nearest to r / sqrt(2) (the half-width of a square congruent
to a diamond whose vertices lie r pixels from the centre), computed with
exact integer arithmetic.
"""
from __future__ import annotations

from math import isqrt


def nearest_half_width(r: int) -> int:
    """Nearest integer to r / sqrt(2): the largest s with s - 1/2 < r/sqrt(2),
    i.e. (2s - 1)^2 < 2 r^2.  Evaluated as floor(r/sqrt(2) + 1/2) through
    isqrt on 2 r^2 scaled by 4 so no floating point is involved."""
    # floor(sqrt(2 r^2)) is r*sqrt(2) rounded down; floor(r/sqrt(2) + 1/2)
    # = floor((sqrt(2 r^2) + 1) / 2) because sqrt(2 r^2) = 2 * r/sqrt(2) is
    # irrational for r > 0 and the floor commutes with the monotone map.
    if r == 0:
        return 0
    return (isqrt(2 * r * r) + 1) // 2


def square_pixels(r: int):
    s = nearest_half_width(r)
    return [(dx, dy) for dy in range(-s, s + 1) for dx in range(-s, s + 1)]


def diamond_pixels(r: int):
    out = []
    for dy in range(-r, r + 1):
        span = r - abs(dy)
        for dx in range(-span, span + 1):
            out.append((dx, dy))
    return out


def gradient_at(img, x: int, y: int) -> int:
    H, W = len(img), len(img[0])
    xr, xl = min(x + 1, W - 1), max(x - 1, 0)
    yd, yu = min(y + 1, H - 1), max(y - 1, 0)
    return abs(int(img[y][xr]) - int(img[y][xl])) + abs(int(img[yd][x]) - int(img[yu][x]))


def star_features(img, x: int, y: int, r: int):
    """(sum I, sum I^2, sum G) over square + diamond, or None if the star
    leaves the image.  ``img`` is a list of rows of ints."""
    H, W = len(img), len(img[0])
    if not (r <= x <= W - 1 - r and r <= y <= H - 1 - r):
        return None
    f = [0, 0, 0]
    for dx, dy in square_pixels(r) + diamond_pixels(r):
        v = int(img[y + dy][x + dx])
        f[0] += v
        f[1] += v * v
        f[2] += gradient_at(img, x + dx, y + dy)
    return tuple(f)


def area(r: int) -> int:
    return len(square_pixels(r)) + len(diamond_pixels(r))
