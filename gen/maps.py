"""Seeded occupancy maps (uint8, shape (H, W), 1 = occupied, 0 = free).

Row index j is the world y axis and column index i the world x axis.  The
outermost ring of cells is always a wall, so every map is closed.
"""

from __future__ import annotations

import numpy as np


def occupancy_fraction(occ: np.ndarray) -> float:
    return float(np.count_nonzero(occ)) / occ.size


def _split_rooms(occ, rng, x0, y0, x1, y1, *, min_room, wall, door, corridor_p,
                 corridor_w, depth):
    """Recursively partition the free rectangle [x0,x1) x [y0,y1) with walls.

    Each partition wall is `wall` cells thick and carries one `door`-cell
    doorway.  With probability `corridor_p` (only near the top of the
    recursion) the partition is a corridor: two parallel walls `corridor_w`
    apart, each with its own doorway.
    """
    w, h = x1 - x0, y1 - y0
    make_corridor = depth < 2 and rng.random() < corridor_p
    span = 2 * min_room + (2 * wall + corridor_w if make_corridor else wall)
    can_v, can_h = w >= span, h >= span
    if not (can_v or can_h):
        return
    if can_v and can_h:
        vertical = (w > h) if rng.random() < 0.75 else bool(rng.random() < 0.5)
    else:
        vertical = can_v

    def doorway(lo, hi):
        d = min(door, hi - lo)
        s = int(rng.integers(lo, hi - d + 1))
        return s, s + d

    if vertical:
        lo = x0 + min_room
        hi = x1 - min_room - (2 * wall + corridor_w if make_corridor else wall)
        x = int(rng.integers(lo, hi + 1))
        walls = [x] if not make_corridor else [x, x + wall + corridor_w]
        for wx in walls:
            occ[y0:y1, wx:wx + wall] = 1
            a, b = doorway(y0, y1)
            occ[a:b, wx:wx + wall] = 0
        if make_corridor:
            # the corridor itself stays open along its whole length
            _split_rooms(occ, rng, x0, y0, x, y1, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
            xr = x + 2 * wall + corridor_w
            _split_rooms(occ, rng, xr, y0, x1, y1, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
        else:
            _split_rooms(occ, rng, x0, y0, x, y1, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
            _split_rooms(occ, rng, x + wall, y0, x1, y1, min_room=min_room, wall=wall,
                         door=door, corridor_p=corridor_p, corridor_w=corridor_w,
                         depth=depth + 1)
    else:
        lo = y0 + min_room
        hi = y1 - min_room - (2 * wall + corridor_w if make_corridor else wall)
        y = int(rng.integers(lo, hi + 1))
        walls = [y] if not make_corridor else [y, y + wall + corridor_w]
        for wy in walls:
            occ[wy:wy + wall, x0:x1] = 1
            a, b = doorway(x0, x1)
            occ[wy:wy + wall, a:b] = 0
        if make_corridor:
            _split_rooms(occ, rng, x0, y0, x1, y, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
            yb = y + 2 * wall + corridor_w
            _split_rooms(occ, rng, x0, yb, x1, y1, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
        else:
            _split_rooms(occ, rng, x0, y0, x1, y, min_room=min_room, wall=wall, door=door,
                         corridor_p=corridor_p, corridor_w=corridor_w, depth=depth + 1)
            _split_rooms(occ, rng, x0, y + wall, x1, y1, min_room=min_room, wall=wall,
                         door=door, corridor_p=corridor_p, corridor_w=corridor_w,
                         depth=depth + 1)


def bsp_rooms(width: int, height: int, seed: int, *, door: int = 8,
              min_room: int = 10) -> np.ndarray:
    """Axis-aligned rectangular rooms with 1-cell walls and `door`-cell doorways.

    A binary space partition of the interior: every partition wall is one
    cell thick and has exactly one doorway, so all rooms are connected.
    """
    rng = np.random.default_rng(seed)
    occ = np.zeros((height, width), np.uint8)
    occ[0, :] = occ[-1, :] = 1
    occ[:, 0] = occ[:, -1] = 1
    _split_rooms(occ, rng, 1, 1, width - 1, height - 1, min_room=min_room, wall=1,
                 door=door, corridor_p=0.0, corridor_w=0, depth=0)
    return occ


def rooms_and_corridors(width: int, height: int, seed: int, *,
                        target_occupied: float = 0.35, tolerance: float = 0.02,
                        wall: int = 2, door: int = 16, min_room: int = 36,
                        corridor_w: int = 28) -> np.ndarray:
    """Room-and-corridor floor plan plus furniture-like clutter.

    Rooms and corridors come from a partition as in `bsp_rooms` (thicker
    walls, wider doorways, corridors near the top of the recursion).  Then
    rectangular clutter blocks are dropped on free cells away from doorways
    until the occupied fraction reaches `target_occupied` (to `tolerance`).
    """
    rng = np.random.default_rng(seed)
    occ = np.zeros((height, width), np.uint8)
    occ[:wall, :] = occ[-wall:, :] = 1
    occ[:, :wall] = occ[:, -wall:] = 1
    _split_rooms(occ, rng, wall, wall, width - wall, height - wall, min_room=min_room,
                 wall=wall, door=door, corridor_p=0.6, corridor_w=corridor_w, depth=0)
    doors_free = occ.copy()
    lo = max(3, min(width, height) // 128)
    hi = max(lo + 2, min(width, height) // 16)
    guard = 0
    while occupancy_fraction(occ) < target_occupied - tolerance / 2 and guard < 100000:
        guard += 1
        bw = int(rng.integers(lo, hi + 1))
        bh = int(rng.integers(lo, hi + 1))
        x = int(rng.integers(wall, width - wall - bw))
        y = int(rng.integers(wall, height - wall - bh))
        # keep a margin around walls so doorways stay passable
        m = 3
        ya, yb = max(0, y - m), min(height, y + bh + m)
        xa, xb = max(0, x - m), min(width, x + bw + m)
        if doors_free[ya:yb, xa:xb].any():
            continue
        occ[y:y + bh, x:x + bw] = 1
        if occupancy_fraction(occ) > target_occupied + tolerance:
            occ[y:y + bh, x:x + bw] = 0
            doors_free[y:y + bh, x:x + bw] = 1  # do not retry this spot
    return occ
