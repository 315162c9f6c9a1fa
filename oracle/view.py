"""Oracle of the view-dependent node selection (TEST INFRASTRUCTURE ONLY:
imported by tests/, and by nothing under paper_2302_05002_amd/).

Section "Octree Rendering": a traversal thread walks the octree with the
camera's position and frustum, checks each node's visibility, and queues the
nodes to draw.  The paper gives no formulas; the readings are:

  * geometry: a node at depth d with cell (cx, cy, cz) (its Morton key
    de-interleaved) covers, per axis, lo = m + c * s and hi = m + (c + 1) * s
    with s = side / 2^d, where m is the cloud's box minimum and side its cube
    side (float32 values taken as doubles).  Centre = m + (2c + 1) * (s / 2);
    radius = (s / 2) * 1.7320508075688772 (the double nearest sqrt(3)).
  * visibility: a frustum plane (a, b, c, e) keeps a*x + b*y + c*z + e >= 0.
    A node is visible unless, for some plane, its corner farthest along the
    plane's normal (hi where the normal's component is >= 0, else lo) gives
    ((a*px + b*py) + c*pz) + e < 0.
  * size on screen: dist = sqrt((dx*dx + dy*dy) + dz*dz) from the eye to the
    centre; infinite when dist <= radius, else proj_factor * (radius / dist)
    pixels.
  * traversal: from the root; an invisible node is skipped with its subtree;
    a visible node is drawn, and its children are visited when its size on
    screen is at least min_size pixels.

All arithmetic is IEEE double with one rounding per operation (Python floats).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

SQRT3 = 1.7320508075688772


@dataclass
class View:
    eye: tuple            # camera position
    planes: tuple         # six (a, b, c, e) tuples
    proj_factor: float    # viewport height / (2 tan(fov_y / 2))
    min_size: float       # pixels


def cell_of(key: int, depth: int):
    """De-interleave a Morton key (x the most significant bit of each triple)."""
    c = [0, 0, 0]
    for b in range(depth):
        t = (key >> (3 * b)) & 7
        c[0] |= ((t >> 2) & 1) << b
        c[1] |= ((t >> 1) & 1) << b
        c[2] |= (t & 1) << b
    return c


def node_box(depth, cell, bmin, side):
    s = float(side) / float(2 ** depth)
    lo = [float(bmin[a]) + cell[a] * s for a in range(3)]
    hi = [float(bmin[a]) + (cell[a] + 1) * s for a in range(3)]
    ctr = [float(bmin[a]) + (2 * cell[a] + 1) * (s / 2) for a in range(3)]
    return lo, hi, ctr, (s / 2) * SQRT3


def visible(lo, hi, planes) -> bool:
    for a, b, c, e in planes:
        px = hi[0] if a >= 0 else lo[0]
        py = hi[1] if b >= 0 else lo[1]
        pz = hi[2] if c >= 0 else lo[2]
        if ((a * px + b * py) + c * pz) + e < 0:
            return False
    return True


def screen_size(ctr, radius, view: View) -> float:
    dx, dy, dz = ctr[0] - view.eye[0], ctr[1] - view.eye[1], ctr[2] - view.eye[2]
    dist = math.sqrt((dx * dx + dy * dy) + dz * dz)
    if dist <= radius:
        return math.inf
    return view.proj_factor * (radius / dist)


def select_nodes(node_depth, node_key, node_count, bmin, side, view: View):
    """(ascending indices of the drawn nodes, their total point count)."""
    index = {(int(d), int(k)): i for i, (d, k) in enumerate(zip(node_depth, node_key))}
    out = []
    if (0, 0) not in index:
        return out, 0
    stack = [(0, 0)]
    while stack:
        d, k = stack.pop()
        lo, hi, ctr, r = node_box(d, cell_of(k, d), bmin, side)
        if not visible(lo, hi, view.planes):
            continue
        out.append(index[(d, k)])
        if screen_size(ctr, r, view) >= view.min_size:
            for o in range(8):
                ch = (d + 1, (k << 3) | o)
                if ch in index:
                    stack.append(ch)
    out.sort()
    return out, int(sum(int(node_count[i]) for i in out))


def perspective_view(eye, target, up, fov_y_deg, aspect, near, far, viewport_height, min_size) -> View:
    """A perspective camera's six planes (left, right, bottom, top, near, far)
    from its position, target, up vector and field of view (test helper)."""
    f = [target[a] - eye[a] for a in range(3)]
    fl = math.sqrt(sum(v * v for v in f))
    f = [v / fl for v in f]
    r = [f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]]
    rl = math.sqrt(sum(v * v for v in r))
    r = [v / rl for v in r]
    u = [r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]]
    th = math.tan(math.radians(fov_y_deg) / 2)
    tw = th * aspect
    planes = []

    def plane(n, p):
        planes.append((n[0], n[1], n[2], -(n[0] * p[0] + n[1] * p[1] + n[2] * p[2])))

    # inside: |(p - eye) . r| <= tw * (p - eye) . f, likewise for u and th
    plane([tw * f[a] + r[a] for a in range(3)], eye)
    plane([tw * f[a] - r[a] for a in range(3)], eye)
    plane([th * f[a] + u[a] for a in range(3)], eye)
    plane([th * f[a] - u[a] for a in range(3)], eye)
    plane(f, [eye[a] + near * f[a] for a in range(3)])
    plane([-v for v in f], [eye[a] + far * f[a] for a in range(3)])
    return View(tuple(eye), tuple(planes), viewport_height / (2 * th), min_size)
