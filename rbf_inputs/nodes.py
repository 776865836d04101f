"""Jittered staggered node sets (stand-in for the DistMesh grids of Sec. 3).

The paper puts pressure on the vertices of an unstructured triangulation (the
P-grid) and velocity on the edge midpoints (the V-grid), N/M ~ 3.  DistMesh is
not available, so the cavity uses a seeded jittered triangulation of the unit
square with the same staggering (``cavity_nodes``).  The operator benchmark
uses two jittered square lattices with N = M (``square_nodes``): V on cell
centres, P on vertices.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used
as a counter-based generator: draw c of stream g is mix(seed + (c'+1)*GAMMA)
with c' = (g << 40) | c, and a uniform double is (draw >> 11) * 2**-53.
The C library implements the same published definition independently; every
floating-point operation below is a single IEEE-754 rounding (no fused
multiply-add), so both produce bit-identical coordinates.

Layout: coordinates are SoA, ``x[2, n]`` (row 0 = x, row 1 = y), in a
row-major lattice order (j outer, i inner) so that stencil neighbours are
close in memory.
"""
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

TAG_INTERIOR = 0
TAG_WALL = 1
TAG_LID = 2

STREAM_V = 0
STREAM_P = 1
SQRT_HALF = 0.7071067811865476  # 1/sqrt(2) rounded to nearest


def splitmix64(seed, counters):
    """SplitMix64 output for the given 64-bit counters (vectorised)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counters, dtype=np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def uniform01(seed, stream, counters):
    """Uniform doubles in [0, 1) for draws ``counters`` of ``stream``."""
    c = (np.uint64(stream) << np.uint64(40)) | np.asarray(counters, dtype=np.uint64)
    return (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _jitter(seed, stream, node_index, amp):
    """Offsets (2u-1)*amp for x (draw 2i) and y (draw 2i+1) of each node."""
    node_index = np.asarray(node_index, dtype=np.uint64)
    ux = uniform01(seed, stream, np.uint64(2) * node_index)
    uy = uniform01(seed, stream, np.uint64(2) * node_index + np.uint64(1))
    return (2.0 * ux - 1.0) * amp, (2.0 * uy - 1.0) * amp


@dataclass
class NodeSet:
    """A staggered pair of node sets with boundary information."""
    xv: np.ndarray        # float64 [2, N]
    v_tag: np.ndarray     # int8 [N]: 0 interior, 1 wall, 2 lid
    xp: np.ndarray        # float64 [2, M]
    p_tag: np.ndarray     # int8 [M]: 0 interior, 1 wall
    p_normal: np.ndarray  # float64 [2, M], outward unit normal on wall P-nodes, 0 elsewhere
    K: int
    h: float

    @property
    def n_v(self):
        return self.xv.shape[1]

    @property
    def n_p(self):
        return self.xp.shape[1]


def cavity_nodes(K, jitter=0.3, seed=0):
    """Unit-square cavity on the paper's staggered layout (Sec. 3).

    P-grid: the vertices (i h, j h), i, j = 0..K, h = 1/K, of a triangulation
    of the square; interior vertices are jittered by U(-jitter h, jitter h)
    per coordinate (draws 2v, 2v+1 of stream P for vertex v = j (K+1) + i),
    boundary vertices (corners included) stay on the walls.  Each lattice cell
    (i, j) is split into two triangles by a diagonal whose direction
    alternates like a checkerboard: (i,j)-(i+1,j+1) when i+j is even,
    (i+1,j)-(i,j+1) when odd.
    V-grid: the midpoints (a + b) * 0.5 of all triangle edges.
    Counts: M = (K+1)^2, N = 3K^2 + 2K (N/M ~ 3, as in the paper).

    Ordering: P row-major over vertices (j outer).  V by owning vertex in the
    same order: vertex (i, j) emits its rightward edge (if i < K), its upward
    edge (if j < K) and the diagonal of cell (i, j) (if i, j < K).
    Tags: wall edges/vertices are 1, V-nodes on the top wall are 2 (lid).
    P normals are outward; at corners the diagonal (+-1, +-1)/sqrt(2).
    """
    if K < 2:
        raise ValueError("K must be >= 2")
    h = 1.0 / K
    amp = jitter * h
    n1 = K + 1
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n1), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    M = n1 * n1
    interior = (ii > 0) & (ii < K) & (jj > 0) & (jj < K)
    ox, oy = _jitter(seed, STREAM_P, np.arange(M), amp)
    px = np.where(ii == K, 1.0, ii * h)
    py = np.where(jj == K, 1.0, jj * h)
    px = np.where(interior, px + ox, px)
    py = np.where(interior, py + oy, py)
    p_tag = np.where(interior, TAG_INTERIOR, TAG_WALL).astype(np.int8)
    nx = np.where(ii == 0, -1.0, np.where(ii == K, 1.0, 0.0))
    ny = np.where(jj == 0, -1.0, np.where(jj == K, 1.0, 0.0))
    corner = (nx != 0.0) & (ny != 0.0)
    nx = np.where(corner, nx * SQRT_HALF, nx)
    ny = np.where(corner, ny * SQRT_HALF, ny)
    # Edges, grouped by owning vertex in row-major order.
    vid = jj * n1 + ii
    right = ii < K
    up = jj < K
    cell = right & up
    even = (ii + jj) % 2 == 0
    ea = np.stack([vid, vid, np.where(even, vid, vid + 1)])
    eb = np.stack([vid + 1, vid + n1, np.where(even, vid + n1 + 1, vid + n1)])
    keep = np.stack([right, up, cell])
    ea = ea.T[keep.T]
    eb = eb.T[keep.T]
    vx = (px[ea] + px[eb]) * 0.5
    vy = (py[ea] + py[eb]) * 0.5
    on_wall = (p_tag[ea] != TAG_INTERIOR) & (p_tag[eb] != TAG_INTERIOR) & (
        (px[ea] == px[eb]) & ((px[ea] == 0.0) | (px[ea] == 1.0))
        | (py[ea] == py[eb]) & ((py[ea] == 0.0) | (py[ea] == 1.0)))
    lid = on_wall & (vy == 1.0)
    v_tag = np.where(lid, TAG_LID, np.where(on_wall, TAG_WALL, TAG_INTERIOR)).astype(np.int8)
    return NodeSet(np.stack([vx, vy]), v_tag, np.stack([px, py]), p_tag,
                   np.stack([nx, ny]), K, h)


def hex_rows(K):
    """Row count R = floor(2K/sqrt(3) + 1/2) of the near-equilateral cavity:
    rows y_j = j/R are about sqrt(3)/2 h apart, h = 1/K."""
    return int(np.floor(2.0 * K / np.sqrt(3.0) + 0.5))


def hex_cavity_nodes(K, jitter=0.3, seed=0):
    """Unit-square cavity on a near-equilateral triangulation (the kind of
    grid DistMesh produces, Sec. 3; rbf_build_nodes kind 2).

    P-grid, row by row (j = 0..R, y_j = j/R, R = ``hex_rows(K)``, h = 1/K):
    rows 0 and R are the bottom and top walls with x = i h, i = 0..K; an even
    interior row holds x = 0, h, 2h, ..., (K-1)h, 1 and an odd one x = 0,
    h/2, 3h/2, ..., (K-1/2)h, 1 (first and last node on the side walls).
    Interior vertices whose unjittered distance to the nearest wall is at
    least 1.5 h are jittered by U(-jitter h, jitter h) per coordinate (draws
    2v, 2v+1 of stream P for vertex v in this order); the band next to the
    walls stays on the rows (with jitter there the Kim-Moin wall values of
    eq. (21) feed a growing near-wall mode).
    Edges: the horizontal edges of each row, and between rows j and j+1 the
    strip triangulation obtained by merging the two rows in order of their
    unjittered x (from the left-wall edge, advance in the lower row while its
    next x is not greater than the upper row's next x, else in the upper
    row; each advance adds one edge and one triangle).  Valid for
    jitter < K/(2R) (about 0.43).
    V-grid: edge midpoints (a + b) * 0.5, ordered row by row: row j's
    horizontal edges left to right, then the strip edges of rows (j, j+1) in
    merge order.  Tags and normals as in ``cavity_nodes``."""
    if K < 2:
        raise ValueError("K must be >= 2")
    h = 1.0 / K
    R = hex_rows(K)
    keys, start = [], []
    px, py, tag = [], [], []
    for j in range(R + 1):
        y = 1.0 if j == R else j / R
        start.append(len(keys))
        if j == 0 or j == R:
            xs = [1.0 if i == K else i * h for i in range(K + 1)]
            tg = [TAG_WALL] * (K + 1)
        elif j % 2 == 0:
            xs = [0.0] + [i * h for i in range(1, K)] + [1.0]
            tg = [TAG_WALL] + [TAG_INTERIOR] * (K - 1) + [TAG_WALL]
        else:
            xs = [0.0] + [(i + 0.5) * h for i in range(K)] + [1.0]
            tg = [TAG_WALL] + [TAG_INTERIOR] * K + [TAG_WALL]
        keys += xs
        py += [y] * len(xs)
        tag += tg
    start.append(len(keys))
    key = np.array(keys)
    px = key.copy()
    py = np.array(py)
    p_tag = np.array(tag, np.int8)
    M = px.size
    dw = np.minimum(np.minimum(px, py), np.minimum(1.0 - px, 1.0 - py))
    jit = (p_tag == TAG_INTERIOR) & (dw >= 1.5 * h)
    ox, oy = _jitter(seed, STREAM_P, np.arange(M), jitter * h)
    px = np.where(jit, px + ox, px)
    py = np.where(jit, py + oy, py)
    ea, eb = [], []
    for j in range(R + 1):
        a0, a1 = start[j], start[j + 1]
        ea += list(range(a0, a1 - 1))
        eb += list(range(a0 + 1, a1))
        if j == R:
            break
        b1 = start[j + 2]
        ia, ib = a0, a1
        ea.append(ia)
        eb.append(ib)
        while ia < a1 - 1 or ib < b1 - 1:
            if ia == a1 - 1:
                ib += 1
            elif ib == b1 - 1:
                ia += 1
            elif key[ia + 1] <= key[ib + 1]:
                ia += 1
            else:
                ib += 1
            ea.append(ia)
            eb.append(ib)
    ea, eb = np.array(ea), np.array(eb)
    vx = (px[ea] + px[eb]) * 0.5
    vy = (py[ea] + py[eb]) * 0.5
    on_wall = (p_tag[ea] != TAG_INTERIOR) & (p_tag[eb] != TAG_INTERIOR) & (
        (px[ea] == px[eb]) & ((px[ea] == 0.0) | (px[ea] == 1.0))
        | (py[ea] == py[eb]) & ((py[ea] == 0.0) | (py[ea] == 1.0)))
    lid = on_wall & (vy == 1.0)
    v_tag = np.where(lid, TAG_LID, np.where(on_wall, TAG_WALL, TAG_INTERIOR)).astype(np.int8)
    wall = p_tag != TAG_INTERIOR
    nx = np.where(wall & (px == 0.0), -1.0, np.where(wall & (px == 1.0), 1.0, 0.0))
    ny = np.where(wall & (py == 0.0), -1.0, np.where(wall & (py == 1.0), 1.0, 0.0))
    corner = (nx != 0.0) & (ny != 0.0)
    nx = np.where(corner, nx * SQRT_HALF, nx)
    ny = np.where(corner, ny * SQRT_HALF, ny)
    return NodeSet(np.stack([vx, vy]), v_tag, np.stack([px, py]), p_tag,
                   np.stack([nx, ny]), K, h)


TAG_CYLINDER = 1
TAG_INFLOW = 3
TAG_OUTFLOW = 4
TAG_SIDE = 5


def cylinder_nodes(h_wall=0.02, grading=0.008, h_far=0.5, box=(-10.0, 30.0, -10.0, 10.0)):
    """Staggered nodes for flow past a cylinder (Sec. 5.2 geometry: diameter
    1 at the origin, in the channel ``box``), graded from spacing ``h_wall``
    on the cylinder to at most ``h_far`` with h(r) = min(h_far, h_wall +
    grading (r - 1/2)): P-nodes on rings of radius r_k (r_0 = 1/2, r_{k+1} =
    r_k + h(r_k) sqrt(3)/2, round(2 pi r_k / h(r_k)) nodes (an even number,
    2 round(pi r_0 / h(r_0)), on the cylinder itself), every other ring
    rotated by half a spacing) kept 1.5 local spacings clear of the channel
    edges, plus channel-edge nodes at the local spacing and a regular row
    beside each edge (gap midpoints moved inward by sqrt(3)/2 of the gap; a
    clipped-ring layer at the edges gives a growing mode there); the Delaunay triangulation of those vertices
    without the triangles inside the cylinder gives the edges, and V-nodes
    are their midpoints.  Deterministic (no random draws).  Tags: 0
    interior, 1 cylinder, 3 inflow (x = x0), 4 outflow (x = x1), 5 sides
    (y = y0, y1; corners count as sides).  P normals point out of the fluid.
    The defaults give 132,565 P- and 396,685 V-nodes."""
    from scipy.spatial import Delaunay
    x0, x1, y0, y1 = box
    hr = lambda r: np.minimum(h_far, h_wall + grading * (r - 0.5))  # noqa: E731
    rmax = max(np.hypot(x, y) for x in (x0, x1) for y in (y0, y1))
    px, py, tag = [], [], []
    r, k = 0.5, 0
    while r < rmax:
        h = float(hr(r))
        n = max(8, int(round(2 * np.pi * r / h)))
        if k == 0:  # an even count on the cylinder (composite Simpson's rule)
            n = 2 * max(4, int(round(np.pi * r / h)))
        th = (np.arange(n) + 0.5 * (k % 2)) * (2 * np.pi / n)
        x, y = r * np.cos(th), r * np.sin(th)
        if k > 0:  # interior rings: clear of the channel edges by half a spacing
            keep = (x > x0 + 1.5 * h) & (x < x1 - 1.5 * h) & (y > y0 + 1.5 * h) & (y < y1 - 1.5 * h)
            x, y = x[keep], y[keep]
        px.append(x)
        py.append(y)
        tag.append(np.full(x.size, TAG_CYLINDER if k == 0 else TAG_INTERIOR, np.int8))
        r += h * np.sqrt(3.0) / 2.0
        k += 1

    def edge(a, b, fixed, horizontal, t):
        # nodes from a to b at the local spacing, endpoints included
        pts = [a]
        while True:
            c = pts[-1]
            q = (c, fixed) if horizontal else (fixed, c)
            nxt = c + float(hr(np.hypot(*q)))
            if nxt >= b - 1e-9:
                if len(pts) > 1 and b - c < 0.5 * (nxt - c):  # no sliver before the corner
                    pts.pop()
                break
            pts.append(nxt)
        pts = np.array(pts + [b])
        # spread the last gap evenly over the edge
        pts = a + (pts - a) * (b - a) / (pts[-1] - a)
        if horizontal:
            return pts, np.full(pts.size, fixed), np.full(pts.size, t, np.int8)
        return np.full(pts.size, fixed), pts, np.full(pts.size, t, np.int8)

    for a, b, fixed, hor, t in ((x0, x1, y0, True, TAG_SIDE), (x0, x1, y1, True, TAG_SIDE),
                                (y0, y1, x0, False, TAG_INFLOW), (y0, y1, x1, False, TAG_OUTFLOW)):
        ex, ey, et = edge(a, b, fixed, hor, t)
        # A regular row along the edge: the midpoints of the edge's gaps moved
        # inward by sqrt(3)/2 of the gap (near-equilateral triangles at the
        # wall; ring nodes keep 1.5 spacings from the edges).
        if hor:
            gap = ex[1:] - ex[:-1]
            mx = 0.5 * (ex[1:] + ex[:-1])
            my = fixed + (1.0 if fixed == y0 else -1.0) * gap * np.sqrt(3.0) / 2.0
            ok = (mx > x0 + 0.75 * gap) & (mx < x1 - 0.75 * gap)
        else:
            gap = ey[1:] - ey[:-1]
            my = 0.5 * (ey[1:] + ey[:-1])
            mx = fixed + (1.0 if fixed == x0 else -1.0) * gap * np.sqrt(3.0) / 2.0
            ok = (my > y0 + 0.75 * gap) & (my < y1 - 0.75 * gap)
        px.append(mx[ok])
        py.append(my[ok])
        tag.append(np.zeros(int(ok.sum()), np.int8))
        if not hor:  # corners belong to the sides
            ex, ey, et = ex[1:-1], ey[1:-1], et[1:-1]
        px.append(ex)
        py.append(ey)
        tag.append(et)
    px, py = np.concatenate(px), np.concatenate(py)
    p_tag = np.concatenate(tag)
    simp = Delaunay(np.stack([px, py], 1)).simplices
    cx, cy = px[simp].mean(axis=1), py[simp].mean(axis=1)
    simp = simp[np.hypot(cx, cy) > 0.5]
    e = np.concatenate([simp[:, [0, 1]], simp[:, [1, 2]], simp[:, [0, 2]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    ea, eb = e[:, 0], e[:, 1]
    vx = (px[ea] + px[eb]) * 0.5
    vy = (py[ea] + py[eb]) * 0.5
    on_cyl = (p_tag[ea] == TAG_CYLINDER) & (p_tag[eb] == TAG_CYLINDER)
    box_a = (p_tag[ea] != TAG_INTERIOR) & (p_tag[ea] != TAG_CYLINDER)
    box_b = (p_tag[eb] != TAG_INTERIOR) & (p_tag[eb] != TAG_CYLINDER)
    vert = box_a & box_b & (px[ea] == px[eb]) & ((px[ea] == x0) | (px[ea] == x1))
    horiz = box_a & box_b & (py[ea] == py[eb]) & ((py[ea] == y0) | (py[ea] == y1))
    v_tag = np.where(on_cyl, TAG_CYLINDER,
                     np.where(vert, np.where(px[ea] == x0, TAG_INFLOW, TAG_OUTFLOW),
                              np.where(horiz, TAG_SIDE, TAG_INTERIOR))).astype(np.int8)
    rr = np.hypot(px, py)
    nx = np.where(p_tag == TAG_CYLINDER, -px / rr, 0.0)
    ny = np.where(p_tag == TAG_CYLINDER, -py / rr, 0.0)
    nx = np.where(p_tag == TAG_INFLOW, -1.0, np.where(p_tag == TAG_OUTFLOW, 1.0, nx))
    ny = np.where(p_tag == TAG_SIDE, np.where(py == y0, -1.0, 1.0), ny)
    return NodeSet(np.stack([vx, vy]), v_tag, np.stack([px, py]), p_tag,
                   np.stack([nx, ny]), 0, h_wall)


def square_nodes(K, jitter=0.3, seed=0):
    """Operator-bench square: K^2 V-nodes ((i+1/2)h, (j+1/2)h) and K^2
    P-nodes (ih, jh), i, j = 0..K-1, h = 1/K, both jittered; no walls."""
    if K < 1:
        raise ValueError("K must be >= 1")
    h = 1.0 / K
    amp = jitter * h
    ii, jj = np.meshgrid(np.arange(K), np.arange(K), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    n = K * K
    ox, oy = _jitter(seed, STREAM_V, np.arange(n), amp)
    vx = (ii + 0.5) * h + ox
    vy = (jj + 0.5) * h + oy
    ox, oy = _jitter(seed, STREAM_P, np.arange(n), amp)
    px = ii * h + ox
    py = jj * h + oy
    return NodeSet(np.stack([vx, vy]), np.zeros(n, np.int8), np.stack([px, py]),
                   np.zeros(n, np.int8), np.zeros((2, n)), K, h)


def build_nodes(kind, K, jitter=0.3, seed=0):
    """kind 0: cavity (right-triangle lattice); kind 1: bench square;
    kind 2: cavity on the near-equilateral triangulation."""
    if kind == 0:
        return cavity_nodes(K, jitter, seed)
    if kind == 1:
        return square_nodes(K, jitter, seed)
    if kind == 2:
        return hex_cavity_nodes(K, jitter, seed)
    raise ValueError(f"unknown node-set kind {kind}")
