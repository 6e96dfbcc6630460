"""Pins of the navigation distance fields (the per-destination walking
distances of sec. 2.1, an input of both the oracle and the library), checked
against definitions that do not use the generator's graph search: the closed
form in an open room, plain Bellman-Ford relaxation on small obstacle maps,
and hand-worked corner cases."""
import math

import numpy as np

from paper_1908_05232_amd import inputs as I


def octile(di, dj, dx, dy):
    # m diagonal steps, then straight steps along the longer offset
    a, b = abs(di), abs(dj)
    m = min(a, b)
    return m * math.hypot(dx, dy) + (a - m) * dx + (b - m) * dy


def relax(walk, sources, dx, dy):
    """Bellman-Ford over the 8-neighbour moves of walkable cells; a diagonal
    move needs both cells beside it walkable (no cutting past a corner)."""
    ny, nx = walk.shape
    d = np.full((ny, nx), np.inf)
    for i, j in sources:
        if walk[j, i]:
            d[j, i] = 0.0
    moves = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1) if (di, dj) != (0, 0)]
    changed = True
    while changed:
        changed = False
        for j in range(ny):
            for i in range(nx):
                if not walk[j, i]:
                    continue
                for di, dj in moves:
                    a, b = i + di, j + dj
                    if not (0 <= a < nx and 0 <= b < ny) or not walk[b, a] or d[b, a] == np.inf:
                        continue
                    if di and dj and not (walk[j, a] and walk[b, i]):
                        continue
                    c = math.hypot(dx, dy) if di and dj else (dx if di else dy)
                    if d[b, a] + c < d[j, i] - 1e-12:
                        d[j, i] = d[b, a] + c
                        changed = True
    return d


def test_open_room_is_the_octile_distance():
    nx, ny, dx, dy = 23, 17, 0.5, 0.8
    walk = np.ones((ny, nx), bool)
    src = (6, 11)
    d = I.distance_field(walk, [src], dx, dy)
    want = np.array([[octile(i - src[0], j - src[1], dx, dy) for i in range(nx)] for j in range(ny)])
    np.testing.assert_allclose(d, want.astype(np.float32), rtol=1e-6)
    # several sources: the nearest one
    srcs = [(0, 0), (22, 16), (11, 3)]
    d = I.distance_field(walk, srcs, dx, dy)
    want = np.array([[min(octile(i - a, j - b, dx, dy) for a, b in srcs) for i in range(nx)]
                     for j in range(ny)])
    np.testing.assert_allclose(d, want.astype(np.float32), rtol=1e-6)


def test_obstacle_maps_equal_plain_relaxation():
    rng = np.random.default_rng(9105)
    for trial in range(4):
        nx, ny = 14 + trial, 11
        walk = rng.random((ny, nx)) > 0.28
        free = np.argwhere(walk)
        j, i = free[rng.integers(len(free))]
        dx, dy = (0.25, 0.25) if trial % 2 == 0 else (0.4, 0.3)
        got = I.distance_field(walk, [(int(i), int(j))], dx, dy)
        want = relax(walk, [(int(i), int(j))], dx, dy)
        assert np.array_equal(np.isinf(got), np.isinf(want)), trial
        fin = np.isfinite(want)
        np.testing.assert_allclose(got[fin], want[fin].astype(np.float32), rtol=1e-6)


def test_no_corner_cutting_and_unreachable_cells():
    dx = dy = 1.0
    # 2 x 2 with the east cell of the bottom row blocked: (0,0) -> (1,1) goes round, not across
    walk = np.array([[True, False], [True, True]])
    d = I.distance_field(walk, [(0, 0)], dx, dy)
    assert d[1, 1] == np.float32(2.0) and d[1, 0] == np.float32(1.0) and np.isinf(d[0, 1])
    # both side cells blocked: the diagonal neighbour is unreachable
    walk = np.array([[True, False], [False, True]])
    d = I.distance_field(walk, [(0, 0)], dx, dy)
    assert d[0, 0] == 0.0 and np.isinf(d[1, 1])
    # a source on an obstacle is ignored; no walkable source gives +inf everywhere
    walk = np.ones((3, 3), bool)
    walk[1, 1] = False
    assert np.isinf(I.distance_field(walk, [(1, 1)], dx, dy)).all()
