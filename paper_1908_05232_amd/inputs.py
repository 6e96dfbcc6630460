"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

This module builds scenario *inputs* only: grids, topography, initial water,
hydrograph tables, navigation maps (distance fields over walkable cells) and
initial agent records.  It contains none of the method's arithmetic (no flux,
no hazard rate, no pedestrian rule), so feeding the same scenario to the GPU
library and to the CPU oracle compares two independent implementations.

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` here, on the
host; nothing random happens inside a simulation step.

The paper's case study (sec. 3) is a 332 m x 332 m shopping centre known only
from a figure, with stores on the east and west sides, corridors to an open
area, a 100 m breach on the south side and an exit on the north side.  The
generators below stand in for it with synthetic layouts of the same kind.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

WALL, TRANSMISSIVE = 0, 1
SIDE_W, SIDE_E, SIDE_S, SIDE_N = 0, 1, 2, 3
ROLE_EVACUEE, ROLE_RESPONDER = 0, 1
ST_EVAC, ST_EXITED, ST_SHOPPING, ST_OUTSIDE = 0, 1, 6, 7


@dataclasses.dataclass
class GridDesc:
    """Grid and flood constants (defaults: g, CFL 0.5, dry threshold, 1 s cap)."""
    nx: int
    ny: int
    dx: float
    dy: float
    g: float = 9.81
    cfl: float = 0.5
    h_dry: float = 1e-5
    dt_max: float = 1.0          # the 1.0 s pedestrian step used while dry (sec. 3)
    bc: tuple = (WALL, WALL, WALL, WALL)   # W, E, S, N
    inflow_side: int = -1
    inflow_c0: int = 0
    inflow_c1: int = 0
    n_base: float = 0.01         # clear cement (sec. 2.4)
    np_cap: int = 20             # at most 20 evacuees counted per cell (sec. 2.4)
    flux: int = 0                # face flux: 0 = HLLC, 1 = HLL for all three components
    order: int = 1               # 1: the paper's first-order scheme; 2: the second-order (MUSCL) variant


@dataclasses.dataclass
class PedParams:
    """Pedestrian constants.  Speeds and thresholds are Table 1; the social-force
    constants are those of Helbing, Farkas & Vicsek (2000) (A = 2000 N over an
    80 kg body, B = 0.08 m, tau = 0.5 s, body radius 0.25 m); r_cut, r_arrive and
    the 30 s waits (sec. 2.4) close the model."""
    tau: float = 0.5
    a_over_m: float = 25.0
    b_range: float = 0.08
    radius: float = 0.25
    r_cut: float = 1.0
    r_arrive: float = 1.0
    v_class: tuple = (0.0, 1.8, 0.9, 0.45, 0.0)
    hr_t: tuple = (0.75, 1.5, 2.5)
    pick_s: float = 30.0
    drop_s: float = 30.0
    # stability of a person standing in flowing water (off: the paper's Table 1 alone)
    stability: int = 0
    c_drag: float = 1.1           # drag coefficient of an upright cylinder
    mu_f: float = 0.45            # friction of feet on a wet floor
    rho_w: float = 1000.0         # water density (kg/m^3)
    rho_body: float = 1000.0      # body density (kg/m^3)
    body_h0: float = 1.71         # body of people without one of their own: height (m)
    body_m0: float = 70.0         # ... and mass (kg)
    # walking speed capped by the drag of wading (off: the paper's Table 1 alone)
    wading: int = 0
    wade_k: float = 0.1           # sustained push of the feet over the weight less buoyancy


@dataclasses.dataclass
class Scenario:
    desc: GridDesc
    h: np.ndarray                     # [ny, nx] float, metres
    qx: np.ndarray                    # [ny, nx] unit discharge, m^2/s
    qy: np.ndarray
    z: np.ndarray                     # [ny, nx] bed elevation, metres
    ped: PedParams = dataclasses.field(default_factory=PedParams)
    t0: float = 0.0
    hydro_t: Optional[np.ndarray] = None   # hydrograph breakpoints, s
    hydro_q: Optional[np.ndarray] = None   # unit discharge at the breakpoints, m^2/s
    dist: Optional[np.ndarray] = None      # [n_dest, ny, nx] float32 navigation distances
    n_exit: int = 0                         # destinations [0, n_exit) are exits
    walk: Optional[np.ndarray] = None      # [ny, nx] uint8, 1 = walkable
    agents: Optional[dict] = None
    barrier: Optional[dict] = None
    doors: Optional[dict] = None           # pre-flood door flow: cells, dests, per_step, seed
    name: str = ""


def rng_of(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# navigation map: 8-connected shortest distances over walkable cells
# ---------------------------------------------------------------------------
def distance_field(walk: np.ndarray, sources, dx: float, dy: float) -> np.ndarray:
    """Shortest walking distance (m) from every walkable cell to the nearest
    source cell, 8-connected (no corner cutting past obstacles).  Unreachable or
    non-walkable cells get +inf.  ``sources`` is a list of (i, j)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra

    ny, nx = walk.shape
    w = walk.astype(bool)
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols, wts = [], [], []

    def link(di, dj, cost):
        # cells (i, j) -> (i+di, j+dj), both walkable
        i0, i1 = max(0, -di), nx - max(0, di)
        j0, j1 = max(0, -dj), ny - max(0, dj)
        a = w[j0:j1, i0:i1] & w[j0 + dj:j1 + dj, i0 + di:i1 + di]
        if di != 0 and dj != 0:
            a = a & w[j0:j1, i0 + di:i1 + di] & w[j0 + dj:j1 + dj, i0:i1]
        src = idx[j0:j1, i0:i1][a]
        dst = idx[j0 + dj:j1 + dj, i0 + di:i1 + di][a]
        rows.append(src)
        cols.append(dst)
        wts.append(np.full(src.shape, cost))

    diag = math.hypot(dx, dy)
    for di, dj, cst in ((1, 0, dx), (-1, 0, dx), (0, 1, dy), (0, -1, dy),
                        (1, 1, diag), (-1, 1, diag), (1, -1, diag), (-1, -1, diag)):
        link(di, dj, cst)
    G = sp.csr_matrix((np.concatenate(wts), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nx * ny, nx * ny))
    src = [j * nx + i for (i, j) in sources if w[j, i]]
    if not src:
        return np.full((ny, nx), np.inf, dtype=np.float32)
    d = dijkstra(G, directed=True, indices=src, min_only=True)
    d = d.reshape(ny, nx)
    d[~w] = np.inf
    return d.astype(np.float32)


def triangular_hydrograph(q_peak: float, duration: float, t_start: float = 0.0):
    """Triangular inflow (sec. 3.1): 0 -> q_peak at mid-duration -> 0."""
    t = np.array([t_start, t_start + 0.5 * duration, t_start + duration], dtype=np.float64)
    q = np.array([0.0, q_peak, 0.0], dtype=np.float64)
    return t, q


def empty_agents(n: int) -> dict:
    return dict(
        x=np.zeros(n, np.float32), y=np.zeros(n, np.float32),
        vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
        v_base=np.full(n, 1.4, np.float32),
        role=np.zeros(n, np.uint8), state=np.zeros(n, np.uint8),
        hr_class=np.zeros(n, np.uint8), dest=np.full(n, -1, np.int32),
        timer=np.zeros(n, np.float32))


def add_bodies(sc: Scenario, seed: int, stability: int = 1) -> Scenario:
    """Variable bodies for every agent: heights N(1.71, 0.09) m clipped to
    [1.45, 1.95] m and body-mass indices N(25, 3.5) clipped to [17, 35] kg/m^2
    (mass = index x height^2), a seeded adult population; switches the
    stability rule on."""
    rng = rng_of(seed + 31337)
    n = len(sc.agents["x"])
    height = np.clip(rng.normal(1.71, 0.09, n), 1.45, 1.95)
    bmi = np.clip(rng.normal(25.0, 3.5, n), 17.0, 35.0)
    sc.agents["height"] = height.astype(np.float32)
    sc.agents["mass"] = (bmi * height ** 2).astype(np.float32)
    sc.ped = dataclasses.replace(sc.ped, stability=stability)
    return sc


def place_uniform(rng, walk: np.ndarray, n: int, dx: float, dy: float):
    """n positions uniform over the walkable area (a random walkable cell, then a
    uniform offset inside it, kept away from the cell edges by 1e-3 of a cell)."""
    ny, nx = walk.shape
    free = np.flatnonzero(walk.reshape(-1))
    cells = free[rng.integers(0, len(free), size=n)]
    ci, cj = cells % nx, cells // nx
    ox = rng.uniform(1e-3, 1 - 1e-3, size=n)
    oy = rng.uniform(1e-3, 1 - 1e-3, size=n)
    x = ((ci + ox) * dx).astype(np.float32)
    y = ((cj + oy) * dy).astype(np.float32)
    return x, y


def concat_agents(*groups) -> dict:
    return {k: np.concatenate([g[k] for g in groups]) for k in groups[0]}


# ---------------------------------------------------------------------------
# scenarios
# ---------------------------------------------------------------------------
def dam_break_1d(nx: int, length: float, h_left: float, h_right: float, x0: float = None,
                 n_manning: float = 0.0, ny: int = 1) -> Scenario:
    """1D dam break along x (ny rows, walls all round, flat bed, no friction by default)."""
    dx = length / nx
    x0 = 0.5 * length if x0 is None else x0
    xc = (np.arange(nx) + 0.5) * dx
    h = np.where(xc < x0, h_left, h_right)[None, :].repeat(ny, 0)
    z = np.zeros((ny, nx))
    desc = GridDesc(nx=nx, ny=ny, dx=dx, dy=dx, n_base=n_manning)
    return Scenario(desc=desc, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=z,
                    name=f"dambreak1d_{nx}")


def cfg1_dam_break(seed: int = 1908, n_ped: int = 100, nx: int = 64, dx: float = 0.5,
                   n_manning: float = 0.02) -> Scenario:
    """64x64 cells of 0.5 m, flat, Manning 0.02, closed walls, h = 1.0 m for
    x < 16 m and 0.1 m elsewhere; 100 evacuees uniform at random, base speed
    U(1.0, 1.5) m/s, one exit cell at the centre of the east wall."""
    rng = rng_of(seed)
    ny = nx
    L = nx * dx
    xc = (np.arange(nx) + 0.5) * dx
    h = np.where(xc < 0.5 * L, 1.0, 0.1)[None, :].repeat(ny, 0)
    z = np.zeros((ny, nx))
    desc = GridDesc(nx=nx, ny=ny, dx=dx, dy=dx, n_base=n_manning)
    walk = np.ones((ny, nx), np.uint8)
    exit_cell = (nx - 1, ny // 2)
    dist = distance_field(walk, [exit_cell], dx, dx)[None]
    A = empty_agents(n_ped)
    A["x"], A["y"] = place_uniform(rng, walk, n_ped, dx, dx)
    A["v_base"] = rng.uniform(1.0, 1.5, size=n_ped).astype(np.float32)
    return Scenario(desc=desc, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=z,
                    dist=dist, n_exit=1, walk=walk, agents=A, name="cfg1_dam_break")


def lake_at_rest(nx: int, ny: int, dx: float, seed: int, eta: float = 1.0) -> Scenario:
    """Still water over a random bed with emerging blocks.  Bed heights are
    multiples of 1/64 m and eta = 1 m so that h = eta - z is exact in FP32."""
    rng = rng_of(seed)
    z = rng.integers(0, 48, size=(ny, nx)) / 64.0          # 0 .. 0.73 m, below eta
    nblk = max(1, (nx * ny) // 200)
    for _ in range(nblk):                                   # +3 m blocks: dry islands
        i, j = rng.integers(0, nx), rng.integers(0, ny)
        w, hgt = rng.integers(1, 4), rng.integers(1, 4)
        z[j:j + hgt, i:i + w] = 3.0
    # a few cells just at / just above the surface
    k = rng.integers(0, nx * ny, size=max(1, nx * ny // 100))
    z.reshape(-1)[k] = rng.choice([1.0, 1.0 + 1 / 64.0, 1.0 - 1 / 64.0], size=len(k))
    h = np.maximum(eta - z, 0.0)
    desc = GridDesc(nx=nx, ny=ny, dx=dx, dy=dx, n_base=0.02)
    return Scenario(desc=desc, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=z,
                    name="lake_at_rest")


def shopping_centre_layout(n: int, dx: float, seed: int, min_block: float = 12.0,
                           corridor: float = 1.5, concourse: float = 0.4,
                           block_height: float = 3.0):
    """Random rectangle tiling of a square site: guillotine cuts at U(0.3, 0.7)
    of the longer side until pieces are under ``min_block`` metres; each piece
    shrunk by a ``corridor`` half-width and raised by ``block_height`` as a
    shop/wall block; a central north-south concourse of ``concourse`` of the
    width kept clear.  Returns (z, walk)."""
    rng = rng_of(seed)
    L = n * dx
    z = np.zeros((n, n))
    stack = [(0.0, 0.0, L, L)]
    leaves = []
    while stack:
        x0, y0, x1, y1 = stack.pop()
        w, hh = x1 - x0, y1 - y0
        if max(w, hh) < min_block:
            leaves.append((x0, y0, x1, y1))
            continue
        f = rng.uniform(0.3, 0.7)
        if w >= hh:
            xm = x0 + f * w
            stack += [(x0, y0, xm, y1), (xm, y0, x1, y1)]
        else:
            ym = y0 + f * hh
            stack += [(x0, y0, x1, ym), (x0, ym, x1, y1)]
    xc = (np.arange(n) + 0.5) * dx
    cx0, cx1 = 0.5 * L * (1 - concourse), 0.5 * L * (1 + concourse)
    for (x0, y0, x1, y1) in leaves:
        bx0, by0, bx1, by1 = x0 + corridor, y0 + corridor, x1 - corridor, y1 - corridor
        if bx1 <= bx0 or by1 <= by0:
            continue
        mi = (xc > bx0) & (xc < bx1) & ~((xc > cx0) & (xc < cx1))
        mj = (xc > by0) & (xc < by1)
        z[np.ix_(mj, mi)] = block_height
    walk = (z == 0.0).astype(np.uint8)
    return z, walk


def _connected(walk, a_cells, b_cells):
    from scipy.ndimage import label
    lab, _ = label(walk.astype(bool), structure=np.ones((3, 3)))
    la = {lab[j, i] for (i, j) in a_cells if walk[j, i]}
    lb = {lab[j, i] for (i, j) in b_cells if walk[j, i]}
    la.discard(0)
    lb.discard(0)
    return bool(la & lb)


def shopping_centre(n: int = 512, dx: float = 0.25, seed: int = 5232, n_evac: int = 2000,
                    q_peak: float = 2.0, duration: float = 600.0, t_flood: float = 0.0,
                    exit_width: float = 2.0, v_base: float = 1.4, n_exits: int = 2,
                    n_manning: float = 0.01, nearest_exit_field: bool = False) -> Scenario:
    """Synthetic shopping-centre evacuation: random building tiling (+3 m
    blocks), south breach over the central 30% of the south edge carrying a
    triangular hydrograph, transmissive ("slip") north side, walls east and
    west, ``n_exits`` exits of ``exit_width`` on the north wall at x = L/3, 2L/3,
    evacuees uniform over the free space at the paper's 1.4 m/s.  With
    ``nearest_exit_field`` the navigation map holds one distance field to the
    nearest cell of any exit instead of one per exit (the same route for every
    evacuee, who heads for the nearest exit either way; one Dijkstra run
    instead of n_exits on large grids)."""
    L = n * dx
    s = seed
    while True:
        z, walk = shopping_centre_layout(n, dx, s)
        c0, c1 = int(round(0.35 * n)), int(round(0.65 * n))
        inflow_cells = [(i, 0) for i in range(c0, c1)]
        half = max(1, int(round(0.5 * exit_width / dx)))
        exits = []
        for k in range(n_exits):
            ic = int(round((k + 1) * n / (n_exits + 1)))
            exits.append([(i, n - 1) for i in range(max(0, ic - half), min(n, ic + half))])
        if all(_connected(walk, inflow_cells, e) for e in exits):
            break
        s += 1
    rng = rng_of(seed)
    if nearest_exit_field:
        dist = distance_field(walk, [c for e in exits for c in e], dx, dx)[None]
        n_exits = 1
    else:
        dist = np.stack([distance_field(walk, e, dx, dx) for e in exits])
    desc = GridDesc(nx=n, ny=n, dx=dx, dy=dx, bc=(WALL, WALL, WALL, TRANSMISSIVE),
                    inflow_side=SIDE_S, inflow_c0=c0, inflow_c1=c1, n_base=n_manning)
    ht, hq = triangular_hydrograph(q_peak, duration, t_flood)
    A = empty_agents(n_evac)
    A["x"], A["y"] = place_uniform(rng, walk, n_evac, dx, dx)
    A["v_base"][:] = v_base
    h = np.zeros((n, n))
    return Scenario(desc=desc, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=z,
                    hydro_t=ht, hydro_q=hq, dist=dist, n_exit=n_exits, walk=walk, agents=A,
                    name=f"shopping_centre_{n}")


def add_barrier(sc: Scenario, seed: int, n_resp: int, height: float, t_bag: float = 0.2,
                bag_area: float = 0.4 * 0.3, y_frac: float = 0.7) -> Scenario:
    """Pre-flood intervention (sec. 2.4, sec. 3.3): a sandbag barrier on the
    row at ``y_frac`` of the site, running from the first free cell west of the
    site centre-line to the east until a wall or obstacle; a sandbag storage cell
    at random in the free space; ``n_resp`` responders uniform in the free space.
    Layers: ceil(height / t_bag), the last one taking the remainder."""
    rng = rng_of(seed + 7919)
    d = sc.desc
    walk = sc.walk
    jb = int(y_frac * d.ny)
    ic = d.nx // 2
    while ic > 0 and not walk[jb, ic]:
        ic -= 1
    i0 = ic
    while i0 - 1 >= 0 and walk[jb, i0 - 1]:
        i0 -= 1
    i1 = i0
    while i1 + 1 < d.nx and walk[jb, i1 + 1]:
        i1 += 1
    cells = np.array([jb * d.nx + i for i in range(i0, i1 + 1)], dtype=np.int32)
    free = np.flatnonzero(walk.reshape(-1))
    free = free[np.abs(free // d.nx - jb) > 4]
    st = int(free[rng.integers(0, len(free))])
    storage = (st % d.nx, st // d.nx)
    d_store = distance_field(walk, [storage], d.dx, d.dy)
    d_bar = distance_field(walk, [(i0, jb)], d.dx, d.dy)
    base = sc.dist.shape[0]
    sc.dist = np.concatenate([sc.dist, d_store[None], d_bar[None]])
    n_layers = max(1, int(math.ceil(height / t_bag - 1e-9)))
    t_last = height - t_bag * (n_layers - 1)
    bags_per = int(math.ceil(d.dx * d.dy / bag_area - 1e-12))
    sc.barrier = dict(cells=cells, storage_dest=base, barrier_dest=base + 1,
                      n_layers=n_layers, bags_per=bags_per, t_bag=t_bag, t_last=t_last)
    R = empty_agents(n_resp)
    R["x"], R["y"] = place_uniform(rng, walk, n_resp, d.dx, d.dy)
    R["role"][:] = ROLE_RESPONDER
    sc.agents = concat_agents(sc.agents, R) if sc.agents is not None else R
    return sc


def door_cells(walk: np.ndarray, n_doors: int = 7):
    """Entrance doors on the site's outer walls (stores east and west, doors
    at the ends of the corridors, sec. 3): alternately on the west and east
    walls at even spacing, and one on the south wall at a sixth of the width
    (clear of the breach) when the count is odd; the north wall holds the
    emergency exit.  Each door is the walkable wall cell nearest to its
    target point.  Returns a list of (i, j)."""
    ny, nx = walk.shape
    n_side = n_doors // 2
    targets = []
    for m in range(n_side):
        jt = int(round((m + 1) * ny / (n_side + 1)))
        targets += [("W", jt), ("E", jt)]
    if n_doors % 2:
        targets.append(("S", int(round(nx / 6))))
    out = []
    for side, c in targets[:n_doors]:
        line = ([(0, j) for j in range(ny)] if side == "W" else
                [(nx - 1, j) for j in range(ny)] if side == "E" else [(i, 0) for i in range(nx)])
        free = [p for p in line if walk[p[1], p[0]] and p not in out]
        if not free:
            raise ValueError(f"no walkable cell on the {side} wall for a door")
        out.append(min(free, key=lambda p: abs((p[1] if side in "WE" else p[0]) - c)))
    return out


def add_doors(sc: Scenario, n_doors: int = 7, per_step: int = 10, seed: int = 1908,
              spin_up: float = 300.0) -> Scenario:
    """The pre-flood pedestrian flow of sec. 3.2: ``n_doors`` entrance doors
    (``door_cells``) with a distance field each, appended to the navigation
    map; every agent becomes a free slot outside the building (state OUTSIDE,
    evacuee role), so the agent count is the most people inside at once (1,000
    in the paper); ``per_step`` entries per door and step; the run starts
    ``spin_up`` seconds before the flood (t0 = -300 s: the paper's -5 min, the
    hydrograph still starting at its own t_flood)."""
    d = sc.desc
    cells = door_cells(sc.walk, n_doors)
    base = sc.dist.shape[0]
    fields = [distance_field(sc.walk, [c], d.dx, d.dy) for c in cells]
    sc.dist = np.concatenate([sc.dist, np.stack(fields).astype(sc.dist.dtype)])
    sc.doors = dict(cells=np.array([j * d.nx + i for (i, j) in cells], np.int32),
                    dests=np.arange(base, base + n_doors, dtype=np.int32), per_step=per_step, seed=seed)
    A = sc.agents
    A["state"][:] = ST_OUTSIDE
    A["role"][:] = ROLE_EVACUEE
    A["dest"][:] = -1
    A["vx"][:] = 0.0
    A["vy"][:] = 0.0
    sc.t0 = -float(spin_up)
    return sc


def wet_probe(n: int = 8192, dx: float = 0.25, seed: int = 8192) -> Scenario:
    """A large, fully wet grid for bandwidth measurements: a 1 m / 0.5 m dam
    break along x over a gently varying bed, walls all round, no agents.
    Every cell does the full flux, friction and time-step work."""
    rng = rng_of(seed)
    x = (np.arange(n, dtype=np.float32) + 0.5) * dx
    z = (0.05 * np.sin(x / 7.0)).astype(np.float32)
    z = np.broadcast_to(z[None, :], (n, n)) + (0.02 * rng.random((n, 1))).astype(np.float32)
    h = np.where(x[None, :] < 0.5 * n * dx, 1.0, 0.5).astype(np.float32) - z
    desc = GridDesc(nx=n, ny=n, dx=dx, dy=dx, n_base=0.02)
    zeros = np.zeros((n, n), np.float32)
    return Scenario(desc=desc, h=h.astype(np.float32), qx=zeros, qy=zeros.copy(),
                    z=np.ascontiguousarray(z, np.float32), name=f"wet_probe_{n}")


def _sweep_member(args):
    seed, k = args
    rng = rng_of(seed * 1000 + k)
    n = int(rng.choice([256, 512, 1024]))
    height = float(rng.choice([0.2, 0.4, 0.6, 0.8]))
    n_resp = int(rng.integers(10, 201))
    n_evac = int(rng.integers(500, 5001))
    q_peak = float(rng.uniform(1.0, 3.0))
    sc = shopping_centre(n=n, dx=0.25, seed=seed * 1000 + k, n_evac=n_evac, q_peak=q_peak)
    sc = add_barrier(sc, seed=seed * 1000 + k, n_resp=n_resp, height=height)
    sc.name = f"sweep_{k}_{n}_bar{height}_resp{n_resp}_evac{n_evac}"
    return sc


def intervention_sweep(S: int = 64, seed: int = 3303, workers: int = 8):
    """Pre-flood intervention sweep (sec. 3.3 as a batch): S shopping centres
    with grids drawn from {256^2, 512^2, 1024^2} at 0.25 m, sandbag barrier
    height from {0.2, 0.4, 0.6, 0.8} m, 10-200 responders, 500-5,000
    evacuees and hydrograph peak U(1, 3) m^2/s, each member from its own seed.
    The host set-up (layouts and navigation fields) runs in worker processes."""
    jobs = [(seed, k) for k in range(S)]
    if workers <= 1:
        return [_sweep_member(j) for j in jobs]
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_sweep_member, jobs))


def _large_member(args):
    seed, k, n, n_evac = args
    rng = rng_of(seed * 1000 + k)
    height = float(rng.uniform(0.2, 1.0))
    q_peak = float(rng.uniform(1.0, 3.0))
    t_flood = -float(rng.uniform(0.0, 300.0))
    sheet = float(rng.uniform(0.02, 0.1))
    sc = shopping_centre(n=n, dx=0.25, seed=seed * 1000 + k, n_evac=n_evac, q_peak=q_peak,
                         t_flood=t_flood, nearest_exit_field=True)
    walk = sc.walk.astype(bool)
    # the water of the earlier part of the flood: a shallow sheet over the free
    # area and 1-3 deeper ponds, so that every free cell is wet and moving
    h = np.where(walk, sheet, 0.0)
    for _ in range(int(rng.integers(1, 4))):
        w, hh = rng.integers(n // 16, n // 4, size=2)
        i0, j0 = rng.integers(0, n - w), rng.integers(n // 8, n - hh)
        h[j0:j0 + hh, i0:i0 + w] = np.where(walk[j0:j0 + hh, i0:i0 + w], rng.uniform(0.2, 1.0), 0.0)
    sc.h = h
    # a completed sandbag line of the drawn height across the free cells of the
    # row at 0.7 of the site (raised bed; the people still cross it)
    jb = int(0.7 * n)
    sc.z[jb, :] += height * walk[jb, :]
    sc.name = f"large_{k}_{n}_bar{height:.2f}_sheet{sheet:.3f}"
    return sc


def large_sweep(S: int = 32, n: int = 2048, n_evac: int = 50000, seed: int = 5, workers: int = 8):
    """Large sweep: S shopping centres of n x n cells of 0.25 m (random
    building tiling as above), each with a completed sandbag line of height
    U(0.2, 1.0) m across the row at 0.7 of the site, ``n_evac`` evacuees
    uniform over the free space heading for the nearest of two north exits,
    the triangular hydrograph (peak U(1, 3) m^2/s over 600 s) already
    U(0, 300) s under way, and the site already wet: a sheet of U(0.02, 0.1) m
    over the free area plus 1-3 ponds of U(0.2, 1.0) m.  Each member from its
    own seed; the host set-up runs in worker processes."""
    jobs = [(seed, k, n, n_evac) for k in range(S)]
    if workers <= 1:
        return [_large_member(j) for j in jobs]
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_large_member, jobs))
