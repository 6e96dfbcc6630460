"""GPU parity of the pre-flood door flow (sec. 3, sec. 3.2, sec. 2.4): the door
kernel's entries against the oracle's (which slot, which door, where, which
leaving door: integer decisions and FP32 positions, bit for bit), one-step
windows of the coupled step with walkers leaving and entering, the flood's
trigger closing the doors, the bins with entrants in every binning path, and
graph replay and ensembles equal to eager solo runs."""
import ctypes as C

import numpy as np
import pytest

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import say, snapshot

pytestmark = pytest.mark.gpu
ST_EVAC, ST_EXITED, ST_SHOPPING, ST_OUTSIDE = 0, 1, 6, 7
AGENT_KEYS = ("x", "y", "vx", "vy", "state", "dest", "hr_class", "timer")


def site(walkers=1000, n=128, dx=332.0 / 128, per_step=10, door_seed=1908, seed=5232):
    """The paper's site (128 x 128 cells over 332 m, one emergency exit north,
    the breach south) with 7 doors and the 5-minute spin-up."""
    sc = I.shopping_centre(n=n, dx=dx, seed=seed, n_evac=walkers, n_exits=1, q_peak=20.0, duration=1800.0)
    return I.add_doors(sc, per_step=per_step, seed=door_seed)


def force_scale(sc, A, idx):
    """Sum of the magnitudes of the repulsions on each agent of idx (m/s^2):
    from the other agents inside within r_cut, A/m exp((2r - d)/B), and from
    the obstacle cells within r_cut, A/m exp((r - d)/B) at the nearest point.
    The FP32 force sum of the kernel is off by a few units of 2^-24 of this
    relative to FP64, whatever the cancellation in the sum itself."""
    from scipy.spatial import cKDTree
    p, d = sc.ped, sc.desc
    inside = np.flatnonzero(np.isin(A["state"], (ST_SHOPPING, ST_EVAC)))
    pts = np.stack([A["x"][inside], A["y"][inside]], 1).astype(np.float64)
    tree = cKDTree(pts)
    out = np.zeros(len(idx))
    R = int(np.ceil(p.r_cut / d.dx - 1e-9))
    for n, a in enumerate(idx):
        x, y = float(A["x"][a]), float(A["y"][a])
        for b in tree.query_ball_point([x, y], p.r_cut):
            r = np.hypot(x - pts[b, 0], y - pts[b, 1])
            if 0.0 < r < p.r_cut:
                out[n] += p.a_over_m * np.exp((2 * p.radius - r) / p.b_range)
        ci, cj = int(x // d.dx), int(y // d.dy)
        for wj in range(max(cj - R, 0), min(cj + R, d.ny - 1) + 1):
            for wi in range(max(ci - R, 0), min(ci + R, d.nx - 1) + 1):
                if sc.walk[wj, wi]:
                    continue
                px = min(max(x, wi * d.dx), (wi + 1) * d.dx)
                py = min(max(y, wj * d.dy), (wj + 1) * d.dy)
                r = np.hypot(x - px, y - py)
                if 0.0 < r < p.r_cut:
                    out[n] += p.a_over_m * np.exp((p.radius - r) / p.b_range)
    return out


def oracle_from(oracle, sim, sc):
    start, d0 = snapshot(sim, sc)
    ref = oracle.OracleSim(start)
    ref.S.t, ref.S.step = d0["t"], d0["step"]
    ref.S.doors_closed, ref.S.door_in, ref.S.door_out = d0["doors_closed"], d0["door_entries"], d0["door_leaves"]
    return ref, start


def test_entries_match_the_oracle_step_by_step(oracle):
    """The first 40 dry steps from all slots outside: after every step the
    state and destination of every slot equal the oracle's (the entries of a
    step depend only on the free slots, and nobody reaches a door this soon),
    the entrants' positions are the oracle's FP32 values bit for bit, and the
    entry counters agree.  The walkers' positions are reported, not held
    here: a crowd at a door sums repulsions of 10^3 m/s^2 that nearly cancel,
    so FP32 and FP64 walks part by millimetres within a few steps and by
    whole routes later (a cell edge taken on the other side); the one-step
    windows below hold them to a bound derived from that conditioning."""
    sc = site()
    sim = fps.Sim(sc)
    ref = oracle.OracleSim(sc)
    worst, early = 0.0, 0.0     # over 40 steps, over the first 3
    for k in range(40):
        before = ref.state.copy()
        sim.step(1)
        ref.coupled_step(sim.diag()["dt_last"])
        A = sim.agents()
        assert np.array_equal(A["state"], ref.state), k
        assert np.array_equal(A["dest"], ref.dest), k
        new = np.flatnonzero((before == ST_OUTSIDE) & (ref.state == ST_SHOPPING))
        assert np.array_equal(A["x"][new], ref.x[new].astype(np.float32)), k
        assert np.array_equal(A["y"][new], ref.y[new].astype(np.float32)), k
        inside = ref.state == ST_SHOPPING
        dk = max(float(np.abs(A["x"] - ref.x)[inside].max()), float(np.abs(A["y"] - ref.y)[inside].max()))
        worst = max(worst, dk)
        if k < 3:
            early = max(early, dk)
    d = sim.diag()
    say(f"40 steps: {d['door_entries']} entries (oracle {ref.S.door_in}), state counts {d['state_count']}, "
        f"walkers' positions within {early:.2e} m of the FP64 oracle over 3 steps, {worst:.2e} m over 40")
    assert d["door_entries"] == ref.S.door_in == 1000 and d["state_count"][ST_SHOPPING] == 1000


@pytest.mark.parametrize("warm", [0, 9, 150, 299, 300, 301])
def test_one_step_parity_with_doors(oracle, warm):
    """One coupled step from the GPU's state after `warm` steps (the spin-up
    fills at step 15, walkers leave from about step 100, the breach starts at
    step 300 and its first wet step closes the doors): entrants bit for bit,
    every other integer decision equal except arrivals that FP32 and FP64
    positions put on either side of a cell edge; positions within 1e-4 m plus
    4e-6 dt^2 times the sum of the repulsion magnitudes on the walker (the
    FP32 force terms carry ~1e-6 relative error each, from the exponential
    and the distance, which a crowd's nearly cancelling sum keeps in
    absolute terms; dt^2 takes a force error to a position error)."""
    sc = site()
    sim = fps.Sim(sc)
    sim.step(warm)
    ref, start = oracle_from(oracle, sim, sc)
    before = start.agents["state"].copy()
    sim.step(1)
    dt = sim.diag()["dt_last"]
    ref.coupled_step(dt)
    A = sim.agents()
    d = sim.diag()
    new_g = np.flatnonzero((before == ST_OUTSIDE) & (A["state"] == ST_SHOPPING))
    new_o = np.flatnonzero((before == ST_OUTSIDE) & (ref.state == ST_SHOPPING))
    st_mism = np.flatnonzero(A["state"] != ref.state)
    moved = np.isin(before, (ST_SHOPPING, ST_EVAC))
    mv = np.flatnonzero(moved)
    err = np.maximum(np.abs(A["x"] - ref.x), np.abs(A["y"] - ref.y))[mv]
    bound = 1e-4 + 4e-6 * dt * dt * force_scale(start, start.agents, mv)
    dpos = float(err.max(initial=0.0))
    worst_ratio = float((err / bound).max(initial=0.0))
    say(f"[warm {warm}] t {d['t']:.2f} dt {dt:.3g} entrants {len(new_g)} (oracle {len(new_o)}), "
        f"left {d['door_leaves']} (oracle {ref.S.door_out}), closed {d['doors_closed']} (oracle {ref.S.doors_closed}), "
        f"state mismatches {len(st_mism)}, max|dpos| {dpos:.2e}, largest error / bound {worst_ratio:.3f}")
    # a walker that reaches its door a hair earlier on one side frees a slot
    # that may enter at once, so an arrival decided differently can move one
    # entry; allow as many differences as the arrivals that differ
    arr_diff = int(np.sum((A["state"] == ST_OUTSIDE) != (ref.state == ST_OUTSIDE)))
    assert len(np.setxor1d(new_g, new_o)) <= 2 * arr_diff
    both = np.intersect1d(new_g, new_o)
    assert np.array_equal(A["x"][both], ref.x[both].astype(np.float32))
    assert np.array_equal(A["dest"][both], ref.dest[both])
    assert len(st_mism) <= max(1, 0.005 * len(A["x"]))
    assert d["doors_closed"] == ref.S.doors_closed
    same = moved & (A["state"] == ref.state)
    assert np.array_equal(A["dest"][same], ref.dest[same])
    assert np.all(err <= bound)
    cnt = sim.counts().cpu().numpy().reshape(-1)
    assert int(np.sum(cnt != ref.np_)) <= 2 * max(1, len(st_mism))


def test_first_wet_step_closes_the_doors_gpu():
    sc = site()
    sim = fps.Sim(sc)
    sim.step(290)
    d = sim.diag()
    while not d["any_wet"]:
        prev = d
        sim.step(1)
        d = sim.diag()
    e0 = d["door_entries"]
    say(f"first wet step ends at t = {d['t']:.2f}: closed {d['doors_closed']}, entries {e0}, "
        f"states {d['state_count']} (before: {prev['state_count']})")
    assert d["doors_closed"] == 1 and prev["doors_closed"] == 0
    assert d["state_count"][ST_SHOPPING] == 0
    assert d["state_count"][ST_EVAC] == prev["state_count"][ST_SHOPPING]
    assert int(sim.counts().sum()) == d["state_count"][ST_EVAC]
    sim.step(200)
    d2 = sim.diag()
    assert d2["door_entries"] == e0 and d2["state_count"][ST_SHOPPING] == 0
    assert d2["state_count"][ST_EVAC] + d2["state_count"][ST_EXITED] == d["state_count"][ST_EVAC]


@pytest.mark.parametrize("which", ["site", "wide", "big"])
def test_bins_with_entrants_bit_exact(oracle, which):
    """The bins after steps with entries against the oracle's stable counting
    sort, in each binning path: the one-block LDS binning (the site, 1,000
    slots), the global histogram with the end-of-step placement (600^2 cells
    of 0.25 m: 22,500 bins, 3,000 slots), and the placement kernels (9,000
    slots, more than the end-of-step block places)."""
    if which == "site":
        sc, checks = site(), (1, 5, 40, 200)
    elif which == "wide":
        sc, checks = site(walkers=3000, n=600, dx=0.25, per_step=40), (1, 5, 40)
    else:
        sc, checks = site(walkers=9000, n=600, dx=0.25, per_step=200), (1, 5, 40)
    sim = fps.Sim(sc)
    P = oracle.make_params(sc.desc, sc.ped)
    done = 0
    for k in checks:
        sim.step(k - done)
        done = k
        A = sim.agents()
        bs, perm = sim.bins()
        bs_ref, perm_ref = oracle.build_bins(P, A["x"], A["y"], A["state"])
        inside = int(np.isin(A["state"], (ST_SHOPPING, ST_EVAC)).sum())
        say(f"[{which}] step {k}: {inside} inside, {len(perm)} binned")
        assert len(perm) == inside
        assert np.array_equal(bs, bs_ref) and np.array_equal(perm, perm_ref)


def test_graph_replay_and_ensemble_equal_eager_solo_runs():
    """320 steps (spin-up, breach, trigger): a graph-replayed run equals the
    eager one bit for bit, and an ensemble of two door-flow scenarios (other
    door seeds) and one without doors equals the three solo runs."""
    scs = [site(door_seed=1), site(door_seed=2),
           I.shopping_centre(n=128, dx=332.0 / 128, seed=77, n_evac=800, n_exits=1, q_peak=20.0, duration=1800.0)]
    eager = fps.Sim(scs[0])
    eager.set_graph(0)
    graph = fps.Sim(scs[0])
    graph.set_graph(16)
    eager.step(320)
    graph.step(320)
    A, B = eager.agents(), graph.agents()
    assert all(np.array_equal(A[k], B[k]) for k in AGENT_KEYS)
    ens = fps.Ensemble(scs)
    ens.step(320)
    for k, sc in enumerate(scs):
        solo = fps.Sim(sc)
        solo.step(320)
        S, E = solo.agents(), ens[k].agents()
        for key in AGENT_KEYS:
            assert np.array_equal(S[key], E[key]), (k, key)
        for a, b in zip(solo.fields(), ens[k].fields()):
            assert np.array_equal(a, b), k
        ds, de = solo.diag(), ens[k].diag()
        assert (ds["door_entries"], ds["door_leaves"], ds["doors_closed"]) == \
               (de["door_entries"], de["door_leaves"], de["doors_closed"])
    say(f"ensemble members equal solo runs; member 0: {ens[0].diag()['door_entries']} entries")


def test_set_doors_validation():
    sc = site()
    sim = fps.Sim(sc)
    L, h = sim._lib, sim.h_
    P = C.POINTER(C.c_int32)

    def call(n, cells, dests, per_step=10):
        c = np.ascontiguousarray(cells, np.int32)
        d = np.ascontiguousarray(dests, np.int32)
        return L.fps_set_doors(h, n, c.ctypes.data_as(P), d.ctypes.data_as(P), per_step, 5)

    cells, dests = sc.doors["cells"], sc.doors["dests"]
    assert call(1, cells[:1], dests[:1]) == fps.FPS_E_INVALID
    assert call(17, np.resize(cells, 17), np.resize(dests, 17)) == fps.FPS_E_INVALID
    assert call(7, cells, dests, per_step=-1) == fps.FPS_E_INVALID
    bad = dests.copy()
    bad[3] = 0                                    # an exit is not a door
    assert call(7, cells, bad) == fps.FPS_E_INVALID
    bad[3] = sc.dist.shape[0]
    assert call(7, cells, bad) == fps.FPS_E_INVALID
    badc = cells.copy()
    badc[0] = 128 * 128
    assert call(7, badc, dests) == fps.FPS_E_INVALID
    assert call(7, cells, dests) == fps.FPS_OK
    assert L.fps_set_doors(h, 0, None, None, 0, 0) == fps.FPS_OK
    sim.step(5)
    assert sim.diag()["door_entries"] == 0        # the flow is off
