"""Pins of the oracle's pre-flood door flow (sec. 3, sec. 3.2, sec. 2.4;
readings D1-D6 in the oracle's header).

The paper fixes the counts: 7 entrance doors, entering and leaving by each
with probability 1/7, 10 per door, 1,000 walking before the flood, a 5-minute
spin-up with no inflow, and no entries once water is on the site.  These
checks hold the oracle to them and to what the readings imply: the random
numbers are the published SplitMix64 generator, door choices are uniform,
the leaving door is never the entry door and is uniform overall, each door
admits the first slots in slot order up to its rate, entrants stand in the
central half of their door cell, a slot freed by a leaving walker can enter
again in the same step, the population is conserved and capped by the slots,
the walkers add no roughness, and the first wet step closes the doors for good
and turns every walker into an evacuee."""
import json
import os

import numpy as np
import pytest

from paper_1908_05232_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ST_EVAC, ST_EXITED, ST_SHOPPING, ST_OUTSIDE = 0, 1, 6, 7


def hall(nx, ny, dx, doors, n_slots, per_step, seed=11, exit_cell=None, v_base=1.4):
    """An open walkable hall, one exit cell (the emergency exit) and the given
    door cells; every agent a free slot outside."""
    walk = np.ones((ny, nx), np.uint8)
    ex = exit_cell or (nx // 2, ny - 1)
    fields = [I.distance_field(walk, [ex], dx, dx)] + [I.distance_field(walk, [c], dx, dx) for c in doors]
    A = I.empty_agents(n_slots)
    A["state"][:] = ST_OUTSIDE
    A["v_base"][:] = v_base
    z = np.zeros((ny, nx))
    d = I.GridDesc(nx=nx, ny=ny, dx=dx, dy=dx)
    sc = I.Scenario(desc=d, h=z.copy(), qx=z.copy(), qy=z.copy(), z=z.copy(), dist=np.stack(fields),
                    n_exit=1, walk=walk, agents=A, name="hall")
    sc.doors = dict(cells=np.array([j * nx + i for (i, j) in doors], np.int32),
                    dests=np.arange(1, 1 + len(doors), dtype=np.int32), per_step=per_step, seed=seed)
    return sc


SEVEN = [(0, 8), (47, 8), (0, 24), (47, 24), (0, 40), (47, 40), (12, 0)]


def entrants(ref, before):
    return np.flatnonzero((before == ST_OUTSIDE) & (ref.state == ST_SHOPPING))


def door_of(sc, ref, a):
    d = sc.desc
    c = int(np.floor(np.float32(ref.y[a]) / np.float32(d.dy))) * d.nx + int(np.floor(np.float32(ref.x[a]) / np.float32(d.dx)))
    return int(np.flatnonzero(sc.doors["cells"] == c)[0])


def test_splitmix64_published_outputs(oracle):
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    got = [oracle.splitmix64(g["seed"], c) for c in range(len(g["outputs_hex"]))]
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_doors_uniform_and_leaving_door_never_the_entry(oracle):
    """Every one of 70,000 free slots enters in one step (rate above the slot
    count): entry doors are uniform over the 7 doors (chi-square, 6 degrees of
    freedom), the leaving door is never the entry door, is uniform over the
    other six given the entry door, and so uniform overall (probability 1/7
    each, sec. 3)."""
    import ctypes
    n = 70000
    sc = hall(48, 48, 1.0, SEVEN, n, per_step=n)
    ref = oracle.OracleSim(sc)
    before = ref.state.copy()
    ref.S.step = 12345
    oracle.lib().or_doors(ctypes.byref(ref.S))
    ent = entrants(ref, before)
    assert len(ent) == n and ref.S.door_in == n
    dests = sc.doors["dests"]
    din = np.array([door_of(sc, ref, a) for a in ent])
    dout = np.searchsorted(dests, ref.dest[ent])
    assert np.all(dests[dout] == ref.dest[ent])
    assert np.all(din != dout)

    def chi2(counts):
        e = counts.sum() / len(counts)
        return float(((counts - e) ** 2 / e).sum())

    assert chi2(np.bincount(din, minlength=7)) < 30.0            # p ~ 4e-5 at 6 dof
    assert chi2(np.bincount(dout, minlength=7)) < 30.0
    for k in range(7):
        cond = np.bincount(dout[din == k], minlength=7)
        assert cond[k] == 0
        assert chi2(np.delete(cond, k)) < 28.0                    # 5 dof


def test_each_door_admits_the_first_slots_in_slot_order(oracle):
    """With the rate at 10 per door, the entrants at each door are exactly the
    10 lowest slots among those that drew it (the draws seen in an unlimited
    run of the same step), and each entrant's position and leaving door are
    the unlimited run's."""
    import ctypes
    n = 1000
    full = oracle.OracleSim(hall(48, 48, 1.0, SEVEN, n, per_step=n))
    lim = oracle.OracleSim(hall(48, 48, 1.0, SEVEN, n, per_step=10))
    for r in (full, lim):
        r.S.step = 77
        oracle.lib().or_doors(ctypes.byref(r.S))
    sc = full.sc
    drew = np.array([door_of(sc, full, a) for a in range(n)])
    expect = np.sort(np.concatenate([np.flatnonzero(drew == k)[:10] for k in range(7)]))
    got = np.flatnonzero(lim.state == ST_SHOPPING)
    assert np.array_equal(got, expect) and lim.S.door_in == 70
    for nm in ("x", "y", "dest"):
        assert np.array_equal(getattr(lim, nm)[got], getattr(full, nm)[got])
    assert np.all(lim.state[np.setdiff1d(np.arange(n), got)] == ST_OUTSIDE)


def test_entrant_placement_and_record(oracle):
    import ctypes
    sc = hall(48, 48, 1.0, SEVEN, 500, per_step=50)
    ref = oracle.OracleSim(sc)
    ref.vx[:] = 3.0
    ref.timer[:] = 9.0
    ref.cls[:] = 4
    oracle.lib().or_doors(ctypes.byref(ref.S))
    ent = np.flatnonzero(ref.state == ST_SHOPPING)
    assert len(ent) == 350
    for a in ent:
        k = door_of(sc, ref, a)
        i, j = sc.doors["cells"][k] % 48, sc.doors["cells"][k] // 48
        fx, fy = ref.x[a] - i, ref.y[a] - j                      # dx = 1 m
        assert 0.25 <= fx < 0.75 and 0.25 <= fy < 0.75
        assert ref.x[a] == float(np.float32(ref.x[a]))           # FP32 positions (D6)
    assert np.all(ref.vx[ent] == 0.0) and np.all(ref.vy[ent] == 0.0) and np.all(ref.timer[ent] == 0.0)
    assert np.all(ref.cls[ent] == 0)


def test_a_slot_freed_by_leaving_enters_again_the_same_step(oracle):
    """One slot, two doors 7 m apart in a 1 m-wide corridor: the walker enters
    by one door and walks to the other at 1.4 m/s; in the step it arrives it
    goes back outside and, the only slot drawing a door, enters again at once
    (D2, D3)."""
    sc = hall(8, 1, 1.0, [(0, 0), (7, 0)], 1, per_step=1, exit_cell=(4, 0))
    ref = oracle.OracleSim(sc)
    seen_leave = False
    for k in range(12):
        ref.coupled_step(1.0)
        assert ref.state[0] == ST_SHOPPING
        assert ref.S.door_in - ref.S.door_out == 1
        seen_leave = seen_leave or ref.S.door_out > 0
    assert seen_leave and ref.S.door_in >= 2


@pytest.fixture(scope="module")
def paper_site_run():
    """The paper's site: 128 x 128 cells over 332 m, one emergency exit on the
    north wall, 7 doors, 1,000 slots, 10 per door, the 5-minute spin-up before
    the breach hydrograph; the oracle run to 2 minutes after the flood starts."""
    from oracle import oracle as O
    g = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    sc = I.shopping_centre(n=128, dx=332.0 / 128, seed=5232, n_evac=g["walkers"], n_exits=1,
                           q_peak=20.0, duration=1800.0)
    sc = I.add_doors(sc, n_doors=g["n_doors"], per_step=g["per_door"], spin_up=g["spin_up_s"])
    ref = O.OracleSim(sc)
    rec = []
    while ref.t < 120.0:
        before = ref.state.copy()
        ref.coupled_step(0.0)
        st = ref.state
        rec.append(dict(t=ref.t, wet=ref.S.any_wet, closed=ref.S.doors_closed, door_in=ref.S.door_in,
                        door_out=ref.S.door_out, inside=int(np.isin(st, (ST_EVAC, ST_SHOPPING)).sum()),
                        shopping=int((st == ST_SHOPPING).sum()), evac=int((st == ST_EVAC).sum()),
                        exited=int((st == ST_EXITED).sum()),
                        entered=int(((before == ST_OUTSIDE) & (st == ST_SHOPPING)).sum()),
                        np_sum=int(ref.np_.sum())))
    return sc, ref, rec, g


def test_spin_up_keeps_the_population(paper_site_run):
    sc, ref, rec, g = paper_site_run
    pre = [r for r in rec if not r["wet"]]
    assert abs(pre[-1]["t"] - 0.0) < 1e-9 and len(pre) == 300     # 300 dry 1 s steps up to t = 0
    for r in rec:       # every slot that entered is inside, left by a door or left by the exit
        assert r["inside"] + r["exited"] == r["door_in"] - r["door_out"]
        assert r["inside"] <= g["walkers"]
    for r in pre:
        assert r["inside"] == r["door_in"] - r["door_out"]
        assert r["entered"] <= g["n_doors"] * g["per_door"]
        assert r["np_sum"] == 0                                    # walkers add no roughness
    full_at = next(k for k, r in enumerate(pre) if r["inside"] == g["walkers"])
    assert full_at == int(np.ceil(g["walkers"] / (g["n_doors"] * g["per_door"]))) - 1
    assert min(r["inside"] for r in pre[full_at:]) >= g["walkers"] - g["n_doors"] * g["per_door"]
    assert pre[-1]["door_out"] > 0                                 # people did leave and were replaced


def test_first_wet_step_closes_the_doors(paper_site_run):
    sc, ref, rec, g = paper_site_run
    k0 = next(k for k, r in enumerate(rec) if r["wet"])
    assert rec[k0]["closed"] == 1 and all(r["closed"] == 0 for r in rec[:k0])
    assert rec[k0]["entered"] == 0
    assert all(r["door_in"] == rec[k0]["door_in"] for r in rec[k0:])
    assert all(r["shopping"] == 0 for r in rec[k0:])
    assert rec[k0]["evac"] == rec[k0 - 1]["inside"]
    for a, b in zip(rec[k0:], rec[k0 + 1:]):
        assert b["inside"] <= a["inside"]
    # from the trigger on every evacuee inside counts toward the roughness
    assert all(r["np_sum"] == r["evac"] for r in rec[k0:])


def test_walkers_spread_over_the_site(paper_site_run):
    """At t = 0 the walkers stand over much of the concourse, not at the doors:
    most are more than 20 m from every door, and they occupy hundreds of cells."""
    sc, ref, rec, g = paper_site_run
    # the state at the end of the fixture is after the trigger; rerun the
    # spin-up alone for the positions at t = 0
    from oracle import oracle as O
    ref0 = O.OracleSim(sc)
    while ref0.t < -1e-9:
        ref0.coupled_step(0.0)
    d = sc.desc
    inside = np.flatnonzero(ref0.state == ST_SHOPPING)
    cells = sc.doors["cells"]
    dxy = np.stack([((cells % d.nx) + 0.5) * d.dx, ((cells // d.nx) + 0.5) * d.dy], 1)
    far = np.min(np.hypot(ref0.x[inside, None] - dxy[None, :, 0], ref0.y[inside, None] - dxy[None, :, 1]), 1)
    occupied = len(np.unique((np.floor(ref0.y[inside] / d.dy) * d.nx + np.floor(ref0.x[inside] / d.dx))))
    assert len(inside) == g["walkers"]
    assert np.median(far) > 20.0 and occupied > 300
