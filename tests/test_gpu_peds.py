"""GPU parity of the pedestrian step, binning, counts and barrier write-back."""
import copy
import json
import os

import numpy as np
import pytest

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import say, snapshot

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def recount(sc, A):
    d = sc.desc
    ci = np.clip(np.floor(A["x"].astype(np.float32) / np.float32(d.dx)).astype(np.int64), 0, d.nx - 1)
    cj = np.clip(np.floor(A["y"].astype(np.float32) / np.float32(d.dy)).astype(np.int64), 0, d.ny - 1)
    act = (A["role"] == I.ROLE_EVACUEE) & (A["state"] == 0)
    cnt = np.zeros(d.nx * d.ny, np.int32)
    np.add.at(cnt, (cj * d.nx + ci)[act], 1)
    return cnt.reshape(d.ny, d.nx)


@pytest.mark.parametrize("which", ["cfg1", "one", "centre", "wide", "big", "chunks", "chunks_big"])
def test_bins_and_counts_bit_exact(oracle, which):
    """The bins after the step against the oracle's stable counting sort:
    the one-block LDS binning (cfg1, one agent, centre), the global histogram
    scanned by the end-of-step block which also places the agents (wide:
    22,500 bins, more than the LDS binning takes, and 3,000 agents), the
    global scan with the placement kernels (big: 9,000 agents, more than the
    end-of-step block places itself), and the multi-block scan (1024^2 cells:
    65,536 bins in 16 chunks, with 3,000 and 12,000 agents)."""
    if which == "cfg1":
        sc = I.cfg1_dam_break(n_ped=400)
        checkpoints = (0, 5, 60)
    elif which == "one":
        sc = I.cfg1_dam_break(n_ped=1)
        checkpoints = (0, 5, 60)
    elif which == "centre":
        sc = I.shopping_centre(n=256, dx=0.25, seed=9, n_evac=3000)
        checkpoints = (0, 20, 200)
    elif which == "wide":
        sc = I.shopping_centre(n=600, dx=0.25, seed=19, n_evac=3000)
        checkpoints = (0, 10, 100)
    elif which == "big":
        sc = I.shopping_centre(n=600, dx=0.25, seed=19, n_evac=9000)
        checkpoints = (0, 10, 100)
    elif which == "chunks":
        sc = I.shopping_centre(n=1024, dx=0.25, seed=23, n_evac=3000)
        checkpoints = (0, 1, 10, 100)
    else:
        sc = I.shopping_centre(n=1024, dx=0.25, seed=23, n_evac=12000)
        checkpoints = (0, 1, 10, 100)
    sim = fps.Sim(sc)
    P = oracle.make_params(sc.desc, sc.ped)
    done = 0
    for k in checkpoints:
        sim.step(k - done)
        done = k
        A = sim.agents()
        bs, perm = sim.bins()
        bs_ref, perm_ref = oracle.build_bins(P, A["x"], A["y"], A["state"])
        say(f"[{which}] step {k}: {len(perm)} binned agents, bins equal:",
            np.array_equal(bs, bs_ref) and np.array_equal(perm, perm_ref))
        assert np.array_equal(bs, bs_ref) and np.array_equal(perm, perm_ref)
        cnt = sim.counts().cpu().numpy()
        assert np.array_equal(cnt, recount(sc, A))


@pytest.mark.parametrize("which,warm", [("cfg1", 0), ("cfg1", 40), ("centre", 300), ("barrier", 400)])
def test_coupled_step_parity_from_identical_state(oracle, which, warm):
    if which == "cfg1":
        sc = I.cfg1_dam_break(n_ped=300)
    elif which == "centre":
        sc = I.shopping_centre(n=256, dx=0.25, seed=9, n_evac=3000)
    else:
        # responders building a barrier before the flood (dry 1 s steps): some
        # walk, some wait out their pick-up or drop timers
        sc = I.add_barrier(I.shopping_centre(n=256, dx=0.25, seed=9, n_evac=500, t_flood=1e9),
                           seed=9, n_resp=150, height=0.4)
    sim = fps.Sim(sc)
    sim.step(warm)
    start, d0 = snapshot(sim, sc)
    ref = oracle.OracleSim(start)
    ref.S.t = d0["t"]
    cnt_gpu0 = sim.counts().cpu().numpy().reshape(-1)
    assert np.array_equal(cnt_gpu0, ref.np_)
    sim.step(1)
    dt = sim.diag()["dt_last"]
    ref.coupled_step(dt)
    h, qx, qy, _ = sim.fields()
    hr, _, _, _ = ref.fields()
    dh = np.abs(h - hr).max()
    A = sim.agents()
    act = start.agents["state"] != 1
    dpos = max(np.abs(A["x"] - ref.x)[act].max(), np.abs(A["y"] - ref.y)[act].max())
    # hazard classes: identical except where the oracle's HR is within 1e-5 of a threshold
    hz = np.zeros(len(ref.cls), bool)
    for a in np.flatnonzero(A["hr_class"] != ref.cls):
        ci = min(int(np.floor(np.float32(start.agents["x"][a]) / np.float32(sc.desc.dx))), sc.desc.nx - 1)
        cj = min(int(np.floor(np.float32(start.agents["y"][a]) / np.float32(sc.desc.dy))), sc.desc.ny - 1)
        _, hrv = oracle.hr_class(ref.S.P, hr[cj, ci], ref.qx[cj * sc.desc.nx + ci], ref.qy[cj * sc.desc.nx + ci])
        hz[a] = min(abs(hrv - t) for t in sc.ped.hr_t) < 1e-5
    mism = np.flatnonzero((A["hr_class"] != ref.cls) & ~hz)
    say(f"[{which} warm {warm}] dt {dt:.4g} max|dh| {dh:.2e} max|dpos| {dpos:.2e} "
        f"class mismatches {len(mism)} (near-threshold {hz.sum()})")
    assert dh <= 1e-4
    assert dpos <= 1e-4
    assert len(mism) == 0
    # exit / arrival decisions come from the cell of the new position: FP32 and FP64
    # positions may straddle a cell edge, so allow a handful (0.5%) of differences
    st_mism = np.flatnonzero(A["state"] != ref.state)
    cnt_mism = int((sim.counts().cpu().numpy().reshape(-1) != ref.np_).sum())
    say(f"    state mismatches {len(st_mism)}, count mismatches {cnt_mism}")
    assert len(st_mism) <= max(1, 0.005 * len(A["x"]))
    assert cnt_mism <= 2 * max(1, 0.005 * len(A["x"]))
    # the rest of the agent record: velocity, destination and wait timer, on
    # every active agent whose class and state came out the same (a class or
    # state decided differently at a threshold changes the walking speed or
    # the destination by design)
    same = act & ~hz & (A["state"] == ref.state) & (A["hr_class"] == ref.cls)
    dv = max(np.abs(A["vx"] - ref.vx)[same].max(), np.abs(A["vy"] - ref.vy)[same].max())
    dtimer = float(np.abs(A["timer"] - ref.timer)[same].max())
    dest_mism = int((A["dest"] != ref.dest)[same].sum())
    waiting = int(np.isin(A["state"], (3, 5)).sum())
    say(f"    max|dv| {dv:.2e} m/s, max|dtimer| {dtimer:.2e} s ({waiting} waiting), "
        f"destination mismatches {dest_mism} of {int(same.sum())}")
    assert dv <= 1e-4
    assert dtimer <= 1e-5
    assert dest_mism == 0
    if which == "barrier":
        assert waiting > 0 and int((A["role"] == 1).sum()) == 150


def test_coupled_window_with_count_replay(oracle):
    """512^2 shopping centre with 2,000 evacuees: the oracle replays the GPU's
    time steps and per-cell evacuee counts; the flood must hold the tolerances
    and the pedestrian statistics must agree."""
    sc = I.shopping_centre(n=512)
    sim = fps.Sim(sc)
    sim.step(200)
    start, d0 = snapshot(sim, sc)
    ref = oracle.OracleSim(start)
    ref.S.t = d0["t"]
    for k in range(1000):
        cnt = sim.counts().cpu().numpy().reshape(-1)
        sim.step(1)
        dt = sim.diag()["dt_last"]
        ref.np_[:] = cnt
        ref.coupled_step(dt)
    h, _, _, _ = sim.fields()
    hr, _, _, _ = ref.fields()
    dh = float(np.abs(h - hr).max())
    d = sim.diag()
    rel = abs(d["mass"] - ref.mass()) / ref.mass()
    A = sim.agents()
    ex_g, ex_o = int((A["state"] == 1).sum()), int((ref.state == 1).sum())
    cls_g = np.bincount(A["hr_class"][A["state"] != 1], minlength=5)
    cls_o = np.bincount(ref.cls[ref.state != 1], minlength=5)
    say(f"coupled window: max|dh| {dh:.2e} mass rel {rel:.2e} exited gpu {ex_g} oracle {ex_o} "
        f"classes gpu {cls_g} oracle {cls_o}")
    assert dh <= 1e-4 and rel <= 1e-6
    assert abs(ex_g - ex_o) <= max(5, 0.02 * len(A["x"]))
    assert np.abs(cls_g - cls_o).sum() <= max(10, 0.02 * len(A["x"]))


def test_evacuation_completes_gpu():
    sc = I.cfg1_dam_break()
    sim = fps.Sim(sc)
    sim.step(2000)
    d = sim.diag()
    say("cfg1 after 2000 steps: states", d["state_count"])
    assert d["state_count"][1] == len(sc.agents["x"])
    assert int(sim.counts().sum()) == 0


def test_sandbag_barrier_hand_timed_gpu():
    gold = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    nx, ny, dx = 20, 4, 1.0
    d = I.GridDesc(nx=nx, ny=ny, dx=dx, dy=dx)
    walk = np.ones((ny, nx), np.uint8)
    h = np.zeros((ny, nx))
    dist = np.stack([I.distance_field(walk, [(19, 3)], dx, dx),
                     I.distance_field(walk, [(2, 1)], dx, dx),
                     I.distance_field(walk, [(3, 1)], dx, dx)])
    A = I.empty_agents(1)
    A["x"][:] = 2.5
    A["y"][:] = 1.5
    A["role"][:] = I.ROLE_RESPONDER
    line = np.array([1 * nx + 3, 1 * nx + 4, 1 * nx + 5], np.int32)
    sc = I.Scenario(desc=d, h=h, qx=h.copy(), qy=h.copy(), z=h.copy(), dist=dist, n_exit=1,
                    walk=walk, agents=A,
                    barrier=dict(cells=line, storage_dest=1, barrier_dest=2, n_layers=3,
                                 bags_per=1, t_bag=gold["bag_thickness"], t_last=gold["bag_thickness"]))
    sim = fps.Sim(sc)
    sim.step(540)
    z = sim.fields()[3]
    dg = sim.diag()
    assert list(z[1, 3:6]) == [0.75, 0.75, 0.5] and dg["drops_total"] == 8 and not dg["barrier_done"]
    sim.step(1)
    z = sim.fields()[3]
    assert list(z[1, 3:6]) == [0.75] * 3 and sim.diag()["barrier_done"] == 1
    sim.step(60)
    assert sim.agents()["state"][0] == 1


def test_barrier_scenario_matches_oracle(oracle):
    """Responders building a barrier on a synthetic layout, dry phase (dt = 1 s).
    FP32 and FP64 trajectories drift apart under the social force, so arrival
    times can differ by a step here and there: the delivered bag counts must
    agree to 15% (+4) and z may differ only at barrier cells."""
    sc = I.shopping_centre(n=128, dx=0.5, seed=21, n_evac=200, t_flood=1e9)
    sc = I.add_barrier(sc, seed=21, n_resp=40, height=0.4)
    sim = fps.Sim(sc)
    ref = oracle.OracleSim(sc)
    for blk in range(6):
        sim.step(100)
        ref.run(100, dts=np.ones(100))
        d = sim.diag()
        zg = sim.fields()[3]
        zr = ref.fields()[3]
        say(f"barrier block {blk}: drops gpu {d['drops_total']} oracle {ref.S.drops_total}, "
            f"layers {d['barrier_layers_done']}/{ref.S.layers_done}")
        assert abs(d["drops_total"] - ref.S.drops_total) <= 4 + 0.15 * ref.S.drops_total
        off_line = np.ones(zg.size, bool)
        off_line[sc.barrier["cells"]] = False
        assert np.array_equal(zg.reshape(-1)[off_line], zr.reshape(-1)[off_line].astype(np.float32))


def test_ped_steps_count_agents_outside_the_exits():
    """The agent-step counter adds, every step, the agents that start the step
    outside the exits (walking, standing or waiting), in single steps and in
    graph-replayed chunks alike."""
    sc = I.cfg1_dam_break()
    n = len(sc.agents["x"])
    one = fps.Sim(sc)
    one.set_graph(0)
    expect = 0
    for _ in range(400):
        expect += n - one.diag()["state_count"][1]
        one.step(1)
    d1 = one.diag()
    many = fps.Sim(sc)
    many.step(400)
    d2 = many.diag()
    say("cfg1 400 steps: ped_steps", d1["ped_steps"], d2["ped_steps"], "expected", expect,
        "exited", d1["state_count"][1])
    assert d1["ped_steps"] == expect
    assert d2["ped_steps"] == expect


@pytest.mark.parametrize("which", ["centre", "barrier", "doors"])
def test_heading_codes_equal_distance_reads(which):
    """The heading and arrival codes derived once per cell (up to 16
    destinations) take the decisions the step takes from the distance fields
    themselves: the same scenario with its navigation map padded to 17
    destinations (beyond the coded ones, so the step reads the fields) walks
    the same agents bit for bit."""
    if which == "centre":
        sc = I.shopping_centre(n=256, dx=0.25, seed=9, n_evac=3000)
        n = 400
    elif which == "barrier":
        sc = I.add_barrier(I.shopping_centre(n=256, dx=0.25, seed=9, n_evac=500, t_flood=1e9),
                           seed=9, n_resp=150, height=0.4)
        n = 600
    else:
        sc = I.add_doors(I.shopping_centre(n=128, dx=332.0 / 128, seed=5232, n_evac=1000, n_exits=1,
                                           q_peak=20.0, duration=1800.0))
        n = 420
    padded = copy.deepcopy(sc)
    pad = np.full((17 - sc.dist.shape[0],) + sc.dist.shape[1:], np.inf, np.float32)
    padded.dist = np.concatenate([sc.dist, pad])
    a, b = fps.Sim(sc), fps.Sim(padded)
    a.step(n)
    b.step(n)
    A, B = a.agents(), b.agents()
    for k in A:
        assert np.array_equal(A[k], B[k]), k
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    say(f"[{which}] {n} steps: coded and field-read headings give the same agents; states {a.diag()['state_count']}")
