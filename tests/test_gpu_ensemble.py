"""GPU checks of the ensemble path: one set of launches per step over
scenarios of uneven grids must give, scenario by scenario, exactly the
results of running each scenario alone; graph replay must equal eager
launches; end times and the dry-step skip must hold."""
import copy

import numpy as np
import pytest

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def mixed_scenarios():
    a = I.shopping_centre(n=96, dx=0.5, seed=11, n_evac=300, q_peak=1.5, duration=120.0)
    b = I.shopping_centre(n=160, dx=0.5, seed=12, n_evac=700, q_peak=2.5, duration=120.0)
    b = I.add_barrier(b, seed=12, n_resp=30, height=0.4)
    c = I.cfg1_dam_break(n_ped=150)
    d = I.lake_at_rest(70, 33, 0.5, seed=5)
    return [a, b, c, d]


def test_ensemble_equals_solo_runs():
    scs = mixed_scenarios()
    ens = fps.Ensemble(scs)
    ens.step(157)
    for k, sc in enumerate(scs):
        solo = fps.Sim(sc)
        solo.step(157)
        fe, fs = ens[k].fields(), solo.fields()
        for x, y in zip(fe, fs):
            assert np.array_equal(x, y), (k, sc.name)
        if sc.agents is not None:
            A, B = ens[k].agents(), solo.agents()
            for key in A:
                assert np.array_equal(A[key], B[key]), (k, key)
        de, ds = ens[k].diag(), solo.diag()
        assert de["t"] == ds["t"] and de["mass"] == ds["mass"] and de["drops_total"] == ds["drops_total"]
        say(f"scenario {k} ({sc.name}): t = {de['t']:.3f} s, identical to the solo run")


@pytest.mark.parametrize("copies", [4, 90])
def test_lanes_per_agent_do_not_change_results(copies):
    """An ensemble of many agents gives each agent fewer lanes than a solo run
    (4 lanes from 8,193 agents, 1 from 262,145; 16 below): the forces are
    summed in the same slot order either way, so every member still equals
    its solo run bit for bit.  4 copies of 3,000 agents run on 4 lanes, 90 on 1."""
    base = [I.shopping_centre(n=160, dx=0.5, seed=40 + k, n_evac=3000, q_peak=4.0, duration=60.0)
            for k in range(4)]
    scs = [copy.deepcopy(base[k % 4]) for k in range(copies)]
    ens = fps.Ensemble(scs)
    ens.step(180)
    moved = 0
    for k in (0, copies - 1):
        solo = fps.Sim(scs[k])
        solo.step(180)
        A, B = ens[k].agents(), solo.agents()
        for key in A:
            assert np.array_equal(A[key], B[key]), (copies, k, key)
        for x, y in zip(ens[k].fields(), solo.fields()):
            assert np.array_equal(x, y), (copies, k)
        moved += int((np.abs(A["x"] - scs[k].agents["x"]) > 0).sum())
    say(f"{copies} x 3000 agents: members 0 and {copies - 1} equal their solo runs ({moved} agents moved)")
    assert moved > 0


def test_graph_replay_equals_eager():
    sc = I.shopping_centre(n=128, dx=0.5, seed=8, n_evac=400)
    a, b = fps.Sim(sc), fps.Sim(sc)
    a.set_graph(0)
    b.set_graph(16)
    a.step(200)
    b.step(200)       # 12 graph replays + 8 eager steps
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    A, B = a.agents(), b.agents()
    for k in A:
        assert np.array_equal(A[k], B[k])
    assert a.diag()["t"] == b.diag()["t"]


def test_end_times_stop_scenarios():
    scs = mixed_scenarios()[:3]
    ens = fps.Ensemble(scs)
    ends = [2.0, 5.0, 1e9]
    for m, t_end in zip(ens.members, ends):
        m.set_end_time(t_end)
    assert ens.active() == 3
    ens.step(400)
    d = [m.diag() for m in ens.members]
    say("times:", [x["t"] for x in d], "active:", [x["active"] for x in d])
    assert ens.active() == 1
    for x, t_end in zip(d[:2], ends[:2]):
        assert x["t"] >= t_end and x["t"] - x["dt_last"] < t_end and x["active"] == 0
    # stopped scenarios no longer change
    f0 = ens[0].fields()
    ens.step(10)
    assert all(np.array_equal(x, y) for x, y in zip(f0, ens[0].fields()))


def test_stopped_member_keeps_its_chunk_scanned_bins(oracle):
    """A member with more bins than one block scans (1024^2 cells: the
    multi-block scan) stops at its end time while the others step on: its
    bins, taken in its last step, stay those of its agents (the oracle's
    stable sort), step after step."""
    big = I.shopping_centre(n=1024, dx=0.25, seed=23, n_evac=3000, q_peak=2.0)
    scs = [big] + mixed_scenarios()[:2]
    ens = fps.Ensemble(scs)
    ens[0].set_end_time(1.0)
    ens.step(200)
    d0 = ens[0].diag()
    assert d0["active"] == 0 and ens.active() == 2
    P = oracle.make_params(big.desc, big.ped)
    bs0, perm0 = ens[0].bins()
    A = ens[0].agents()
    bs_ref, perm_ref = oracle.build_bins(P, A["x"], A["y"], A["state"])
    assert np.array_equal(bs0, bs_ref) and np.array_equal(perm0, perm_ref)
    ens.step(30)
    bs1, perm1 = ens[0].bins()
    assert np.array_equal(bs0, bs1) and np.array_equal(perm0, perm1)
    assert all(np.array_equal(A[k], v) for k, v in ens[0].agents().items())
    say(f"stopped member: t = {d0['t']:.3f}, {len(perm0)} agents binned, bins unchanged over 30 more steps")


def test_dry_steps_skip_the_flood_update(oracle):
    sc = I.shopping_centre(n=128, dx=0.5, seed=21, n_evac=50, t_flood=30.0, q_peak=1.0,
                           duration=60.0)
    sc = I.add_barrier(sc, seed=21, n_resp=20, height=0.2)
    sim = fps.Sim(sc)
    sim.step(40)
    d = sim.diag()
    say(f"after 40 steps: t = {d['t']:.2f} s, flood updates run: {d['flood_steps']}")
    # 30 dry steps of 1 s before the hydrograph starts; the first step always runs
    assert d["flood_steps"] < d["step"] and d["any_wet"] == 1
    ref = oracle.OracleSim(sc)
    dts = []
    sim2 = fps.Sim(sc)
    for _ in range(40):
        sim2.step(1)
        dts.append(sim2.diag()["dt_last"])
    ref.run(40, dts=np.array(dts))
    h, _, _, _ = sim2.fields()
    assert np.abs(h - ref.fields()[0]).max() <= 1e-4


def test_ensemble_hll_equals_solo_runs():
    """The HLL flux set on a whole ensemble equals solo HLL runs bit for bit;
    a member's own flux cannot differ from its ensemble's."""
    scs = mixed_scenarios()[:2]
    for sc in scs:
        sc.desc.flux = fps.FPS_FLUX_HLL
    ens = fps.Ensemble(scs)
    ens.step(120)
    for k, sc in enumerate(scs):
        solo = fps.Sim(sc)
        solo.step(120)
        for x, y in zip(ens[k].fields(), solo.fields()):
            assert np.array_equal(x, y), (k, sc.name)
    with pytest.raises(fps.FpsError):
        ens[0].set_flux(fps.FPS_FLUX_HLLC)


def test_ensemble_autotune_cache(tmp_path):
    """fps_ens_autotune keys its cache by the mix of grids: the first call
    times and appends one line, a second ensemble of the same mix reads the
    same rows per wave back without timing, a single-grid line in the same
    file is still read by fps_autotune, and another mix does not match."""
    cache = tmp_path / "tiles.txt"
    scs = mixed_scenarios()
    sim = fps.Sim(scs[0])
    rows0, _ = sim.autotune(cache)
    ens = fps.Ensemble(scs)
    ens.autotune(cache)
    rows = [m.rows_per_wave() for m in ens.members]
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1].split()[1] == "ens"
    again = fps.Ensemble(scs)
    again.autotune(cache)
    assert [m.rows_per_wave() for m in again.members] == rows
    assert len(cache.read_text().splitlines()) == 2
    assert fps.Sim(scs[0]).autotune(cache)[0] == rows0
    other = fps.Ensemble(scs[:2])
    other.autotune(cache)
    assert len(cache.read_text().splitlines()) == 3
    again.step(40)
    ref = fps.Ensemble(scs)
    ref.step(40)
    for a, b in zip(again.members, ref.members):
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)
    say(f"ensemble rows per wave {rows}, cached")
