"""GPU parity of the wading rule (readings W1-W3): one coupled step against
the oracle from the GPU's state on the dam break with 600 people of varied
bodies, the rule alone and together with the stability rule: positions to
the pedestrian bar, with people in the water whose cap is below Table 1's
speed; a push no water can hold back gives the run without the rule bit for
bit; ensemble members equal solo runs."""
import copy
import dataclasses

import numpy as np
import pytest

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import say, snapshot

pytestmark = pytest.mark.gpu
ST_EXITED = 1


def dam_break(stability):
    sc = I.add_bodies(I.cfg1_dam_break(n_ped=600), seed=3, stability=stability)
    sc.ped = dataclasses.replace(sc.ped, wading=1)
    return sc


@pytest.mark.parametrize("stability", [0, 1])
@pytest.mark.parametrize("warm", [20, 60])
def test_one_step_parity_with_the_wading_rule(oracle, stability, warm):
    sc = dam_break(stability)
    sim = fps.Sim(sc)
    sim.step(warm)
    start, d0 = snapshot(sim, sc)
    ref = oracle.OracleSim(start)
    ref.S.t = d0["t"]
    sim.step(1)
    dt = sim.diag()["dt_last"]
    ref.coupled_step(dt)
    A = sim.agents()
    act = start.agents["state"] != ST_EXITED
    # a class may differ only where the oracle's HR is within 1e-5 of a Table 1
    # threshold or its force balance within 1e-4 of tipping (as in the other pedestrian tests)
    d = sc.desc
    mism = np.flatnonzero((A["hr_class"] != ref.cls) & act)
    for a in mism:
        ci = min(int(np.floor(np.float32(start.agents["x"][a]) / np.float32(d.dx))), d.nx - 1)
        cj = min(int(np.floor(np.float32(start.agents["y"][a]) / np.float32(d.dy))), d.ny - 1)
        c = cj * d.nx + ci
        hc, qxc, qyc = start.h.reshape(-1)[c], start.qx.reshape(-1)[c], start.qy.reshape(-1)[c]
        _, hrv = oracle.hr_class(ref.S.P, hc, qxc, qyc)
        _, margin = oracle.unstable(ref.S.P, hc, qxc, qyc, start.agents["height"][a], start.agents["mass"][a])
        assert min(abs(hrv - t) for t in sc.ped.hr_t) < 1e-5 or abs(margin) < 1e-4, (a, hrv, margin)
    same = act & (A["hr_class"] == ref.cls)
    dpos = max(np.abs(A["x"] - ref.x)[same].max(), np.abs(A["y"] - ref.y)[same].max())
    # the people in water whose cap binds (below their class's Table 1 speed)
    wet = np.zeros(len(act), bool)
    capped = 0
    for a in np.flatnonzero(same & (ref.cls >= 1) & (ref.cls <= 4)):
        ci = min(int(np.floor(np.float32(start.agents["x"][a]) / np.float32(d.dx))), d.nx - 1)
        cj = min(int(np.floor(np.float32(start.agents["y"][a]) / np.float32(d.dy))), d.ny - 1)
        cap = oracle.wade_speed(ref.S.P, start.h.reshape(-1)[cj * d.nx + ci], start.agents["height"][a],
                                start.agents["mass"][a])
        wet[a] = True
        capped += cap < sc.ped.v_class[int(ref.cls[a])]
    say(f"[stability {stability}, warm {warm}] t {d0['t']:.1f} s: {int(wet.sum())} people in water, "
        f"{capped} of them capped by wading, class mismatches {len(mism)}, max|dpos| {dpos:.2e}")
    assert capped > 0
    assert dpos <= 1e-4


def test_a_push_no_water_holds_back_changes_nothing():
    sc = dam_break(0)
    giants = copy.deepcopy(sc)
    giants.agents["height"][:] = 100.0
    giants.agents["mass"][:] = 1e7
    giants.ped = dataclasses.replace(giants.ped, wade_k=1e12)
    off = copy.deepcopy(sc)
    off.ped = I.PedParams()
    a, b = fps.Sim(giants), fps.Sim(off)
    a.step(400)
    b.step(400)
    A, B = a.agents(), b.agents()
    for k in ("x", "y", "vx", "vy", "state", "dest", "hr_class"):
        assert np.array_equal(A[k], B[k]), k
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


def test_wading_ensemble_equals_solo_runs():
    more = I.shopping_centre(n=128, dx=0.5, seed=11, n_evac=400, q_peak=1.5, duration=120.0)
    more.ped = dataclasses.replace(more.ped, wading=1)              # the default body for everyone
    scs = [dam_break(1), dam_break(0), more]
    ens = fps.Ensemble(scs)
    ens.step(300)
    for k, sc in enumerate(scs):
        solo = fps.Sim(sc)
        solo.step(300)
        S, E = solo.agents(), ens[k].agents()
        for key in ("x", "y", "vx", "vy", "state", "hr_class"):
            assert np.array_equal(S[key], E[key]), (k, key)
