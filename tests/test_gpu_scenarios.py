"""The paper's two experiments driven end to end on reduced sites
(``paper_1908_05232_amd.scenarios``): the evacuation with and without the
people's effect on the flood (sec. 3.2), and the deployment sweep of responder
group sizes x sandbag layers with the flood over each finished barrier (sec. 3.3)."""
import copy

import numpy as np
import pytest

from paper_1908_05232_amd import fps, scenarios as S
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

N, DX = 64, S.SITE_DX            # half the paper's site at its cell size


def test_uncoupled_evacuation_leaves_the_flood_alone():
    """With the evacuee cap at zero the people do not touch the flood: its flood
    equals a run with no people bit for bit, while the coupled run, whose
    evacuees raise the roughness of the wet cells they stand in, differs."""
    coupled, uncoupled = S.evacuation_pair(population=200, n=N, dx=DX, duration=600.0)
    plain = copy.deepcopy(uncoupled)
    plain.agents = None
    sims = [fps.Sim(sc) for sc in (coupled, uncoupled, plain)]
    for s in sims:
        s.step(800)
    (hc, qc, _, _), (hu, qu, _, _), (hp, qp, _, _) = (s.fields() for s in sims)
    d = [s.diag() for s in sims]
    say(f"evacuation {d[0]['t']:.0f} s: exited coupled {d[0]['state_count'][1]}, uncoupled {d[1]['state_count'][1]}; "
        f"coupled vs uncoupled max|dh| {np.abs(hc - hu).max():.3e}")
    assert np.array_equal(hu, hp) and np.array_equal(qu, qp)
    assert not np.array_equal(hc, hu)


def test_deployment_sweep_and_barrier_floods():
    """More responders finish a barrier sooner, more layers take longer, every
    finished barrier has its layers and at least the bags they need; behind the
    tallest barrier the water arrives later than with none (on this layout the
    line spans the concourse only, so the flood still reaches the north part
    through the side corridors)."""
    scs = S.deployment_sweep(population=400, n=N, dx=DX, groups=(0.1, 0.4), layers=(1, 2))
    res = S.run_deployment(scs, t_max=8 * 3600.0)
    t = {(r["group"], r["layers"]): r["t_complete"] for r in res}
    say("deployment minutes:", {k: None if v is None else round(v / 60.0, 1) for k, v in t.items()})
    assert all(v is not None for v in t.values())
    for L in (1, 2):
        assert t[(0.4, L)] < t[(0.1, L)]
    for g in (0.1, 0.4):
        assert t[(g, 2)] > t[(g, 1)]
    for r in res:
        assert r["layers_done"] == r["layers"]
        assert r["drops"] >= r["layers"] * r["line_cells"] * r["bags_per_cell_layer"]
    fl = S.barrier_floods(population=200, n=N, dx=DX, layers=(0, 2, 6), duration=600.0, t_run=600.0)
    say("barrier floods (layers, max depth, max HR, wet cells downstream, arrival behind the line):",
        [(f["layers"], round(f["max_depth_downstream_m"], 3), round(f["max_hr_downstream"], 3),
          f["wet_cells_downstream"], f["t_water_behind_line"]) for f in fl])
    a0, a6 = fl[0]["t_water_behind_line"], fl[-1]["t_water_behind_line"]
    assert a0 is not None and (a6 is None or a6 > a0)


@pytest.mark.parametrize("q_peak", [2.0, 10.0])
def test_evacuation_matches_the_oracle(oracle, q_peak):
    """Scenario 1 on the paper's site (128^2 cells over 332 m, the door flow
    from t = -5 min, 1,000 people, the breach at t = 0), run to the end on
    the GPU and on the FP64 oracle, both polled every step: the same number
    of evacuees, the evacuation time within 3 % (FP32 and FP64 walks part
    after a few hundred steps, so arrival times differ by a few steps), the
    door entries within 2 % and the largest number of people seen at once in
    the wet hazard classes, a statistic of the crowd, within 25 % or, for the
    few people of a small flood, within the counting noise 3 sqrt(N) + 3."""
    sc, _ = S.evacuation_pair(population=1000, q_peak=q_peak)

    def run_gpu():
        sim = fps.Sim(sc)
        peak, n_evac, t_evac = np.zeros(6, int), None, None
        while t_evac is None:
            sim.step(1)
            d = sim.diag()
            sc_ = d["state_count"]
            if d["any_wet"] or d["doors_closed"]:
                peak = np.maximum(peak, d["class_count"])
            if n_evac is None and d["doors_closed"]:
                n_evac = sc_[0] + sc_[1]
            if n_evac is not None and sc_[0] + sc_[6] == 0:
                t_evac = d["t"]
            assert d["t"] < 4000.0
        return t_evac, n_evac, peak, d["door_entries"]

    def run_oracle():
        ref = oracle.OracleSim(sc)
        peak, n_evac, t_evac = np.zeros(6, int), None, None
        while t_evac is None:
            ref.coupled_step(0.0)
            st = ref.state
            inside = (st == 0) | (st == 6)
            if ref.S.any_wet or ref.S.doors_closed:
                peak = np.maximum(peak, np.bincount(ref.cls[inside], minlength=6))
            if n_evac is None and ref.S.doors_closed:
                n_evac = int((st == 0).sum() + (st == 1).sum())
            if n_evac is not None and inside.sum() == 0:
                t_evac = ref.t
            assert ref.t < 4000.0
        return t_evac, n_evac, peak, ref.S.door_in

    tg, ng, pg, eg = run_gpu()
    to, no, po, eo = run_oracle()
    say(f"breach {q_peak} m^2/s: evacuated gpu {tg:.1f} s oracle {to:.1f} s, evacuees {ng} / {no}, "
        f"entries {eg} / {eo}, wet-class peaks gpu {pg[1:5]} oracle {po[1:5]}")
    assert ng == no == 1000
    assert abs(tg - to) <= 0.03 * to
    assert abs(eg - eo) <= 0.02 * eo
    n_o = int(po[1:5].sum())
    assert abs(int(pg[1:5].sum()) - n_o) <= max(0.25 * n_o, 3.0 * np.sqrt(n_o) + 3.0)
