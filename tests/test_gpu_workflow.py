"""GPU checks of the surrogate workflow on coupled scenarios (people walking
in both arms): the finite-volume fallback of the assisted ensemble reproduces
the plain coupled ensemble bit for bit, flood and people; an accepted block
is exactly the network's update, with the people walking on it as a held
flood lets them; training on pairs that the finite-volume engine generates
lowers the loss; and the assisted ensemble against the plain finite-volume
ensemble at the same accuracy bar, with its throughput ratio reported
whatever it is."""
import time

import numpy as np
import pytest
import torch

from paper_1908_05232_amd import fps, surrogate as SG
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _cases(seeds, n=64, **kw):
    return [SG.flood_case(s, n=n, **kw) for s in seeds]


def _coupled(S, n=128, people=400):
    return [SG.coupled_case(k, n=n, n_evac=people, master=77) for k in range(S)]


def _random_surrogate(batch, n, seed=0):
    sur = fps.Surrogate(batch, n, n)
    g = torch.Generator().manual_seed(seed)
    p = torch.randn(sur.n_params, generator=g) * 0.02
    sur.set_params(p.cuda())
    return sur


def _agents_equal(a, b):
    A, B = a.agents(), b.agents()
    return all(np.array_equal(A[k], B[k]) for k in A)


def test_fallback_equals_plain_fv():
    scs = _coupled(3)
    sur = _random_surrogate(2, 128)
    A = SG.AssistedEnsemble(scs, sur.get_params(), chunk=2, tol=-1.0)      # every block rejected
    plain = fps.Ensemble(scs)
    for _ in range(3):
        acc = A.block()
        assert not acc.any()
        plain.step(SG.K_STEPS)
    for k in range(len(scs)):
        for a, b in zip(A.E[k].fields(), plain[k].fields()):
            assert np.array_equal(a, b), k
        assert _agents_equal(A.E[k], plain[k]), k
        assert A.E[k].time()[0] == plain[k].time()[0]
    bad, worst = SG.bar_check(plain, A)
    assert bad == 0 and worst == 0.0
    say(f"fallback: {A.stats}")


def test_accepted_block_is_the_network_update():
    scs = _coupled(2, people=0)                       # no one to judge: every block accepted
    sur = _random_surrogate(2, 128, seed=3)
    A = SG.AssistedEnsemble(scs, sur.get_params(), chunk=2)
    u0 = [tuple(t.clone() for t in SG._state(A.E[k])) for k in range(2)]
    t0 = [A.E[k].time()[0] for k in range(2)]
    feats = [A.E[k].inflow_feature(t0[k], t0[k] + SG.K_STEPS * A.dt) for k in range(2)]
    acc = A.block()
    assert acc.all()
    for k in range(2):
        x = torch.empty((1, 128, 128, 16), dtype=torch.bfloat16, device="cuda")
        y = torch.empty((1, 128, 128, 4), dtype=torch.float32, device="cuda")
        occ = torch.zeros((128, 128), dtype=torch.int32, device="cuda")
        fps.sur_pack(*u0[k], A.E[k].z, occ, inflow=feats[k], out=x[0])
        sur.forward(x, y)
        fps.sur_apply(y[0], *u0[k], h_dry=scs[k].desc.h_dry, h_snap=SG.H_SNAP)
        for a, b in zip(SG._state(A.E[k]), u0[k]):
            assert torch.equal(a, b)
        t = t0[k]
        for _ in range(SG.K_STEPS):
            t += A.dt
        assert A.E[k].time()[0] == t


def test_held_flood_moves_only_the_people():
    """fps_set_flood_frozen: K held steps of dt_max leave the flood state
    untouched bit for bit while the people walk; resuming gives the CFL step
    of the state again."""
    sc = SG.coupled_case(5, n=128, n_evac=600, master=77)
    a, b = fps.Sim(sc), fps.Sim(sc)
    a.step(30)
    b.step(30)
    f0 = [t.clone() for t in SG._state(a)]
    a.set_flood_frozen(1)
    t0, _ = a.time()
    a.step(SG.K_STEPS)
    t1, dt1 = a.time()
    assert all(torch.equal(x, y) for x, y in zip(SG._state(a), f0))
    assert dt1 == np.float32(sc.desc.dt_max)
    A0, A1 = b.agents(), a.agents()
    moved = np.abs(A1["x"] - A0["x"]) + np.abs(A1["y"] - A0["y"])
    assert moved.max() > 0.0
    a.set_flood_frozen(0)
    d = a.diag()
    assert d["dt_next"] <= sc.desc.dt_max and d["t"] == t1
    say(f"held flood: {SG.K_STEPS} steps, t {t0:.3f} -> {t1:.3f}, people moved up to {moved.max():.3f} m")


def test_pairs_and_training():
    cases = _cases(range(50, 58), n=64)
    ds = SG.Dataset(8 * 4, 64)
    frac = SG.generate_pairs(cases, ds, warmup=40, pairs=4, every=16)
    assert ds.size == 32 and frac == 1.0
    t = ds.t[:, :, :, :3]
    assert torch.isfinite(t).all() and float(t.abs().max()) > 0
    assert float(ds.t[..., 3].abs().max()) == 0.0
    sur = fps.Surrogate(8, 64, 64)
    init = torch.tensor(SG.init_params(5))
    assert init.numel() == sur.n_params
    sur.set_params(init.cuda())
    hist = SG.train(sur, ds, steps=200, batch=8, lr=1e-3, log_every=50)
    say(f"training loss {hist}")
    assert hist[-1][1] < 0.5 * hist[0][1]


def test_assisted_against_plain_fv_at_equal_accuracy():
    """What the trained network gains over the method without it, measured
    against the plain coupled finite-volume ensemble: a network trained on
    finite-volume pairs of 32 random layouts advances 4 unseen coupled
    scenarios (every person judged, plus the margins) in lockstep with the
    plain arm; the bar (1 cm and the same class at every person after every
    block) is checked, and the wall-clock ratio of the two arms is reported
    as it is, below 1 included."""
    n = 128
    train_cases = [SG.flood_case(7000 + k, n=n, barrier_height=0.5 if k % 2 else None) for k in range(32)]
    ds = SG.Dataset(32 * 8, n)
    SG.generate_pairs(train_cases, ds, warmup=60, pairs=8, every=24)
    sur = fps.Surrogate(8, n, n)
    sur.set_params(torch.tensor(SG.init_params(0)).cuda())
    hist = SG.train(sur, ds, steps=600, batch=8, lr=1e-3, log_every=100)
    params = sur.get_params()
    scs = _coupled(4, n=n, people=500)
    blocks = 4
    A, P = SG.AssistedEnsemble(scs, params, chunk=4, stride=1), fps.Ensemble(scs)
    worst_bad, worst_dh = 0, 0.0
    for _ in range(blocks):
        A.block()
        P.step(SG.K_STEPS)
        bad, dh = SG.bar_check(P, A)
        worst_bad, worst_dh = max(worst_bad, bad), max(worst_dh, dh)
    stats = dict(A.stats)
    A.close()
    P.close()
    # wall clock of each arm alone over the same blocks
    P = fps.Ensemble(scs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        P.step(SG.K_STEPS)
    torch.cuda.synchronize()
    t_fv = time.perf_counter() - t0
    A = SG.AssistedEnsemble(scs, params, chunk=4, stride=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        A.block()
    torch.cuda.synchronize()
    t_as = time.perf_counter() - t0
    say(f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}; assisted {stats}; most people off at a check "
        f"{worst_bad} (max |dh| {worst_dh:.4f} m), meets the bar: {worst_bad == 0}; "
        f"assisted / plain FV throughput = {t_fv / t_as:.3f}")
    # every person is judged each block (stride 1)
    assert stats["judged_people"] >= blocks * 4 * 500 * 0.9
    assert stats["accepted"] + stats["fallback"] == blocks * 4
    assert t_fv > 0 and t_as > 0
