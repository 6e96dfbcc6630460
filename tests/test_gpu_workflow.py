"""GPU checks of the surrogate workflow: the finite-volume fallback of the
assisted ensemble reproduces the plain finite-volume ensemble bit for bit,
an accepted block is exactly the network's update, and training on pairs
that the finite-volume engine generates lowers the loss."""
import numpy as np
import pytest
import torch

from paper_1908_05232_amd import fps, surrogate as SG
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _cases(seeds, n=64, **kw):
    return [SG.flood_case(s, n=n, **kw) for s in seeds]


def _random_surrogate(batch, n, seed=0):
    sur = fps.Surrogate(batch, n, n)
    g = torch.Generator().manual_seed(seed)
    p = torch.randn(sur.n_params, generator=g) * 0.02
    sur.set_params(p.cuda())
    return sur


def test_fallback_equals_plain_fv():
    cases = _cases([31, 32, 33])
    sur = _random_surrogate(2, 64)
    A = SG.AssistedEnsemble(cases, sur.get_params(), chunk=2, tol=-1.0)      # every block rejected
    plain, _ = SG._flood_ensemble(cases)
    for _ in range(3):
        acc = A.block()
        assert not acc.any()
    plain.step(3 * SG.K_STEPS)
    for k in range(len(cases)):
        for a, b in zip(A.E[k].fields(), plain[k].fields()):
            assert np.array_equal(a, b), k
        assert A.E[k].diag()["t"] == plain[k].diag()["t"] == A.t[k]
    say(f"fallback: {A.stats}")


def test_accepted_block_is_the_network_update():
    cases = _cases([41, 42], n=64)
    for c in cases:                                  # no crowd: nothing to judge, every block accepted
        c.agents = {k: v[:0] for k, v in c.agents.items()}
    sur = _random_surrogate(2, 64, seed=3)
    A = SG.AssistedEnsemble(cases, sur.get_params(), chunk=2)
    u0 = [tuple(t.clone() for t in SG._state(A.E[k])) for k in range(2)]
    feats = [A.E[k].inflow_feature(0.0, SG.K_STEPS * A.dt) for k in range(2)]
    assert all(f[3] > 0 for f in feats)
    acc = A.block()
    assert acc.all()
    for k in range(2):
        x = torch.empty((1, 64, 64, 16), dtype=torch.bfloat16, device="cuda")
        y = torch.empty((1, 64, 64, 4), dtype=torch.float32, device="cuda")
        fps.sur_pack(*u0[k], A.E[k].z, A.crowds[k].occ, inflow=feats[k], out=x[0])
        sur.forward(x, y)
        fps.sur_apply(y[0], *u0[k], h_dry=cases[k].sc.desc.h_dry, h_snap=SG.H_SNAP)
        for a, b in zip(SG._state(A.E[k]), u0[k]):
            assert torch.equal(a, b)
        assert A.E[k].diag()["t"] == A.t[k] == A._acc_time(0.0)


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


def test_trained_network_beats_no_update_on_held_out_pairs():
    """What the learned part gains over the method without it: trained on
    finite-volume pairs of 32 random layouts, the network's depth error on
    pairs of 8 unseen layouts is well below that of keeping the state (the
    update a block would make without the network)."""
    n = 128
    train_cases = [SG.flood_case(7000 + k, n=n, barrier_height=0.5 if k % 2 else None) for k in range(32)]
    ds = SG.Dataset(32 * 4, n)
    SG.generate_pairs(train_cases, ds, warmup=60, pairs=4, every=24)
    sur = fps.Surrogate(8, n, n)
    sur.set_params(torch.tensor(SG.init_params(0)).cuda())
    hist = SG.train(sur, ds, steps=600, batch=8, lr=1e-3, log_every=100)
    held = [SG.flood_case(8000 + k, n=n) for k in range(8)]
    kept = []
    SG.generate_pairs(held, SG.Dataset(16, n), warmup=90, pairs=2, every=40, keep=kept)
    ev = SG.evaluate(sur, held, kept)
    say(f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}; held-out {ev}")
    assert ev["sur_rmse_h"] < 0.5 * ev["persist_rmse_h"]
    assert ev["sur_bad_people"] < ev["persist_bad_people"]
