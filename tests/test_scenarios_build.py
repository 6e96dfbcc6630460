"""Host-side construction of the paper's experiments (``scenarios``): the
deployment sweep's groups, layers and bag counts, and the evacuation pair's
coupling switch.  No GPU."""
import math

import numpy as np

from paper_1908_05232_amd import inputs as I, scenarios as S


def test_deployment_sweep_groups_layers_and_bags():
    scs = S.deployment_sweep(population=400, n=64, dx=S.SITE_DX, groups=(0.05, 0.5), layers=(1, 3))
    assert [(sc.group, sc.layers) for sc in scs] == [(0.05, 1), (0.05, 3), (0.5, 1), (0.5, 3)]
    for sc in scs:
        n_resp = int(np.sum(sc.agents["role"] == I.ROLE_RESPONDER))
        assert n_resp == round(sc.group * 400)
        assert len(sc.agents["x"]) == 400                   # responders are part of the population
        b = sc.barrier
        assert b["n_layers"] == sc.layers and b["t_bag"] == S.LAYER_M and b["t_last"] == S.LAYER_M
        # one bag covers 0.4 m x 0.3 m: a 2.59 m cell takes ceil(2.59^2 / 0.12) bags per layer
        assert b["bags_per"] == math.ceil(S.SITE_DX ** 2 / 0.12 - 1e-12)
        assert sc.hydro_t[0] >= S.NO_FLOOD                  # no water during the deployment
        line = b["cells"]
        assert len(line) > 0 and np.all(sc.walk.reshape(-1)[line] == 1)
        assert len(set((line // 64).tolist())) == 1          # one row


def test_evacuation_pair_differs_only_in_the_coupling():
    a, b = S.evacuation_pair(population=50, n=48, dx=S.SITE_DX)
    assert a.desc.np_cap == 20 and b.desc.np_cap == 0
    for k in ("x", "y", "role", "v_base"):
        assert np.array_equal(a.agents[k], b.agents[k])
    assert np.array_equal(a.z, b.z) and a.n_exit == b.n_exit == 1
