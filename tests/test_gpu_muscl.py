"""GPU parity of the second-order variant of the flood update (MUSCL with the
minmod limiter, Audusse et al.'s second-order bed slope, Heun's two-stage
step; fps_set_order(2)) against the FP64 oracle's same variant, with the
first-order tolerances: max |dh| <= 1e-4 m, max |dq| <= 5e-4 m^2/s, relative
mass error <= 1e-6 per window, the oracle replaying the GPU's time steps
and its own time step agreeing to 1e-5.  Also: still water stays still,
results do not depend on the tile shape, ensemble members equal their solo
runs bit for bit, and the calls refuse what the variant does not support."""
import numpy as np
import pytest

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import random_wet_dry, say
from tests.test_gpu_flood import check_window

pytestmark = pytest.mark.gpu


def _o2(sc, flux=0):
    sc.desc.order = 2
    sc.desc.flux = flux
    return sc


def test_lake_at_rest_second_order_gpu():
    sc = _o2(I.lake_at_rest(130, 97, 0.5, seed=11))
    sim = fps.Sim(sc)
    sim.step(500)
    h, qx, qy, _ = sim.fields()
    say("second order, lake at rest: max|q|", np.abs(qx).max(), np.abs(qy).max(), "max|dh|",
        np.abs(h - sc.h).max())
    # the centred bed-slope term cancels the face terms exactly only in exact
    # arithmetic: in FP32 each step leaves about g h 6e-8 dt / dx of discharge,
    # accumulating over the 500 steps (the FP64 oracle holds 1e-12)
    assert np.abs(qx).max() <= 5e-5 and np.abs(qy).max() <= 5e-5
    assert np.abs(h - sc.h.astype(np.float32)).max() <= 1e-6


def test_dam_breaks_second_order(oracle):
    sc = _o2(I.cfg1_dam_break())
    sc.agents = None
    check_window(oracle, fps.Sim(sc), sc, 500, "order 2, cfg1 dam break 64x64")
    for nx, hR in ((400, 0.1), (300, 0.0)):
        sc = _o2(I.dam_break_1d(nx, 32.0, 1.0, hR))
        check_window(oracle, fps.Sim(sc), sc, 300, f"order 2, 1d dam break nx={nx} hR={hR}")


@pytest.mark.parametrize("nx,ny", [(1, 9), (7, 1), (62, 5), (63, 64), (131, 70)])
def test_ragged_grids_second_order(oracle, nx, ny):
    sc = _o2(random_wet_dry(nx, ny, 0.5, seed=nx * 100 + ny, bc=(0, 1, 0, 1)))
    check_window(oracle, fps.Sim(sc), sc, 200, f"order 2, random {nx}x{ny}", throughput=True)


@pytest.mark.parametrize("side,flux", [(0, 0), (2, 0), (3, 1)])
def test_inflow_second_order(oracle, side, flux):
    nx, ny = 70, 45
    n_along = ny if side <= 1 else nx
    bc = [1, 1, 1, 1]
    bc[side] = 0
    sc = _o2(random_wet_dry(nx, ny, 0.5, seed=40 + side, bc=tuple(bc), inflow=(side, 5, n_along - 7)), flux)
    sim = fps.Sim(sc)
    check_window(oracle, sim, sc, 200, f"order 2, flux {flux}, inflow side {side}", throughput=True)
    assert sim.diag()["v_in"] > 0.0


def test_shopping_centre_second_order(oracle):
    sc = _o2(I.shopping_centre(n=128, dx=0.5, seed=3, n_evac=10, q_peak=2.0, duration=120.0))
    sc.agents = None
    sim = fps.Sim(sc)
    sim.step(300)
    check_window(oracle, sim, sc, 500, "order 2, shopping centre 128^2 steps 300-800")


def test_second_order_tile_shapes_and_ensemble_bit_for_bit():
    a = _o2(I.shopping_centre(n=96, dx=0.5, seed=11, n_evac=200, q_peak=1.5, duration=120.0))
    b = _o2(I.shopping_centre(n=160, dx=0.5, seed=12, n_evac=300, q_peak=2.5, duration=120.0))
    ref = []
    for sc in (a, b):
        sim = fps.Sim(sc)
        sim.step(150)
        ref.append(sim.fields()[:3])
        sim2 = fps.Sim(sc)
        sim2.set_rows_per_wave(16)
        sim2.step(150)
        for u, v in zip(sim2.fields()[:3], ref[-1]):
            assert np.array_equal(u, v)
    ens = fps.Ensemble([a, b])
    ens.step(150)
    for k in range(2):
        for u, v in zip(ens[k].fields()[:3], ref[k]):
            assert np.array_equal(u, v), k


def test_second_order_refusals():
    sc = I.cfg1_dam_break()
    sim = fps.Sim(sc)
    with pytest.raises(fps.FpsError):
        sim.set_order(3)
    import torch
    mask = torch.ones((4, 4), dtype=torch.uint8, device="cuda")
    sim.set_judge_region(mask, 16)
    with pytest.raises(fps.FpsError):
        sim.set_order(2)
    sim.set_judge_region(None, 16)
    sim.set_order(2)
    with pytest.raises(fps.FpsError):
        sim.set_judge_region(mask, 16)
    ens = fps.Ensemble([I.cfg1_dam_break(), I.cfg1_dam_break(n_ped=5)])
    with pytest.raises(fps.FpsError):
        ens[0].set_order(2)
    ens.set_order(2)
