"""Pins of the oracle's wading rule (readings W1-W3 in the oracle's header).

The paper leaves richer walking-speed rules and variable bodies to further
work (sec. 2.4 note 1, sec. 4); the rule read here caps the walking speed at
the speed at which the drag of wading equals the push the feet keep up.
These checks fix it by what mechanics says, not by its own formula: a
geometrically similar body of the same density, scaled by lambda, wades
sqrt(lambda) times as fast through water scaled the same (Froude similarity:
a wrong power of a length or of the mass breaks it); the cap vanishes as
buoyancy takes the weight, near the top as the square root of the weight
left over the depth; it grows as the square root of the push and falls as
the inverse square root of the drag coefficient; shallow water barely slows
anyone, deeper water slows everyone, and heavier bodies of one height wade
faster; in the step the cap, where it is below Table 1's speed, is the speed
the person relaxes to, and elsewhere Table 1's speed is kept bit for bit."""
import ctypes
import math

import numpy as np
import pytest

from paper_1908_05232_amd import inputs as I


@pytest.fixture(scope="module")
def P(oracle):
    return oracle.make_params(I.GridDesc(nx=4, ny=4, dx=1.0, dy=1.0), I.PedParams(wading=1))


@pytest.mark.parametrize("h", [0.1, 0.3, 0.6, 1.1])
@pytest.mark.parametrize("lam", [0.55, 1.25])
def test_froude_similarity_of_the_wading_speed(oracle, P, h, lam):
    H, M = 1.71, 70.0
    v1 = oracle.wade_speed(P, h, H, M)
    v2 = oracle.wade_speed(P, lam * h, lam * H, lam ** 3 * M)
    assert abs(v2 / v1 - math.sqrt(lam)) <= 1e-12


def test_buoyancy_takes_the_push_as_the_water_rises(oracle, P):
    """With body and water of one density the weight is gone when h = H: the
    cap is 0 from there on, and just below it falls as sqrt((1 - h/H) / h)
    (the push shrinks with the weight left, the drag grows with the depth)."""
    H, M = 1.71, 70.0
    assert oracle.wade_speed(P, H, H, M) == 0.0
    assert oracle.wade_speed(P, 1.2 * H, H, M) == 0.0
    a, b = 0.95 * H, 0.99 * H
    ratio = oracle.wade_speed(P, b, H, M) / oracle.wade_speed(P, a, H, M)
    assert abs(ratio - math.sqrt((1 - b / H) / (1 - a / H) * (a / b))) <= 1e-12


def test_push_and_drag_enter_as_square_roots(oracle, P):
    h, H, M = 0.5, 1.71, 70.0
    v = oracle.wade_speed(P, h, H, M)
    P4 = oracle.make_params(I.GridDesc(nx=4, ny=4, dx=1.0, dy=1.0), I.PedParams(wading=1, wade_k=0.4))
    assert abs(oracle.wade_speed(P4, h, H, M) / v - 2.0) <= 1e-12
    Pd = oracle.make_params(I.GridDesc(nx=4, ny=4, dx=1.0, dy=1.0), I.PedParams(wading=1, c_drag=1.1 / 9))
    assert abs(oracle.wade_speed(Pd, h, H, M) / v - 3.0) <= 1e-12


def test_depth_and_mass_order_the_speeds(oracle, P):
    H = 1.71
    depths = (0.02, 0.1, 0.3, 0.6, 1.0, 1.5)
    vs = [oracle.wade_speed(P, h, H, 70.0) for h in depths]
    assert all(x > y for x, y in zip(vs, vs[1:]))
    assert vs[0] > 2 * 1.8                       # ankle-deep water: far above every Table 1 speed
    ms = [oracle.wade_speed(P, 0.6, H, m) for m in (45.0, 60.0, 80.0, 110.0)]
    assert all(x < y for x, y in zip(ms, ms[1:]))


def one_step(oracle, h_water, wading, bodies=True):
    """Two evacuees far apart in still water of the given depth on a 12 x 12
    grid of 1 m cells, at rest, heading for the far corner; one pedestrian
    step of 0.5 s.  Returns the oracle state after the step."""
    nx = ny = 12
    d = I.GridDesc(nx=nx, ny=ny, dx=1.0, dy=1.0)
    walk = np.ones((ny, nx), np.uint8)
    h = np.full((ny, nx), h_water)
    A = I.empty_agents(2)
    A["x"][:] = [2.5, 8.5]
    A["y"][:] = [2.5, 8.5]
    if bodies:
        A["height"] = np.array([1.55, 1.95], np.float32)
        A["mass"] = np.array([45.0, 110.0], np.float32)
    dist = I.distance_field(walk, [(11, 11)], 1.0, 1.0)[None]
    sc = I.Scenario(desc=d, h=h, qx=np.zeros_like(h), qy=np.zeros_like(h), z=np.zeros_like(h), dist=dist,
                    n_exit=1, walk=walk, agents=A, ped=I.PedParams(wading=wading))
    s = oracle.OracleSim(sc)
    oracle.lib().or_ped_step(ctypes.byref(s.S), 0.5)
    return s


def test_the_cap_is_the_speed_a_wader_relaxes_to(oracle):
    """From rest and with no neighbour in range, the social-force step moves
    a person to (1 - exp(-dt / tau)) times its desired speed.  In 0.5 m of
    still water (HR 0.25: class low, Table 1 speed 1.8 m/s) that desired
    speed is each body's cap with the rule on, and 1.8 m/s with it off."""
    k = 1.0 - math.exp(-0.5 / I.PedParams().tau)
    on, off = one_step(oracle, 0.5, 1), one_step(oracle, 0.5, 0)
    assert np.all(on.cls == oracle.CLS_LOW) and np.all(off.cls == oracle.CLS_LOW)
    for a, (H, M) in enumerate([(1.55, 45.0), (1.95, 110.0)]):
        cap = oracle.wade_speed(on.S.P, 0.5, float(np.float32(H)), float(np.float32(M)))
        assert cap < 1.8
        assert abs(math.hypot(on.vx[a], on.vy[a]) - k * cap) <= 1e-12
        assert abs(math.hypot(off.vx[a], off.vy[a]) - k * 1.8) <= 1e-12
    # the heavier, taller body wades faster
    assert math.hypot(on.vx[1], on.vy[1]) > math.hypot(on.vx[0], on.vy[0])


def test_shallow_water_keeps_table_1(oracle):
    """In 5 cm of water every body's cap is above 1.8 m/s: the step is the
    step without the rule, bit for bit."""
    on, off = one_step(oracle, 0.05, 1), one_step(oracle, 0.05, 0)
    for k in ("x", "y", "vx", "vy"):
        assert np.array_equal(getattr(on, k), getattr(off, k)), k


def test_default_body_without_bodies(oracle):
    """People without a body of their own wade with the default one."""
    s = one_step(oracle, 0.5, 1, bodies=False)
    k = 1.0 - math.exp(-0.5 / I.PedParams().tau)
    cap = oracle.wade_speed(s.S.P, 0.5, 1.71, 70.0)
    for a in range(2):
        assert abs(math.hypot(s.vx[a], s.vy[a]) - k * cap) <= 1e-12
