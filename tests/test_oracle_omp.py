"""The OpenMP build of the oracle (used to time it on all host cores) gives
the serial build's results bit for bit: flood state, volumes, agents."""
import numpy as np

from paper_1908_05232_amd import inputs as I


def test_openmp_build_equals_serial_build(oracle):
    sc = I.add_barrier(I.shopping_centre(n=128, dx=0.5, seed=21, n_evac=300, t_flood=-200.0),
                       seed=21, n_resp=20, height=0.4)
    a, b = oracle.OracleSim(sc), oracle.OracleSim(sc, omp=True)
    a.run(150)
    b.run(150)
    for u, v in zip(a.fields(), b.fields()):
        assert np.array_equal(u, v)
    for k in ("x", "y", "vx", "vy", "timer", "state", "cls", "dest", "np_"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert (a.S.v_in, a.S.v_out, a.S.v_clip, a.S.drops_total) == (b.S.v_in, b.S.v_out, b.S.v_clip,
                                                                   b.S.drops_total)
    assert a.S.v_in > 0.0
