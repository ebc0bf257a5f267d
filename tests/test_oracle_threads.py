"""The oracle's time step gives the same bits on any number of threads (its
nodes are updated independently), so the all-core CPU timing of the bench
runs the same arithmetic as the tests."""
import numpy as np

from paper_1508_02960_amd import inputs


def test_threads_do_not_change_the_oracle_step(orc):
    shape = (9, 10, 11)
    sp = inputs.random_spheres(shape, 3, (1.5, 3.0), seed=21)
    g0 = inputs.random_populations(shape, 1e-3, seed=22)
    out = []
    for n in (1, 4):
        orc.set_threads(n)
        o = orc.Oracle(shape, tau=0.7, magic=3 / 16, delta_rho=1e-3, collision="mrt",
                       wall="cli", spheres=sp)
        o.set_state(g0)
        o.step(4)
        out.append(o.g.copy())
    orc.set_threads(1)
    assert np.array_equal(out[0], out[1])
