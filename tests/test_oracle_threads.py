"""The oracle's threaded loops give the serial program's results bit for bit.

The long-run reference data under tests/golden/ are produced with every host
core; these tests show that the thread count changes no bit of any field the
parity tests compare (populations, moments, particle state, hydrodynamic and
contact forces, q), in 2D and 3D, with walls, periodic seams, spinning
particles, contacts, and lattices whose outer axis is longer and shorter
than the number of footprint slabs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2613_amd import inputs as I


def _run(dim, box, n, R, threads, steps, wall_y, seed):
    O.set_threads(threads)
    O.set_parallel_minimum(1, 1)  # these small boxes take the threaded path too
    try:
        pos = I.place_particles(dim, box, R, n, seed, wall_y=wall_y)
        # one overlapping pair (a contact from the first step) and, with
        # walls, one particle touching the lower wall
        pos[2] = pos[1]
        pos[2, 0] = (pos[1, 0] + 2.0 * R - 0.15) % box[0]
        if wall_y:
            pos[3, 1] = R - 0.5 - 0.1
        vel = I.random_velocities(dim, n, 0.02, seed + 1)
        om = I.random_velocities(3, n, 2e-3, seed + 2)
        rad = np.full(n, R)
        rho = np.full(n, 3.0)
        fixed = np.zeros(n, np.uint8)
        fixed[0] = 1
        sim = O.OracleSim(dim, box, 0.58, wall_y=wall_y, fluid_force=(3e-6, 1e-6, 0),
                          particle_accel=(0, -1e-5, 0), samples=4 if dim == 3 else 8,
                          kn=400.0, restitution=0.8)
        sim.set_particles(pos, vel, om, rad, rho, fixed)
        sim.step(1)
        fc_first = sim.contact_forces()
        sim.step(steps - 1)
        out = {"f": sim.get_f(), "q": sim.q(), "Fc_first": fc_first}
        out["rho"], out["u"] = sim.macro()
        out["x"], out["v"], out["w"] = sim.particles()
        out["F"], out["T"] = sim.forces()
        out["Fc"] = sim.contact_forces()
        out["count"] = sim.footprint_counts()
        sim.close()
        return out
    finally:
        O.set_threads(0)
        O.set_parallel_minimum()


@pytest.mark.parametrize("dim,box,n,R,wall_y", [
    (3, (40, 36, 24), 8, 4.0, True),      # outer axis (z) shorter than 64 slabs
    (3, (24, 20, 72), 10, 3.5, False),    # outer axis longer: slabs of several planes
    (2, (64, 100), 14, 5.0, True),        # 2D, outer axis (y) with walls
    (2, (80, 70), 12, 6.0, False),
])
def test_threaded_oracle_equals_serial(dim, box, n, R, wall_y):
    steps = 25
    a = _run(dim, box, n, R, 1, steps, wall_y, 101 + dim)
    b = _run(dim, box, n, R, 4, steps, wall_y, 101 + dim)
    c = _run(dim, box, n, R, 7, steps, wall_y, 101 + dim)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    # the run is not trivial: particles moved, forces and contacts are nonzero
    assert np.abs(a["F"]).max() > 0 and np.abs(a["T"]).max() > 0
    assert np.count_nonzero(np.abs(a["Fc_first"]).max(axis=1)) >= (3 if wall_y else 2)


def test_set_threads_reports_count():
    assert O.set_threads(3) == 3
    assert O.set_threads(1) == 1
    assert O.set_threads(0) >= 1
