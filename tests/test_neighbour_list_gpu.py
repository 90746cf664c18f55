"""DEM neighbour lists rebuilt every `every` steps with a displacement guard
("Parallel implementation": a list rebuilt about every 100th step) against the
oracle's all-pairs contact search and against the per-step cell list.

The lists hold every pair within R_i + R_j + skin at the last build and are
rebuilt before any particle has moved 0.49 skin, so no touching pair is ever
missing, and the touching listed neighbours are summed in ascending id as the
per-step search does: every field must agree bit for bit.
"""
import math

import numpy as np
import pytest

from paper_1011_2613_amd import inputs as I
from tests.parity_util import compare, make_pair

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def hex_discs(box, R, rows, seed, v):
    s = 2 * R - 0.2
    per_row = int(box[0] // s)
    pos = []
    for r in range(rows):
        y = R - 0.6 + r * s * math.sqrt(3) / 2
        for k in range(per_row):
            pos.append([(0.5 * s * (r % 2) + 1.0 + k * s) % box[0], y, 0.0])
    pos = np.array(pos)
    return pos, I.random_velocities(2, len(pos), v, seed)


def exact(errs):
    return all(e == 0.0 for e in errs.values())


@pytest.mark.parametrize("every,skin,v", [(100, 1.0, 0.01), (100, 0.15, 0.06), (7, 0.5, 0.02)])
def test_lists_equal_oracle_and_cell_search_2d(gpu_lib, every, skin, v):
    """Packed discs on the lower wall under gravity, crossing the periodic
    seam: lists with a wide skin (rebuilt by age), a narrow skin with fast
    particles (rebuilt by the guard) and a short interval."""
    box, R = (96, 64), 4.0
    pos, vel = hex_discs(box, R, 4, 124, v)
    n = len(pos)
    parts = (pos, vel, np.zeros((n, 3)), np.full(n, R), np.full(n, 10.0), np.zeros(n, np.uint8))
    say("2D lists every %d skin %g v %g, %d discs" % (every, skin, v, n))
    kw = dict(wall_y=True, particle_accel=(0, -1e-4, 0), samples=4, kn=200.0, restitution=0.9, particles=parts)
    orc, gpu = make_pair(gpu_lib, 2, box, 0.7, **kw)
    _, cell = make_pair(gpu_lib, 2, box, 0.7, **kw)
    gpu.set_neighbour_list(every, skin)
    assert gpu.neighbour_list[:2] == (every, skin)
    steps = 0
    for chunk in (1, 9, 40, 150):
        orc.step(chunk)
        gpu.step(chunk)
        cell.step(chunk)
        steps += chunk
        e_orc = compare(orc, gpu)
        e_cell = compare(cell, gpu)
        say("  t=%d vs oracle %s" % (steps, {k: "%.1e" % x for k, x in e_orc.items()}))
        assert exact(e_orc), e_orc
        assert exact(e_cell), e_cell
    builds = gpu.neighbour_list[2]
    say("  %d steps, %d list builds" % (steps, builds))
    assert builds >= 1 + (steps - 1) // every
    if skin < 0.2:
        assert builds > 1 + (steps - 1) // every  # the guard fired before the lists aged


def test_lists_3d_spinning_spheres(gpu_lib):
    """3D spheres with random velocities and spins between walls, lists every
    100 steps with the guard, against the oracle."""
    box, R, n = (40, 36, 24), 3.0, 60
    pos = I.place_particles(3, box, R, n, 77, wall_y=True)
    vel = I.random_velocities(3, n, 0.04, 78)
    om = I.random_velocities(3, n, 3e-3, 79)
    parts = (pos, vel, om, np.full(n, R), np.full(n, 5.0), np.zeros(n, np.uint8))
    say("3D lists, %d spheres" % n)
    orc, gpu = make_pair(gpu_lib, 3, box, 0.65, wall_y=True, particle_accel=(0, -2e-5, 0), samples=4,
                         kn=300.0, restitution=0.8, particles=parts)
    gpu.set_neighbour_list(100, 0.4)
    touched = 0
    for chunk in (1, 30, 70, 100):
        orc.step(chunk)
        gpu.step(chunk)
        errs = compare(orc, gpu)
        touched += int(np.count_nonzero(np.abs(orc.contact_forces()).sum(axis=1)))
        say("  t=%d %s" % (orc.t, {k: "%.1e" % x for k, x in errs.items()}))
        assert exact(errs), errs
    say("  %d list builds, %d particles in contact at the checkpoints" % (gpu.neighbour_list[2], touched))
    assert gpu.neighbour_list[2] >= 2 and touched > 0


def test_mode_switches_keep_the_bits(gpu_lib):
    """Cell list, then lists, then the cell list again on one context: the
    same bits as the cell list throughout."""
    box, R = (96, 64), 4.0
    pos, vel = hex_discs(box, R, 3, 125, 0.02)
    n = len(pos)
    parts = (pos, vel, np.zeros((n, 3)), np.full(n, R), np.full(n, 10.0), np.zeros(n, np.uint8))
    kw = dict(wall_y=True, particle_accel=(0, -1e-4, 0), samples=4, kn=200.0, restitution=0.9, particles=parts)
    orc, gpu = make_pair(gpu_lib, 2, box, 0.7, **kw)
    for mode in ((0, 1.0), (50, 0.6), (0, 1.0), (25, 0.3)):
        gpu.set_neighbour_list(*mode)
        orc.step(40)
        gpu.step(40)
        errs = compare(orc, gpu)
        say("  mode %s t=%d %s" % (mode, orc.t, {k: "%.1e" % x for k, x in errs.items()}))
        assert exact(errs), errs


def test_bad_list_settings_are_rejected(gpu_lib):
    from paper_1011_2613_amd import binding
    box, R = (64, 32), 4.0
    pos, vel = hex_discs(box, R, 1, 126, 0.01)
    n = len(pos)
    parts = (pos, vel, np.zeros((n, 3)), np.full(n, R), np.full(n, 10.0), np.zeros(n, np.uint8))
    _, gpu = make_pair(gpu_lib, 2, box, 0.7, wall_y=True, samples=4, kn=200.0, particles=parts, max_radius=4.0)
    for every, skin in ((-1, 1.0), (10, 0.0), (10, -1.0), (10, float("nan")), (10, 8.5)):
        with pytest.raises(binding.LbmError):
            gpu.set_neighbour_list(every, skin)
    assert gpu.neighbour_list[:2] == (0, 1.0)
