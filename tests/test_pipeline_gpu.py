"""The slab pipeline (lbm_set_pipeline) against the plain step and the oracle.

With walls in y the lattice update of a step runs slab by slab and each
particle group's force sums, integration and next footprint run on a second
stream as soon as its slabs are done.  Every node and particle runs the same
arithmetic as in the plain step, so every field must agree bit for bit with
the plain step (graph replay) and with the oracle, with and without phase
timing, across mode switches, and in what the getters read
(the statistics and q use the last completed step's footprint, which the
pipeline keeps beside the one it paints ahead).
"""
import numpy as np
import pytest

from paper_1011_2613_amd import inputs as I
from tests.parity_util import compare, make_pair

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def exact(errs):
    return all(e == 0.0 for e in errs.values())


def spheres(box, R, n, seed, v0):
    pos = I.place_particles(3, box, R, n, seed, wall_y=True)
    vel = I.random_velocities(3, n, v0, seed + 1)
    om = I.random_velocities(3, n, 2e-3, seed + 2)
    return pos, vel, om, np.full(n, R), np.full(n, 6.0), np.zeros(n, np.uint8)


KW3 = dict(wall_y=True, fluid_force=(2e-6, 0, 1e-6), particle_accel=(0, -3e-5, 0), samples=4, kn=400.0,
           restitution=0.8)


@pytest.mark.parametrize("slabs", [2, 3, 4, 8])
def test_pipeline_equals_plain_and_oracle_3d(gpu_lib, slabs):
    box = (40, 8 * 13 + 6, 24)
    parts = spheres(box, 4.0, 24, 91, 0.02)
    say("3D pipeline, %d slabs requested, box %s" % (slabs, box))
    orc, pipe = make_pair(gpu_lib, 3, box, 0.62, particles=parts, **KW3)
    _, plain = make_pair(gpu_lib, 3, box, 0.62, particles=parts, **KW3)
    pipe.set_pipeline(slabs)
    plain.set_pipeline(1)
    assert pipe.pipeline == slabs and plain.pipeline == 1
    for chunk in (1, 7, 16, 40, 3):
        orc.step(chunk)
        pipe.step(chunk)
        plain.step(chunk)
        e_orc, e_plain = compare(orc, pipe), compare(plain, pipe)
        say("  t=%d vs oracle %s" % (orc.t, {k: "%.1e" % v for k, v in e_orc.items()}))
        assert exact(e_orc), e_orc
        assert exact(e_plain), e_plain
    # getters of the last completed step
    sp, sq = pipe.stats(), plain.stats()
    for k in sp:
        assert np.array_equal(np.asarray(sp[k]), np.asarray(sq[k])), k
    assert np.array_equal(pipe.q(), plain.q())


def test_pipeline_2d_dense_discs_and_timing_mode(gpu_lib):
    """Discs packed on the lower wall with contacts, 4 slabs, with every phase
    timed and without, against the plain step."""
    box, R = (96, 160), 4.0
    s = 2 * R - 0.2  # three hexagonal rows on the lower wall, neighbours overlapping
    hexp = [[(0.5 * s * (r % 2) + 1.0 + k * s) % box[0], R - 0.6 + r * s * np.sqrt(3) / 2, 0.0]
            for r in range(3) for k in range(int(box[0] // s))]
    upper = I.place_particles(2, (96, 110), R, 40, 93) + np.array([0.0, 40.0, 0.0])
    pos = np.concatenate([np.array(hexp), upper])
    n = len(pos)
    vel = I.random_velocities(2, n, 0.03, 94)
    parts = (pos, vel, np.zeros((n, 3)), np.full(n, R), np.full(n, 10.0), np.zeros(n, np.uint8))
    kw = dict(wall_y=True, particle_accel=(0, -1e-4, 0), samples=8, kn=200.0, restitution=0.9, particles=parts)
    say("2D pipeline, box %s" % (box,))
    orc, graph = make_pair(gpu_lib, 2, box, 0.7, **kw)
    _, timed = make_pair(gpu_lib, 2, box, 0.7, **kw)
    _, plain = make_pair(gpu_lib, 2, box, 0.7, **kw)
    assert graph.pipeline == 1  # off by default
    graph.set_pipeline(0)
    timed.set_pipeline(0)
    assert graph.pipeline == 4 and timed.pipeline == 4  # automatic
    timed.set_timing(True)
    contacts = []
    for chunk in (1, 24, 75):
        for s in (orc, graph, timed, plain):
            s.step(chunk)
        contacts.append(int(np.count_nonzero(np.abs(orc.contact_forces()).sum(axis=1))))
        for other in (timed, plain):
            errs = compare(other, graph)
            assert exact(errs), errs
        e = compare(orc, graph)
        say("  t=%d vs oracle %s" % (orc.t, {k: "%.1e" % v for k, v in e.items()}))
        assert exact(e), e
    t = timed.get_timing()
    assert t["lattice"][1] == 4 * 100 and t["force"][1] == 4 * 100 and t["footprint"][1] == 4 * 100
    say("  particles in contact at t = 1, 25, 100: %s" % contacts)
    assert contacts[0] > 0


def test_pipeline_mode_switches(gpu_lib):
    """Pipeline on, off, on with another slab count, automatic, and a new
    particle set in between: the same bits as the plain step throughout."""
    box = (40, 70, 24)
    parts = spheres(box, 4.0, 14, 95, 0.02)
    orc, gpu = make_pair(gpu_lib, 3, box, 0.62, particles=parts, **KW3)
    for slabs in (4, 1, 3, 0, 2, 1):
        gpu.set_pipeline(slabs)
        orc.step(11)
        gpu.step(11)
        errs = compare(orc, gpu)
        say("  slabs %d (in use %d) t=%d %s" % (slabs, gpu.pipeline, orc.t, {k: "%.1e" % v for k, v in errs.items()}))
        assert exact(errs), errs
    parts2 = spheres(box, 3.0, 10, 96, 0.02)
    orc.set_particles(*parts2)
    gpu.set_pipeline(0)
    gpu.set_particles(*parts2)
    assert gpu.pipeline == 4
    orc.step(13)
    gpu.step(13)
    errs = compare(orc, gpu)
    assert exact(errs), errs


def test_pipeline_slab_count_is_limited(gpu_lib):
    """Slabs stay at least 2 R_max + 5 rows high; no walls in y or no
    particles: the plain step; requests beyond 8 are refused."""
    from paper_1011_2613_amd import binding
    box = (40, 40, 24)
    parts = spheres(box, 4.0, 4, 97, 0.0)
    _, gpu = make_pair(gpu_lib, 3, box, 0.62, particles=parts, **KW3)
    gpu.set_pipeline(8)
    assert gpu.pipeline == 40 // 13
    with pytest.raises(binding.LbmError):
        gpu.set_pipeline(9)
    _, per = make_pair(gpu_lib, 3, box, 0.62, particles=spheres(box, 4.0, 4, 98, 0.0),
                       fluid_force=(1e-6, 0, 0), samples=4)
    per.set_pipeline(0)
    assert per.pipeline == 1
    _, empty = make_pair(gpu_lib, 3, box, 0.62, wall_y=True)
    empty.set_pipeline(4)
    assert empty.pipeline == 1


def test_pipeline_flags_a_particle_faster_than_a_node(gpu_lib):
    """A particle moving down by 1.5 nodes in a step: its next footprint still
    lies in slabs its group has finished (the guard's margin covers the
    downward side), and the step reports LBM_E_NONFINITE."""
    from paper_1011_2613_amd import binding
    box = (40, 70, 24)
    pos = np.array([[20.0, 40.0, 12.0], [8.0, 10.0, 6.0], [30.0, 10.0, 18.0], [8.0, 60.0, 6.0],
                    [30.0, 60.0, 18.0], [20.0, 22.0, 12.0]])
    vel = np.zeros((6, 3))
    vel[0] = [0.0, -1.5, 0.0]
    parts = (pos, vel, np.zeros((6, 3)), np.full(6, 4.0), np.full(6, 6.0), np.zeros(6, np.uint8))
    _, gpu = make_pair(gpu_lib, 3, box, 0.62, particles=parts, **KW3)
    gpu.set_pipeline(0)
    assert gpu.pipeline == 4
    with pytest.raises(binding.LbmError) as ei:
        gpu.step(1)
    assert ei.value.code == -4
