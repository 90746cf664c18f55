"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

FP64 bar: every field within 1e-12 relative (max |gpu - oracle| / max |oracle|)
after the stated number of steps.  Both sides evaluate every per-node formula
in the same order without fused multiply-add, and the per-particle sums are
compensated, so in practice the fields agree bit for bit; the tests report the
largest error seen.
"""
import math
import os
import tempfile

import numpy as np
import pytest

from paper_1011_2613_amd import inputs as I
from tests.parity_util import compare, make_pair, rel_err, seeded_f

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)


def assert_close(errs, tol=TOL, label=""):
    say(label, {k: "%.2e" % v for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, "%s exceeds %g: %s" % (label, tol, bad)


def c1_particles():
    w = I.workload("C1")
    return w, w.particles()


# ------------------------------------------------------------------ C1 (D2Q9)
def test_c1_one_step_bitwise(gpu_lib):
    w, parts = c1_particles()
    say("C1 one step", w.shape)
    orc, gpu = make_pair(gpu_lib, 2, w.shape, w.tau, fluid_force=w.fluid_force, samples=w.samples,
                         kn=w.kn, restitution=w.restitution, particles=parts)
    orc.step(1)
    gpu.step(1)
    assert np.array_equal(gpu.get_f(), orc.get_f())
    assert np.array_equal(gpu.q(), orc.q()[:2])
    F0, T0 = orc.forces()
    F1, T1 = gpu.forces()
    assert np.array_equal(F1, F0) and np.array_equal(T1, T0)


def test_c1_full_run(gpu_lib):
    """C1: D2Q9 256x256, tau 0.6, fluid force 1e-6, 16 discs R=6, 1000 steps."""
    w, parts = c1_particles()
    say("C1 full", w.shape, w.steps)
    orc, gpu = make_pair(gpu_lib, 2, w.shape, w.tau, fluid_force=w.fluid_force, samples=w.samples,
                         kn=w.kn, restitution=w.restitution, particles=parts)
    for chunk in (1, 99, 400, 500):
        orc.step(chunk)
        gpu.step(chunk)
        errs = compare(orc, gpu)
        assert_close(errs, label="C1 t=%d" % orc.t)
    # the discs have been dragged along +x by the flow
    x0 = parts[0]
    x1, _, _ = gpu.particles()
    assert np.all(((x1[:, 0] - x0[:, 0]) % 256.0) > 0)


# ------------------------------------------------------- D3Q19 with walls
def spheres(box, R, n, seed, v0, wall_y=True, rho=5.0):
    pos = I.place_particles(3, box, R, n, seed, wall_y=wall_y)
    vel = I.random_velocities(3, n, v0, seed + 1)
    om = I.random_velocities(3, n, 1e-3, seed + 2)
    return pos, vel, om, np.full(n, R), np.full(n, rho), np.zeros(n, np.uint8)


def test_d3q19_walls_moving_spheres(gpu_lib):
    box = (40, 36, 24)
    parts = spheres(box, 4.0, 8, 31, 0.01)
    say("D3Q19 walls", box)
    orc, gpu = make_pair(gpu_lib, 3, box, 0.62, wall_y=True, fluid_force=(2e-6, 0, 1e-6),
                         particle_accel=(0, -2e-5, 0), samples=4, kn=500.0, restitution=0.8,
                         particles=parts)
    for chunk in (1, 60, 140):
        orc.step(chunk)
        gpu.step(chunk)
        assert_close(compare(orc, gpu), label="D3Q19 walls t=%d" % orc.t)


@pytest.mark.parametrize("dim,shape,wall", [(2, (100, 37), True), (2, (67, 70), False),
                                            (3, (70, 19, 13), True), (3, (33, 30, 29), False)])
def test_ragged_random_state(gpu_lib, dim, shape, wall):
    """Seeded random populations on ragged lattices (not multiples of the
    wavefront), with particles, both boundary kinds."""
    N = int(np.prod(shape))
    f0 = seeded_f(dim, N, 0.02, 77 + N)
    R = 3.0
    n = 4
    pos = I.place_particles(dim, shape, R, n, 5 + N, wall_y=wall)
    vel = I.random_velocities(dim, n, 0.01, 9)
    om = np.zeros((n, 3)); om[:, 2] = 2e-3
    if dim == 3:
        om = I.random_velocities(3, n, 2e-3, 11)
    parts = (pos, vel, om, np.full(n, R), np.full(n, 3.0), np.array([0, 1, 0, 0], np.uint8))
    say("ragged", dim, shape, wall)
    orc, gpu = make_pair(gpu_lib, dim, shape, 0.55, wall_y=wall, fluid_force=(1e-5, -3e-6, 2e-6),
                         particle_accel=(0, -1e-5, 0), samples=3, kn=300.0, restitution=0.7,
                         particles=parts, f0=f0)
    assert_close(compare(orc, gpu), label="ragged t=0")
    for chunk in (1, 30):
        orc.step(chunk)
        gpu.step(chunk)
        assert_close(compare(orc, gpu), label="ragged t=%d" % orc.t)


def test_large_mixed_particles_many_chunks(gpu_lib):
    """Mixed radii whose bounding boxes exceed the footprint kernel's chunk
    of 1024 nodes (3D R = 6.5: 15^3 = 3375 nodes in four chunks, the last
    ragged; 2D R = 20: 42^2 = 1764 nodes in two), so list positions carry
    across chunks; moving and rotating, walls in y."""
    pos = np.array([[12.0, 12.0, 10.0], [34.0, 14.0, 24.0], [14.0, 28.0, 26.0], [36.0, 30.0, 8.0]])
    rad = np.array([6.5, 6.0, 5.2, 3.0])
    vel = I.random_velocities(3, 4, 0.01, 61)
    om = I.random_velocities(3, 4, 2e-3, 62)
    parts = (pos, vel, om, rad, np.full(4, 4.0), np.zeros(4, np.uint8))
    box = (48, 40, 36)
    say("large spheres", box)
    orc, gpu = make_pair(gpu_lib, 3, box, 0.6, wall_y=True, fluid_force=(2e-6, 0, 1e-6),
                         particle_accel=(0, -1e-5, 0), samples=4, kn=400.0, restitution=0.8,
                         particles=parts, max_radius=6.5)
    for chunk in (1, 25):
        orc.step(chunk)
        gpu.step(chunk)
        assert_close(compare(orc, gpu), label="large spheres t=%d" % orc.t)
    pos2 = np.array([[30.0, 30.0, 0.0], [75.0, 50.0, 0.0], [70.0, 15.0, 0.0]])
    rad2 = np.array([20.0, 9.5, 14.0])
    vel2 = I.random_velocities(2, 3, 0.01, 63)
    om2 = np.zeros((3, 3)); om2[:, 2] = [1e-3, -2e-3, 5e-4]
    parts2 = (pos2, vel2, om2, rad2, np.full(3, 3.0), np.zeros(3, np.uint8))
    box2 = (96, 80)
    say("large discs", box2)
    orc, gpu = make_pair(gpu_lib, 2, box2, 0.7, wall_y=True, fluid_force=(1e-6, 0, 0),
                         particle_accel=(0, -1e-5, 0), samples=5, kn=400.0, restitution=0.8,
                         particles=parts2, max_radius=20.0)
    for chunk in (1, 40):
        orc.step(chunk)
        gpu.step(chunk)
        assert_close(compare(orc, gpu), label="large discs t=%d" % orc.t)


@pytest.mark.parametrize("dim", [2, 3])
def test_table_lookup_eps_parity(gpu_lib, dim):
    """The paper's table-lookup solid fraction (Eq. 6): the library's table
    (built on the host) and lookup (in the footprint kernel) against the
    oracle's own, moving particles, walls in y, every field compared."""
    if dim == 3:
        box = (40, 36, 24)
        parts = spheres(box, 4.0, 8, 71, 0.01)
        kw = dict(samples=4, fluid_force=(2e-6, 0, 1e-6))
    else:
        box = (96, 64)
        pos = I.place_particles(2, box, 6.0, 10, 72, wall_y=True)
        vel = I.random_velocities(2, 10, 0.01, 73)
        om = np.zeros((10, 3)); om[:, 2] = 1e-3
        parts = (pos, vel, om, np.full(10, 6.0), np.full(10, 3.0), np.zeros(10, np.uint8))
        kw = dict(samples=8, fluid_force=(2e-6, 0, 0))
    say("table eps", dim, box)
    orc, gpu = make_pair(gpu_lib, dim, box, 0.62, wall_y=True, particle_accel=(0, -2e-5, 0), kn=500.0,
                         restitution=0.8, particles=parts, eps="table", **kw)
    for chunk in (1, 40):
        orc.step(chunk)
        gpu.step(chunk)
        assert_close(compare(orc, gpu), label="table eps %dD t=%d" % (dim, orc.t))
    # a second particle radius is refused in table mode
    pos2 = np.array(parts[0][:2]); rad2 = np.array([parts[3][0], parts[3][0] + 1.0])
    with pytest.raises(gpu_lib.LbmError):
        gpu.set_particles(pos2, radius=rad2, rho_s=np.ones(2))


def hex_pack(box, R, rows, gap=-0.2, y0=None, seed=0, v=0.01):
    """Discs in a hexagonal packing resting on the lower wall, neighbours
    overlapping by -gap, with seeded random velocities."""
    s = 2 * R + gap
    per_row = int(box[0] // s)
    pos = []
    for r in range(rows):
        y = (R - 0.6 if y0 is None else y0) + r * s * math.sqrt(3) / 2
        for k in range(per_row):
            pos.append([(0.5 * s * (r % 2) + 1.0 + k * s) % box[0], y, 0.0])
    pos = np.array(pos)
    n = len(pos)
    vel = I.random_velocities(2, n, v, seed)
    return pos, vel


def test_dense_dem_contacts(gpu_lib):
    """Discs packed in contact on the lower wall, gravity: pair contacts, the
    periodic seam, the wall and the cell list must reproduce the oracle's
    all-pairs search step by step."""
    box = (96, 64)
    R = 4.0
    pos, vel = hex_pack(box, R, 4, seed=124)
    n = len(pos)
    parts = (pos, vel, np.zeros((n, 3)), np.full(n, R), np.full(n, 10.0), np.zeros(n, np.uint8))
    say("dense DEM", box, n)
    orc, gpu = make_pair(gpu_lib, 2, box, 0.7, wall_y=True, particle_accel=(0, -1e-4, 0),
                         samples=4, kn=200.0, restitution=0.9, particles=parts)
    contacts = []
    for chunk in (1, 9, 40, 150):
        orc.step(chunk)
        gpu.step(chunk)
        contacts.append(int(np.count_nonzero(np.abs(orc.contact_forces()).sum(axis=1))))
        assert_close(compare(orc, gpu), label="dense DEM t=%d contacts %d" % (orc.t, contacts[-1]))
    assert contacts[0] == n and min(contacts) >= 5


def test_pure_fluid_no_particles(gpu_lib):
    for dim, shape in ((2, (64, 24)), (3, (20, 16, 12))):
        say("pure fluid", dim, shape)
        f0 = seeded_f(dim, int(np.prod(shape)), 0.01, 3)
        orc, gpu = make_pair(gpu_lib, dim, shape, 0.8, wall_y=True, fluid_force=(1e-5, 0, 0), f0=f0)
        orc.step(50)
        gpu.step(50)
        assert_close(compare(orc, gpu), label="fluid %dD" % dim)


# ----------------------------------------------------------- runtime paths
def test_graph_and_eager_agree_bitwise(gpu_lib):
    """Graph replay (timing off) and one-by-one launches (every phase timed,
    or the lattice phase only) give the same state bit for bit; two runs are
    identical (no races)."""
    w, parts = c1_particles()
    say("graph vs eager")
    sims = []
    for timing, lat_only in ((False, False), (True, False), (False, False), (True, True)):
        s = gpu_lib.Simulation(2, w.shape, w.tau, fluid_force=w.fluid_force, samples=w.samples,
                               kn=w.kn, restitution=w.restitution, max_particles=16)
        s.set_particles(*parts)
        s.set_timing(timing, lattice_only=lat_only)
        s.step(37)
        sims.append(s)
    f = [s.get_f() for s in sims]
    x = [s.particles()[0] for s in sims]
    for k in (1, 2, 3):
        assert np.array_equal(f[0], f[k]) and np.array_equal(x[0], x[k])
    t = sims[1].get_timing()
    assert t["lattice"][1] == 37 and t["lattice"][0] > 0
    assert t["footprint"][1] == 37 and t["force"][1] == 37 and t["dem"][1] == 37
    t = sims[3].get_timing()   # lattice-only mode: no other phase is timed
    assert t["lattice"][1] == 37 and t["lattice"][0] > 0
    assert all(n == 0 for k, (ms, n) in t.items() if k != "lattice")


@pytest.mark.parametrize("storage", ["fp64", "fp32s", "fp16s"])
def test_lattice_block_widths_bitwise(gpu_lib, storage):
    """The lattice kernel's launch shape changes nothing but the launch:
    every width (the last workgroup of a row overhanging it by up to 170
    threads) in linear and in XCD order, and with caps of workgroups per CU, (grids of 1 x 39 x 23 up to
    5 x 47 x 1 workgroups, counts of 1, 2, 3, 5 and 6 mod 8 among them, so
    both branches of the renumbering run) gives the state of
    the default launch bit for bit, in 3D with walls and moving spheres and in
    2D with rows wider than one workgroup."""
    cases = [(3, (150, 39, 23), spheres((150, 39, 23), 4.0, 10, 51, 0.01)),
             (2, (300, 47, 1), None)]
    for dim, box, parts in cases:
        shape = box if dim == 3 else box[:2]
        say("lattice widths", storage, shape)
        kw = dict(storage=storage, wall_y=True, fluid_force=(2e-6, 0, 0), particle_accel=(0, -2e-5, 0),
                  samples=4, kn=500.0, restitution=0.8, max_particles=10)
        f0 = seeded_f(dim, int(np.prod(shape)), 0.02, 7)
        ref = None
        shapes = [(0, "linear", 0)] + [(w, o, 0) for o in ("linear", "xcd") for w in (64, 128, 192, 256)]
        shapes += [(64, "linear", 3), (256, "xcd", 4), (192, "xcd", 8)]
        for width, order, cap in shapes:
            s = gpu_lib.Simulation(dim, shape, 0.62, **kw)
            s.set_f(f0)
            s.set_particles(*(parts if parts is not None else ()))
            s.set_lattice_block(width, order, cap)
            assert s.lattice_block == (width or (192 if box[0] == 150 else 256), order, cap)
            s.step(23)
            got = (s.get_f(), s.particles()[0] if parts is not None else None,
                   s.forces()[0] if parts is not None else None)
            s.close()
            if ref is None:
                ref = got
                continue
            for a, b in zip(got, ref):
                assert a is None or np.array_equal(a, b), "shape %d %s %d differs" % (width, order, cap)


@pytest.mark.parametrize("order", ["linear", "xcd"])
def test_lattice_block_width_fp64_parity(gpu_lib, order):
    """A non-default launch shape against the oracle directly (FP64 bar)."""
    box = (150, 21, 13)
    parts = spheres(box, 3.0, 6, 61, 0.01)
    say("width 64 %s vs oracle" % order)
    orc, gpu = make_pair(gpu_lib, 3, box, 0.7, wall_y=True, fluid_force=(1e-6, 0, 0),
                         particle_accel=(0, -1e-5, 0), samples=4, kn=400.0, restitution=0.9,
                         particles=parts)
    gpu.set_lattice_block(64, order, 3)
    orc.step(6)
    gpu.step(6)
    assert_close(compare(orc, gpu), label="width 64 %s t=6" % order)


def test_lattice_block_autotune(gpu_lib):
    """The autotuner advances the state by 48 (steps + 1) real steps, keeps
    one of the 24 launch shapes, restores the timing mode with cleared
    counters, and the tuned run continues bit for bit like an untuned one."""
    box = (96, 30, 20)
    parts = spheres(box, 4.0, 5, 71, 0.01)
    say("lattice width autotune")
    kw = dict(storage="fp32s", wall_y=True, fluid_force=(1e-6, 0, 0), particle_accel=(0, -1e-5, 0),
              samples=4, kn=500.0, restitution=0.9, max_particles=5)
    a = gpu_lib.Simulation(3, box, 0.65, **kw)
    a.set_particles(*parts)
    a.set_timing(True, lattice_only=True)
    best, ms = a.autotune_lattice_block(steps=3)
    assert a.t == 48 * 4
    assert best[0] in (64, 128, 192, 256) and best[1] in ("linear", "xcd") and best[2] in (0, 4, 3)
    assert a.lattice_block == best
    assert len(ms) == 24 and best in ms
    assert all(math.isfinite(v) and v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    t = a.get_timing()
    assert all(n == 0 for _, n in t.values())   # counters cleared, mode kept
    a.step(5)
    assert a.get_timing()["lattice"][1] == 5 * a.pipeline  # one launch per slab
    a.set_timing(False)
    a.step(6)
    b = gpu_lib.Simulation(3, box, 0.65, **kw)
    b.set_particles(*parts)
    b.step(48 * 4 + 11)
    assert np.array_equal(a.get_f(), b.get_f())
    assert np.array_equal(a.particles()[0], b.particles()[0])
    with pytest.raises(gpu_lib.LbmError):
        a.set_lattice_block(96)
    with pytest.raises(ValueError):
        a.set_lattice_block(64, "spiral")
    for cap in (1, 2, 9):
        with pytest.raises(gpu_lib.LbmError):
            a.set_lattice_block(64, "linear", cap)
    with pytest.raises(gpu_lib.LbmError):
        a.autotune_lattice_block(steps=0)
    assert a.lattice_block == best


def test_save_load_resume_bitwise(gpu_lib):
    box = (40, 36, 24)
    parts = spheres(box, 4.0, 6, 41, 0.01)
    say("save/load")
    kw = dict(storage="fp64", wall_y=True, fluid_force=(1e-6, 0, 0), particle_accel=(0, -1e-5, 0),
              samples=4, kn=500.0, restitution=0.8, max_particles=6)
    a = gpu_lib.Simulation(3, box, 0.6, **kw)
    a.set_particles(*parts)
    a.step(40)
    b = gpu_lib.Simulation(3, box, 0.6, **kw)
    b.set_particles(*parts)
    b.step(20)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "state.bin")
        b.save(p)
        c = gpu_lib.Simulation(3, box, 0.6, **kw)
        c.load_state(p)
    c.step(20)
    assert c.t == 40
    assert np.array_equal(a.get_f(), c.get_f())
    assert np.array_equal(a.particles()[0], c.particles()[0])


def test_slot_overflow_is_reported(gpu_lib):
    """Five spheres around one node (triangular bipyramid, overlaps below half
    a radius): the node has more owners than the library keeps."""
    R, r = 4.0, 4.3
    c = np.array([12.0, 12.0, 12.0])
    dirs = [(0, 0, 1), (0, 0, -1)] + [(math.cos(a), math.sin(a), 0) for a in
                                     (0.0, 2 * math.pi / 3, 4 * math.pi / 3)]
    pos = np.array([c + r * np.array(d) for d in dirs])
    say("slot overflow")
    s = gpu_lib.Simulation(3, (24, 24, 24), 0.7, samples=4, kn=10.0, max_particles=5)
    s.set_particles(pos, radius=np.full(5, R), rho_s=np.full(5, 2.0))
    with pytest.raises(gpu_lib.LbmError) as ei:
        s.step(1)
    assert ei.value.code == -5


@pytest.mark.parametrize("n_far", [0, 16384])
def test_contact_overflow_is_reported(gpu_lib, n_far):
    """A disc of radius 12 ringed by 36 discs of radius 1, each overlapping it
    by 0.3 (and not each other): 36 contacts, more than the library keeps.
    Without other discs the contacts run one wavefront per disc; 16 384 more
    discs far away (a grid of pitch 6.5, so no DEM cell of edge >= 24 holds
    more than 16) switch them to one thread per disc.  Both report the
    overflow, and nothing else overflows first (at most two owners per node,
    at most ten discs per cell around the ring)."""
    L = 1024
    R, r, ring = 12.0, 1.0, 12.7
    c = np.array([928.0, 928.0])
    ang = 2 * np.pi * np.arange(36) / 36
    small = c + ring * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    assert 2 * np.pi * ring / 36 > 2 * r  # ring discs do not touch each other
    k = int(np.sqrt(n_far))
    g = (np.arange(k) * 6.5 + 3.0) if k else np.zeros(0)
    far = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    assert far.shape[0] == n_far and (n_far == 0 or far.max() + 1.0 < c[0] - ring - 2.0)
    pos2 = np.concatenate([c[None, :], small, far])
    n = len(pos2)
    pos = np.concatenate([pos2, np.zeros((n, 1))], axis=1)
    rad = np.concatenate([[R], np.full(36, r), np.full(n_far, r)])
    say("contact overflow", n, "discs")
    s = gpu_lib.Simulation(2, (L, L), 0.8, samples=4, kn=10.0, max_particles=n, max_radius=R)
    s.set_particles(pos, radius=rad, rho_s=np.full(n, 2.0))
    with pytest.raises(gpu_lib.LbmError) as ei:
        s.step(1)
    assert ei.value.code == -9


def test_runaway_particle_is_reported(gpu_lib):
    """A particle that moves more than a box length in one step leaves the
    box after the single periodic wrap of the integrator: the next footprint
    gives it no nodes and the step reports LBM_E_NONFINITE."""
    say("runaway particle")
    s = gpu_lib.Simulation(3, (24, 24, 24), 0.8, samples=2, kn=0.0, max_particles=1)
    s.set_particles([[12.0, 12.0, 12.0]], vel=[[60.0, 0.0, 0.0]], radius=[3.0], rho_s=[1000.0])
    with pytest.raises(gpu_lib.LbmError) as ei:
        s.step(2)
    assert ei.value.code == -4


def test_invalid_inputs_rejected(gpu_lib):
    say("invalid inputs")
    with pytest.raises(gpu_lib.LbmError):
        gpu_lib.Simulation(2, (16, 16), 0.5)
    s = gpu_lib.Simulation(2, (32, 32), 0.7, max_particles=2)
    with pytest.raises(gpu_lib.LbmError):  # overlap of more than half a radius
        s.set_particles([[10, 10, 0], [12, 10, 0]], radius=[3, 3], rho_s=[1, 1])
    with pytest.raises(gpu_lib.LbmError):  # more particles than reserved
        s.set_particles(np.zeros((3, 3)) + 5, radius=[1, 1, 1], rho_s=[1, 1, 1])
    with pytest.raises(gpu_lib.LbmError):  # wider than the periodic box
        s.set_particles([[10, 10, 0]], radius=[20], rho_s=[1])


# ------------------------------------------------- full-size workloads, 5 steps
@pytest.mark.parametrize("name,steps", [("C2", 5), ("C3", 5), ("C2dense", 5), ("C3dense", 5)])
def test_full_size_first_steps(gpu_lib, name, steps):
    """The full C2 / C3 workloads and their dense variants (40,000 discs at
    solid fraction 0.19, 16,000 spheres at 0.15) from the seeded initial
    state, 5 steps, every field compared, the populations of every node
    included.  (The long-run tests follow C2 and C3 over their stated step
    counts.)"""
    w = I.workload(name)
    parts = w.particles()
    say("full size", name, w.shape, w.count, "particles", steps, "steps")
    orc, gpu = make_pair(gpu_lib, w.dim, w.shape, w.tau, wall_y=w.wall_y,
                         fluid_force=w.fluid_force, particle_accel=w.particle_accel,
                         samples=w.samples, kn=w.kn, restitution=w.restitution, particles=parts)
    orc.step(steps)
    gpu.step(steps)
    errs = compare(orc, gpu, with_f=True)
    assert_close(errs, label=name)
    # mass is conserved to rounding at full size
    rho, _ = gpu.macro()
    assert abs(rho.sum() - w.nodes) / w.nodes < 1e-13


# ------------------------------------- the paper's 3D suspension at full size
@pytest.mark.parametrize("name,E,steps,nsample", [("P3", 64, 5, 6), ("P2", 96, 5, 8)])
def test_paper_scale_sampled(gpu_lib, name, E, steps, nsample):
    """The paper's suspensions at full size on one GPU, FP64: 3D 512x2016x512
    D3Q19 with 129,024 spheres (about 188 GB of device memory) and 2D
    15360x61440 D2Q9 with 1,166,400 discs (about 184 GB), checked after one
    step and after `steps` steps from the seeded initial state.

    The oracle cannot hold these lattices, but the method is local: after k
    steps a particle's force, contact force and state depend only on the
    initial fluid (uniform) and on the particles within about k + 3R of it.
    Each sampled particle is checked against the oracle run on a periodic
    sub-box of edge E centred on it, holding every particle whose nearest image
    lies within E/2 - R - 1 of it on every axis, shifted by whole lattice
    units: a particle left out covers nodes at least E/2 - 2R - 2 away, and
    its influence travels one node per step, so the sampled particle's nodes
    (within R + 1) stay exact while k < E/2 - 3R - 3.

    The shift is exact for the initial positions, so after one step every
    field meets the bar relative to its own size.  Later positions x + v are
    rounded at the magnitude of the coordinate, which differs between the full
    box (up to 2016 or 61440) and the sub-box (below E): the two runs'
    positions then differ by about one unit in the last place of the larger
    coordinate (P2: k ulp(61440) = k 7.3e-12 after k steps, about 1e-11 of R
    at k = 5).  The torque sum over the footprint nearly cancels, so after k
    steps the torque is measured against the torque scale R |F| and the
    angular velocity against k R |F| / I (I the moment of inertia), with the
    bar raised to 1e-11 of those scales, the size of that lever-arm change;
    the other fields keep the 1e-12 bar against their own size.  The total
    mass of the full lattice is checked from the library's statistics."""
    import torch
    from oracle import oracle as O
    w = I.workload(name)
    assert steps < E // 2 - 3 * w.radius - 3
    say("paper scale %s: %s, %d particles, %d steps, sub-box %d (placing particles)"
        % (name, w.shape, w.count, steps, E))
    parts = w.particles()
    pos = parts[0]
    D = w.dim
    L = np.array(list(w.shape) + [1] * (3 - D), dtype=np.float64)
    torch.cuda.empty_cache()
    gpu = gpu_lib.Simulation(D, w.shape, w.tau, storage="fp64", wall_y=False,
                             fluid_force=w.fluid_force, particle_accel=w.particle_accel,
                             samples=w.samples, kn=w.kn, restitution=w.restitution,
                             max_particles=w.count, max_radius=w.radius)
    gpu.set_particles(*parts)
    snap = {}
    for t in (1, steps):
        gpu.step(t - gpu.t)
        snap[t] = (gpu.forces(), gpu.contact_forces(), gpu.particles())
    mass = gpu.stats()["mass"]
    gpu.close()
    del gpu
    torch.cuda.empty_cache()
    say("  mass error %.2e" % (abs(mass - w.nodes) / w.nodes))
    assert abs(mass - w.nodes) / w.nodes < 1e-13
    R = w.radius
    m = w.rho_ratio * (math.pi * R ** 2 if D == 2 else 4.0 / 3.0 * math.pi * R ** 3)
    inertia = (0.5 if D == 2 else 0.4) * m * R ** 2
    rng = np.random.default_rng(5)
    sub_shape = (E,) * D
    for p in sorted(rng.choice(w.count, nsample, replace=False)):
        c = pos[p]
        org = np.floor(c) - E // 2
        org[D:] = 0.0
        img = pos - L * np.round((pos - c) / L)
        sel = np.flatnonzero(np.all(np.abs(img - c)[:, :D] < E // 2 - R - 1, axis=1))
        sub = img[sel] - org               # exact for particles that needed no wrap
        k = int(np.flatnonzero(sel == p)[0])
        orc = O.OracleSim(D, sub_shape, w.tau, wall_y=False, fluid_force=w.fluid_force,
                          particle_accel=w.particle_accel, samples=w.samples, kn=w.kn,
                          restitution=w.restitution)
        orc.set_particles(sub, parts[1][sel], parts[2][sel], parts[3][sel], parts[4][sel], parts[5][sel])
        for t in (1, steps):
            orc.step(t - orc.t)
            (F1, T1), Fc1, (x1, v1, w1) = snap[t]
            F0, T0 = orc.forces()
            x0, v0, w0 = orc.particles()
            xg = x1[p] - org
            xg -= L * np.round((xg - x0[k]) / L)
            errs = {"F": rel_err(F1[p], F0[k]), "Fc": rel_err(Fc1[p], orc.contact_forces()[k]),
                    "v": rel_err(v1[p], v0[k]), "x": rel_err(xg, x0[k])}
            if t == 1:
                errs["T"] = rel_err(T1[p], T0[k])
                errs["w"] = rel_err(w1[p], w0[k])
            else:
                fmag = float(np.abs(F0[k]).max())
                errs["T/(R|F|)"] = float(np.abs(T1[p] - T0[k]).max() / max(R * fmag, np.abs(T0[k]).max()))
                errs["w/(kR|F|/I)"] = float(np.abs(w1[p] - w0[k]).max()
                                            / max(t * R * fmag / inertia, np.abs(w0[k]).max()))
            label = "%s particle %d (%d in sub-box), step %d" % (name, p, len(sel), t)
            if t > 1:
                rot = {key: errs.pop(key) for key in ("T/(R|F|)", "w/(kR|F|/I)")}
                assert_close(rot, tol=1e-11, label=label + " rotation")
            assert_close(errs, label=label)
        orc.close()
