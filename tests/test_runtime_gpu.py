"""Runtime behaviour of the C ABI on the GPU: call order, health flags, state
files that must be rejected, and the suspension-wide sums of lbm_get_stats
against the FP64 oracle."""
import ctypes
import math
import os
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2613_amd import inputs as I
from tests.parity_util import make_pair

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def spheres(box, R, n, seed, speed):
    pos = I.place_particles(3, box, R, n, seed, wall_y=True)
    vel = I.random_velocities(3, n, speed, seed + 1)
    om = I.random_velocities(3, n, 1e-3, seed + 2)
    return pos, vel, om, np.full(n, R), np.full(n, 4.0), np.zeros(n, np.uint8)


def test_step_before_particles_is_a_state_error(gpu_lib):
    say("call order")
    s = gpu_lib.Simulation(3, (16, 12, 10), 0.7, max_particles=1)
    with pytest.raises(gpu_lib.LbmError) as ei:
        s.step(1)
    assert ei.value.code == -6
    s.set_particles()          # a fluid without particles is a valid set
    s.step(3)
    assert s.t == 3


def test_flags_cleared_by_a_new_particle_set(gpu_lib):
    """A slot overflow keeps failing every step until the state is replaced;
    a new particle set clears it and stepping resumes."""
    say("flags cleared")
    R, r = 4.0, 4.3
    c = np.array([12.0, 12.0, 12.0])
    dirs = [(0, 0, 1), (0, 0, -1)] + [(math.cos(a), math.sin(a), 0) for a in
                                     (0.0, 2 * math.pi / 3, 4 * math.pi / 3)]
    pos = np.array([c + r * np.array(d) for d in dirs])
    s = gpu_lib.Simulation(3, (24, 24, 24), 0.7, samples=4, kn=10.0, max_particles=5)
    s.set_particles(pos, radius=np.full(5, R), rho_s=np.full(5, 2.0))
    for _ in range(2):
        with pytest.raises(gpu_lib.LbmError) as ei:
            s.step(1)
        assert ei.value.code == -5
    s.set_particles(pos[:2], radius=np.full(2, R), rho_s=np.full(2, 2.0))
    s.step(4)


def _save_layout(gpu_lib, sim):
    """Byte offsets of the sections of a state file written by lbm_save."""
    cfg = ctypes.sizeof(gpu_lib.lbm_config)
    off = {"t": 8 + cfg, "np": 16 + cfg, "f": 20 + cfg}
    es = {"fp64": 8, "fp32s": 4, "fp16s": 2}["fp64"]
    P = max(sim.np_, 1)
    off["x"] = off["f"] + sim.Q * sim.N * es
    off["R"] = off["x"] + 6 * 3 * P * 8
    off["m"] = off["R"] + P * 8
    off["end"] = off["R"] + 3 * P * 8 + P + 12
    return off


def test_load_rejects_bad_files_and_keeps_the_state(gpu_lib):
    box = (24, 20, 22)
    parts = spheres(box, 3.0, 4, 31, 0.01)
    kw = dict(wall_y=True, fluid_force=(1e-6, 0, 0), particle_accel=(0, -1e-5, 0), samples=4,
              kn=300.0, restitution=0.8, max_particles=4, max_radius=4.0)
    say("state files")
    a = gpu_lib.Simulation(3, box, 0.65, **kw)
    a.set_particles(*parts)
    a.step(6)
    with tempfile.TemporaryDirectory() as d:
        good = os.path.join(d, "good.bin")
        a.save(good)
        raw = open(good, "rb").read()
        off = _save_layout(gpu_lib, a)
        assert off["end"] == len(raw)
        b = gpu_lib.Simulation(3, box, 0.65, **kw)
        b.set_particles(*parts)
        b.step(2)
        f_before, x_before = b.get_f(), b.particles()[0]

        def rejected(blob, code):
            path = os.path.join(d, "bad.bin")
            with open(path, "wb") as fh:
                fh.write(blob)
            with pytest.raises(gpu_lib.LbmError) as ei:
                b.load_state(path)
            assert ei.value.code == code, ei.value
            # nothing changed: same time, populations and particles
            assert b.t == 2
            assert np.array_equal(b.get_f(), f_before)
            assert np.array_equal(b.particles()[0], x_before)

        rejected(raw[: len(raw) // 2], -7)                 # truncated in the populations
        rejected(raw[:-5], -7)                             # truncated in the cell grid
        rejected(raw + b"\0", -7)                          # trailing bytes
        bad = bytearray(raw)
        bad[off["R"]:off["R"] + 8] = np.float64(9.0).tobytes()   # radius above max_radius
        rejected(bytes(bad), -1)
        bad = bytearray(raw)
        bad[off["x"]:off["x"] + 8] = np.float64(-3.0).tobytes()  # centre outside the periodic box
        rejected(bytes(bad), -1)
        bad = bytearray(raw)
        bad[off["m"]:off["m"] + 8] = np.float64(0.0).tobytes()   # zero mass
        rejected(bytes(bad), -1)
        bad = bytearray(raw)
        bad[off["np"]:off["np"] + 4] = np.int32(99).tobytes()    # more particles than reserved
        rejected(bytes(bad), -1)
        # a foreign cell grid in the file is ignored: the grid is rebuilt
        bad = bytearray(raw)
        bad[-12:] = np.array([100000, -3, 7], np.int32).tobytes()
        path = os.path.join(d, "grid.bin")
        with open(path, "wb") as fh:
            fh.write(bytes(bad))
        b.load_state(path)
        assert b.t == 6
        a.step(9)
        b.step(9)
        assert np.array_equal(a.get_f(), b.get_f())
        assert np.array_equal(a.particles()[0], b.particles()[0])


def _expected_stats(orc, dim, counts, S, R, rho_s):
    f = orc.get_f().reshape(orc.Q, -1)
    c, _ = O.velocities(dim)
    rho = f.sum(axis=0)
    j = np.zeros((3, f.shape[1]))
    j[:dim] = c.T @ f
    eps = np.minimum(counts.reshape(-1), S ** dim) / S ** dim
    x, v, _ = orc.particles()
    F, _ = orc.forces()
    m = rho_s * (math.pi * R ** 2 if dim == 2 else 4.0 / 3.0 * math.pi * R ** 3)
    fluid_mass = ((1.0 - eps) * rho).sum()
    uf = ((1.0 - eps) * j).sum(axis=1) / fluid_mass
    up = (m * v).sum(axis=0) / (m * len(v))
    return {"mass": rho.sum(), "fluid_momentum": j.sum(axis=1), "solid_fraction": eps.mean(),
            "fluid_velocity": uf, "particle_momentum": (m * v).sum(axis=0),
            "particle_velocity": up, "mean_particle_velocity": v.mean(axis=0),
            "slip_velocity": uf - up, "mean_drag": F.mean(axis=0)}


@pytest.mark.parametrize("dim", [2, 3])
def test_stats_against_oracle(gpu_lib, dim):
    """lbm_get_stats after K steps equals the same sums formed from the
    oracle's fields, with eps from the oracle's footprint of the last step."""
    if dim == 3:
        box, R, n, S = (36, 30, 28), 3.5, 9, 4
        pos, vel, om, rad, rho, fx = spheres(box, R, n, 41, 0.01)
    else:
        box, R, n, S = (64, 48), 5.0, 8, 8
        pos = I.place_particles(2, box, R, n, 43, wall_y=True)
        vel = I.random_velocities(2, n, 0.01, 44)
        om = np.zeros((n, 3))
        om[:, 2] = 1e-3
        rad, rho, fx = np.full(n, R), np.full(n, 4.0), np.zeros(n, np.uint8)
    say("stats %dD" % dim)
    orc, gpu = make_pair(gpu_lib, dim, box, 0.7, wall_y=True, fluid_force=(2e-6, 0, 0),
                         particle_accel=(0, -1e-5, 0), samples=S, kn=300.0, restitution=0.8,
                         particles=(pos, vel, om, rad, rho, fx))
    st0 = gpu.stats()
    assert st0["t"] == 0 and st0["solid_fraction"] == 0.0   # no footprint before the first step
    K = 30
    orc.step(K - 1)
    gpu.step(K - 1)
    counts = orc.footprint_counts()           # the footprint step K uses
    orc.step(1)
    gpu.step(1)
    st = gpu.stats()
    exp = _expected_stats(orc, dim, counts, S, R, 4.0)
    assert st["t"] == K and st["np"] == n and st["nodes"] == int(np.prod(box))
    for k, e in exp.items():
        e = np.atleast_1d(np.asarray(e, dtype=np.float64))
        g = np.atleast_1d(st[k])[: len(e)]
        scale = max(np.abs(e).max(), 1e-300)
        if k == "fluid_momentum" or k == "particle_momentum":
            # totals with cancellation: scale by the sum of magnitudes
            scale = max(scale, 1e-14 * exp["mass"])
        say("  %s gpu %s oracle %s" % (k, g, e))
        assert np.abs(g - e).max() <= 1e-11 * scale, k
    # the same state gives the same bits every time
    st2 = gpu.stats()
    for k in st:
        assert np.array_equal(np.atleast_1d(st[k]), np.atleast_1d(st2[k]))


def test_stats_shifted_storage_mass(gpu_lib):
    """Shifted storage: the fluid at rest holds mass N (the binary64 rest
    weights sum to 1 within one rounding), no momentum, and a fluid force adds
    momentum rho g per node and step (no particles)."""
    say("stats fp32s")
    box = (40, 24, 18)
    s = gpu_lib.Simulation(3, box, 0.8, storage="fp32s", fluid_force=(1e-5, 0, 0), max_particles=1)
    s.set_particles()
    st = s.stats()
    N = int(np.prod(box))
    assert abs(st["mass"] - N) <= 1e-14 * N and np.all(st["fluid_momentum"] == 0.0)
    s.step(10)
    st = s.stats()
    assert abs(st["mass"] - N) <= 1e-9 * N
    assert abs(st["fluid_momentum"][0] - 10 * 1e-5 * N) <= 1e-4 * 10 * 1e-5 * N
