"""Batched drag ensemble (many periodic boxes, fixed spheres, shifted FP32).

- A box advanced inside a batch gives the same bits as the same box advanced
  alone through lbm_step (shifted FP32 storage, particles fixed at rest).
- The persistent launch and one launch per step give the same bits.
- Drag against the FP64 oracle: mean relative error <= 1e-3 (the shifted-FP32
  target).
"""
import numpy as np
import pytest

from paper_1011_2613_amd import inputs as I
from tests.parity_util import rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def make_boxes():
    boxes = []
    specs = [(32, 0.8, 4.0, 3, 101), (48, 0.6, 5.0, 4, 102), (32, 1.1, 6.0, 2, 103), (64, 0.7, 4.0, 5, 104)]
    for L, tau, R, n, seed in specs:
        pos = I.place_particles(3, (L, L, L), R, n, seed)
        boxes.append({"edge": L, "tau": tau, "fluid_force": (2e-6, 1e-7, -3e-7), "pos": pos, "radius": R})
    return boxes


def single_box(gpu_lib, d, steps):
    L = d["edge"]
    n = len(d["pos"])
    s = gpu_lib.Simulation(3, (L, L, L), d["tau"], storage="fp32s", fluid_force=d["fluid_force"],
                           samples=4, kn=0.0, max_particles=n, max_radius=d["radius"])
    s.set_particles(d["pos"], radius=np.full(n, d["radius"]), rho_s=np.full(n, 2.0),
                    fixed=np.ones(n, np.uint8))
    s.step(steps)
    return s


def test_batch_box_equals_single_box(gpu_lib):
    boxes = make_boxes()
    say("batch vs single box")
    b = gpu_lib.Batch(boxes, samples=4)
    b.set_tile_rows(48, 4)
    b.run(40)
    F, T = b.forces()
    start = 0
    for k, d in enumerate(boxes):
        s = single_box(gpu_lib, d, 40)
        fb = b.get_f(k)
        fs = s.get_f()
        Fs, Ts = s.forces()
        n = len(d["pos"])
        eq_f = np.array_equal(fb, fs)
        eq_F = np.array_equal(F[start:start + n], Fs)
        say("box %d (L=%d): f bitwise %s (rel %.2e), F bitwise %s (rel %.2e)"
            % (k, d["edge"], eq_f, rel_err(fb - fb.mean(), fs - fs.mean()), eq_F, rel_err(F[start:start + n], Fs)))
        assert eq_f and eq_F
        start += n


def test_persistent_equals_per_step(gpu_lib):
    boxes = make_boxes()
    say("persistent vs per-step")
    a = gpu_lib.Batch(boxes, samples=4)
    b = gpu_lib.Batch(boxes, samples=4)
    for e, r in ((32, 2), (48, 8), (64, 16)):
        b.set_tile_rows(e, r)
    a.run(30, gpu_lib.LBM_BATCH_PER_STEP)
    b.run(17, gpu_lib.LBM_BATCH_PERSISTENT)
    b.run(13, gpu_lib.LBM_BATCH_PERSISTENT)
    for k in range(len(boxes)):
        assert np.array_equal(a.get_f(k), b.get_f(k))
    assert np.array_equal(a.forces()[0], b.forces()[0])


def test_retired_box_is_frozen(gpu_lib):
    boxes = make_boxes()
    b = gpu_lib.Batch(boxes, samples=4)
    b.run(10)
    f1 = b.get_f(1)
    b.set_active([1, 0, 1, 1])
    b.run(10, gpu_lib.LBM_BATCH_PERSISTENT)
    assert np.array_equal(b.get_f(1), f1)
    assert not np.array_equal(b.get_f(0), f1[:, :32, :32, :32])


def test_batch_drag_against_fp64_oracle(gpu_lib):
    from oracle import oracle as O
    L, R, tau, g = 32, 4.0, 0.9, 5e-6
    pos = I.place_particles(3, (L, L, L), R, 3, 7)
    say("batch drag vs oracle")
    b = gpu_lib.Batch([{"edge": L, "tau": tau, "fluid_force": (g, 0, 0), "pos": pos, "radius": R}], samples=4)
    orc = O.OracleSim(3, (L, L, L), tau, fluid_force=(g, 0, 0), samples=4)
    orc.set_particles(pos, radius=np.full(3, R), rho_s=np.full(3, 2.0), fixed=np.ones(3, np.uint8))
    errs = []
    b.run(300)
    orc.step(300)
    for _ in range(20):
        b.run(1)
        orc.step(1)
        F0, _ = orc.forces()
        F1, _ = b.forces()
        errs.append(np.linalg.norm(F1 - F0, axis=1) / np.linalg.norm(F0, axis=1))
    mean = float(np.mean(errs))
    say("batch FP32s drag vs FP64 oracle: mean rel err %.2e" % mean)
    assert mean <= 1e-3
    U = b.mean_velocity()
    rho, u = orc.macro()
    Uo = np.array([(rho * u[a]).mean() for a in range(3)])
    assert abs(U[0, 0] - Uo[0]) / abs(Uo[0]) < 1e-3


def test_autotune_resets_and_keeps_results(gpu_lib):
    boxes = make_boxes()
    b = gpu_lib.Batch(boxes, samples=4)
    res = b.autotune(steps=5)
    say("autotune", res)
    assert set(res["rows"]) == {32, 48, 64} and res["mode"] in (0, 1) and res["ms_per_step"] > 0
    assert b.t == 0
    ref = gpu_lib.Batch(boxes, samples=4)
    b.run(8, res["mode"])
    ref.run(8)
    for k in range(len(boxes)):
        assert np.array_equal(b.get_f(k), ref.get_f(k))


def test_initial_velocity_is_kept_without_forcing(gpu_lib):
    """A box without spheres or body force started at a uniform velocity
    keeps it (to binary32 rounding); a box without init_velocity starts at
    rest and stays there bit for bit."""
    u0 = (0.03, -0.01, 0.02)
    b = gpu_lib.Batch([{"edge": 32, "tau": 0.8, "init_velocity": u0},
                       {"edge": 32, "tau": 0.8}], samples=4)
    b.run(50)
    U = b.mean_velocity()
    say("uniform box after 50 steps:", U[0])
    assert np.allclose(U[0], u0, rtol=1e-5, atol=1e-9)
    assert np.array_equal(U[1], np.zeros(3))


def _shell_reference(f, pos, R, L, covered):
    """Mean of u = sum c f / sum f over nodes with R + 1 <= |r| <= 2R
    (minimum image) that no sphere covers, computed from [19][L,L,L] f."""
    c = np.array([[0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
                  [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1],
                  [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]], dtype=float)
    # f is [i][z][y][x] in node order x fastest
    rho = f.sum(axis=0)
    u = np.einsum("ai,izyx->azyx", c, f) / rho
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    out = []
    for p in pos:
        d = [x - p[0], y - p[1], z - p[2]]
        d = [dd - L * np.round(dd / L) for dd in d]
        r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        m = (r2 >= (R + 1) ** 2) & (r2 <= 4 * R * R) & ~covered
        out.append([u[a][m].mean() for a in range(3)])
    return np.array(out)


def test_shell_velocity_matches_populations(gpu_lib):
    """Shell-averaged local fluid velocity from the library against the same
    average taken in numpy over the box's pre-collision populations; two
    spheres far apart, so no shell node is covered by the other sphere."""
    L, R = 40, 5.0
    pos = np.array([[10.3, 11.7, 9.2], [30.1, 29.4, 31.6]])
    b = gpu_lib.Batch([{"edge": L, "tau": 0.8, "fluid_force": (3e-6, -1e-6, 2e-6), "pos": pos, "radius": R}],
                      samples=4)
    b.run(60)
    us = b.shell_velocity()
    f = b.get_f(0)
    covered = np.zeros((L, L, L), dtype=bool)   # shell nodes are beyond R + 1 of both centres
    ref = _shell_reference(f, pos, R, L, covered)
    say("shell velocity", us, "reference", ref)
    assert np.allclose(us, ref, rtol=1e-5, atol=1e-12)
