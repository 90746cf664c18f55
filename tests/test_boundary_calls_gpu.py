"""The ensemble and closure calls of the C ABI on the GPU:

- lbm_batch_run_steady (steady check and retirement on the device, chunks
  replayed as a captured graph) against the same check written on the host
  over lbm_batch_run / lbm_batch_forces / lbm_batch_set_active: identical
  steady flags, stop steps and bitwise identical forces;
- lbm_batch_get_drag's 40 inputs against the numpy reference of their
  definition (tests/closure_features_ref.py), to binary32 rounding;
- mlp_infer (normalisation and envelope flags on the device) against
  mlp_forward on inputs normalised on the host, and the flags against the
  envelope test in binary32.
"""
import numpy as np
import pytest

import closure_features_ref as REF
from paper_1011_2613_amd import binding, ensemble as E

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def small_boxes(n, seed):
    return E.sample_boxes(n, seed, edges=(32, 48), r_range=(4.0, 6.0), re_range=(0.1, 20.0))


def host_steady(b, boxes, check_every, max_steps, tol, mode):
    """The steady check on the host (the previous implementation)."""
    nb = len(boxes)
    counts = [len(x["pos"]) for x in boxes]
    offs = np.concatenate([[0], np.cumsum(counts)])
    active = np.ones(nb, dtype=np.uint8)
    steady = np.zeros(nb, dtype=bool)
    stop = np.full(nb, max_steps)
    prev = None
    t = 0
    while t < max_steps and active.any():
        k = min(check_every, max_steps - t)
        b.run(k, mode)
        t += k
        F, _ = b.forces()
        if prev is not None:
            for i in range(nb):
                if not active[i] or counts[i] == 0:
                    continue
                Fb, Pb = F[offs[i]:offs[i + 1]], prev[offs[i]:offs[i + 1]]
                scale = np.linalg.norm(Fb, axis=1).mean()
                if scale > 0 and np.abs(Fb - Pb).max() / scale < tol:
                    active[i] = 0
                    steady[i] = True
                    stop[i] = t
            b.set_active(active)
        prev = F.copy()
    for i in range(nb):
        if active[i]:
            stop[i] = t
    return steady, stop


@pytest.mark.parametrize("mode", [binding.LBM_BATCH_PER_STEP, binding.LBM_BATCH_PERSISTENT])
def test_run_steady_matches_the_host_check(mode):
    boxes = small_boxes(12, 41)
    boxes.append({"edge": 32, "tau": 0.8, "fluid_force": (1e-6, 0.0, 0.0), "pos": np.zeros((0, 3)),
                  "radius": 4.0})  # no spheres: never retires
    check, steps, tol = 150, 2250, 1e-4  # the last chunk is partial (2250 = 15 x 150)
    say("run_steady mode %d: %d boxes, check every %d, %d steps" % (mode, len(boxes), check, steps))
    dev = binding.Batch(boxes, samples=4)
    steady_d, stop_d = dev.run_steady(steps, tol, check, mode)
    host = binding.Batch(boxes, samples=4)
    steady_h, stop_h = host_steady(host, boxes, check, steps, tol, mode)
    say("  steady device %s host %s" % (steady_d.astype(int).tolist(), steady_h.astype(int).tolist()))
    say("  stop device %s host %s" % (stop_d.tolist(), stop_h.tolist()))
    assert 0 < steady_d.sum() < len(boxes)
    assert np.array_equal(steady_d, steady_h)
    assert np.array_equal(stop_d, stop_h)
    assert not steady_d[-1] and stop_d[-1] == steps
    Fd, _ = dev.forces()
    Fh, _ = host.forces()
    assert np.array_equal(Fd.view(np.uint64), Fh.view(np.uint64))
    # a second call continues from the batch time; retired boxes stay retired
    t1 = dev.t
    steady2, stop2 = dev.run_steady(300, tol, check, mode)
    assert dev.t == t1 + 300 or not (~steady_d).any()
    assert not np.any(steady2 & steady_d)
    assert np.all(stop2[steady_d] == t1)


def test_run_steady_rejects_bad_arguments():
    b = binding.Batch(small_boxes(2, 43), samples=4)
    lib = binding.load()
    for args in ((-1, 1e-4, 10, 0), (10, 0.0, 10, 0), (10, float("nan"), 10, 0), (10, 1e-4, 0, 0),
                 (10, 1e-4, 10, 7)):
        rc = lib.lbm_batch_run_steady(b._ctx, args[0], args[1], args[2], args[3], None, None)
        assert rc == -1, args
    assert b.t == 0


def test_features_match_the_reference():
    boxes = small_boxes(10, 47)
    # a box with one sphere and one with more than 16 others exercise the padding and the cut
    boxes.append({"edge": 32, "tau": 0.7, "fluid_force": (2e-6, 0.0, 0.0), "pos": np.array([[7.5, 9.0, 20.25]]),
                  "radius": 4.5})
    boxes += E.sample_boxes(1, 53, edges=(32,), r_range=(4.0, 4.0), phi_range=(0.2, 0.2))  # 24 spheres
    say("features: %d boxes, %d spheres" % (len(boxes), sum(len(x["pos"]) for x in boxes)))
    b = binding.Batch(boxes, samples=4)
    b.run(400)
    F, X = b.get_drag()
    U = b.mean_velocity()
    Us = b.shell_velocity()
    Fr, _ = b.forces()
    assert np.array_equal(F, Fr)
    Xr, _ = REF.features(boxes, U, Us)
    Xr32 = Xr.astype(np.float32)
    diff = np.abs(X.astype(np.float64) - Xr32.astype(np.float64))
    tol = 4.0 * np.spacing(np.abs(Xr32)).astype(np.float64) + 1e-7
    bad = np.argwhere(diff > tol)
    say("  max |diff| %.2e; entries beyond 4 ulp + 1e-7: %d" % (diff.max(), len(bad)))
    assert len(bad) == 0, bad[:10]
    assert max(len(x["pos"]) for x in boxes) > 17


def test_infer_matches_forward_and_envelope():
    rng = np.random.default_rng(61)
    n = 3001
    Xtr = (rng.standard_normal((5000, 40)) * rng.uniform(0.1, 5.0, 40) + rng.uniform(-2, 2, 40))
    Xtr = Xtr.astype(np.float32).astype(np.float64)
    norm = E.Normaliser(Xtr)
    X = (rng.standard_normal((n, 40)) * 1.2 * np.sqrt(np.var(Xtr, axis=0)) + Xtr.mean(axis=0)).astype(np.float32)
    X[5, 3] = np.float32(norm.lo[3])  # on the edge: inside
    X[6, 7] = np.float32(np.nan)      # NaN: outside
    m = binding.Mlp(max_batch=64)
    m.set_params(binding.mlp_pack(E.I.mlp_initial_params(3)))
    with pytest.raises(binding.LbmError):
        m.infer(X)  # no normaliser yet
    m.set_normaliser(norm.mu, norm.sd, norm.lo, norm.hi)
    y, flag = m.infer(X)
    y = y.cpu().numpy().astype(np.float64)
    flag = flag.cpu().numpy().astype(bool)
    ok = ~np.isnan(X).any(axis=1)
    y_ref = m.forward(norm(X[ok].astype(np.float64)).astype(np.float32)).cpu().numpy().astype(np.float64)
    err = np.abs(y[ok] - y_ref).max() / max(np.abs(y_ref).max(), 1e-3)
    lo32, hi32 = norm.lo.astype(np.float32), norm.hi.astype(np.float32)
    with np.errstate(invalid="ignore"):
        flag_ref = ~np.all((X >= lo32) & (X <= hi32), axis=1)
    say("infer: rel err vs host-normalised forward %.2e; %d of %d rows outside" % (err, flag.sum(), n))
    assert err < 1e-2
    assert np.array_equal(flag, flag_ref)
    assert flag[6]
    assert 0 < flag.sum() < n
