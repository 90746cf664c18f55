"""Host-side logic that needs no GPU: the resolution study's extrapolation
and the numpy reference of the closure's input features (the check of the
device feature kernel)."""
import numpy as np


def test_validation_extrapolation_recovers_limit_and_order():
    """K = K_inf + a d^-p sampled at three resolutions gives back K_inf and p;
    a non-monotone triple gives no estimate; Hasimoto's K tends to 1 as the
    solid fraction vanishes."""
    from paper_1011_2613_amd import validation as V
    for Kinf, a, p in ((2.15, -11.0, 1.9), (1.0, 3.0, 1.0), (5.0, -0.5, 2.5)):
        ds = [8.0, 12.0, 16.0]
        K, q = V.extrapolate(ds, [Kinf + a * d ** -p for d in ds])
        assert abs(K - Kinf) < 1e-9 * abs(Kinf) and abs(q - p) < 1e-9
    assert V.extrapolate([4.0, 8.0, 16.0], [1.0, 2.0, 1.5]) == (None, None)
    assert abs(V.hasimoto_K(1e-12) - 1.0) < 1e-3


def test_closure_neighbour_features():
    """The 16 neighbour inputs: nearest first, distance along the mean flow
    and across it over d (minimum image), padded with L/d when the box holds
    fewer spheres; the other inputs sit where the evaluation expects them."""
    import math
    import closure_features_ref as E
    L, R = 32, 2.0
    d = 2 * R
    pos = np.array([[5.0, 5.0, 5.0], [9.0, 5.0, 5.0], [5.0, 11.0, 5.0], [30.0, 5.0, 8.0]])
    box = {"pos": pos, "radius": R, "edge": L, "tau": 0.8}
    U = [np.array([0.02, 0.0, 0.0])]
    Us = np.zeros((4, 3))
    X, scale = E.features([box], U, Us)
    assert X.shape == (4, E.NFEAT)
    nb = X[0, 5:5 + 2 * E.NNEIGH]
    # neighbours of sphere 0: (4,0,0) at 4, (-7,0,3) at 7.6 (image of sphere 3), (0,6,0) at 6
    assert np.allclose(nb[0:2], [4.0 / d, 0.0])
    assert np.allclose(nb[2:4], [0.0, 6.0 / d])
    assert np.allclose(nb[4:6], [-7.0 / d, 3.0 / d])
    assert np.all(nb[6:] == L / d)
    nu = (0.8 - 0.5) / 3.0
    assert abs(X[0, 1] - math.log10(0.02 * d / nu)) < 1e-12
    assert abs(X[0, E.NFEAT - 3] - 4 * 4.0 / 3.0 * math.pi * R ** 3 / L ** 3) < 1e-12
    assert abs(X[0, E.NFEAT - 1] - (4.0 - d) / d) < 1e-12
    assert np.allclose(scale, 3 * math.pi * nu * d * 0.02)


def test_bench_launch_shape_option():
    """bench.py --lattice-block: "auto", one shape for all, or per variant;
    a shape is a width with an optional "/xcd" workgroup order and "/cuN"
    cap, and the text form round-trips."""
    import bench
    assert bench.parse_blocks("auto") == {}
    assert bench.parse_blocks("192") == {v: (192, "linear", 0) for v in ("fp64", "fp32s", "fp16s")}
    assert bench.parse_blocks("fp64=256/xcd/cu3,fp32s=64") == {"fp64": (256, "xcd", 3),
                                                             "fp32s": (64, "linear", 0)}
    for shape in ((64, "linear", 0), (256, "xcd", 0), (192, "linear", 4), (256, "xcd", 3)):
        assert bench.parse_shape(bench.shape_text(shape)) == shape


def test_bench_traffic_lookup_by_shape(tmp_path, monkeypatch):
    """The committed counter records are matched on kernel source and launch
    shape; a storage mode may carry one record or a list of them."""
    import json
    import bench
    (tmp_path / "profiles").mkdir()
    recs = {"C3_fp64": [{"kernel_source_sha": "s1", "lattice_block": "256/xcd/cu4", "bytes_per_launch": 11},
                        {"kernel_source_sha": "s1", "lattice_block": "192/xcd/cu4", "bytes_per_launch": 12}],
            "C3_fp32s": {"kernel_source_sha": "s1", "lattice_block": "64", "bytes_per_launch": 21}}
    (tmp_path / "profiles" / "lb_kernel_traffic.json").write_text(json.dumps(recs))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "s1")
    assert bench.measured_traffic("fp64", "C3", "192/xcd/cu4") == 12
    assert bench.measured_traffic("fp64", "C3", "256/xcd/cu4") == 11
    assert bench.measured_traffic("fp64", "C3", "256") is None
    assert bench.measured_traffic("fp32s", "C3", "64") == 21
    assert bench.measured_traffic("fp16s", "C3", "64") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "s2")
    assert bench.measured_traffic("fp32s", "C3", "64") is None


def test_closure_ensemble_cache(tmp_path):
    """Ensembles saved per seed are read back instead of being run again (from
    the first folder that holds them), and with the time budget spent and no
    saved copy nothing runs."""
    import json
    from paper_1011_2613_amd import closure_pipeline as CP
    kw = dict(max_steps=20000, tol=1e-5)
    name = CP._cache_name(1007, 512, 20000, 1e-5)
    X = np.arange(12, dtype=np.float32).reshape(3, 4)
    y = np.array([1.0, 2.0, 3.0])
    box_of = np.array([0, 0, 1])
    rs = np.array([True, False, True])
    st = {"boxes": 512, "steady_boxes": 1, "samples": 2, "run_s": 1.5, "mlups": 3.0e4}
    other = tmp_path / "other"
    other.mkdir()
    np.savez_compressed(str(tmp_path / name), X=X, y=y, box_of=box_of, row_steady=rs, stats=json.dumps(st))
    got = CP.cached_ensemble(1007, 512, [str(other), str(tmp_path)], None, budget_end=0.0, **kw)
    assert got is not None
    gX, gy, gb, grs, gst = got
    assert np.array_equal(gX, X) and np.array_equal(gy, y) and np.array_equal(gb, box_of)
    assert np.array_equal(grs, rs)
    assert gst["cached"] is True and gst["samples"] == 2 and gst["run_s"] == 1.5
    # another seed, budget spent: nothing is run
    assert CP.cached_ensemble(1008, 512, [str(tmp_path)], None, budget_end=0.0, **kw) is None
    # the file name carries the box count, the step cap and the tolerance
    assert CP._cache_name(1007, 64, 20000, 1e-5) != name and CP._cache_name(1007, 512, 10000, 1e-5) != name
