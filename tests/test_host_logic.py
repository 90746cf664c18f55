

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
