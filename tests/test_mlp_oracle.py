"""Pins of the MLP-closure oracle: bfloat16 rounding against its bit-level
definition, gradients against central finite differences in exact FP64, the
SiLU derivative, the closed form of Adam's first step, and a decreasing loss."""
import numpy as np

from oracle import mlp_oracle as M


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 lies halfway between bf16 1.0 and 1 + 2^-7: ties go to even (1.0)
    assert M.bf16(np.float32(1.0 + 2.0 ** -8))[()] == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert M.bf16(np.float32(1.0 + 3 * 2.0 ** -8))[()] == 1.0 + 2.0 ** -6
    # just above the half-way point rounds up
    assert M.bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20))[()] == 1.0 + 2.0 ** -7
    assert M.bf16(np.float32(-3.0))[()] == -3.0
    assert np.isnan(M.bf16(np.float32(np.nan)))
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    r = M.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
    # representable: the low 16 bits of the binary32 pattern are zero
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_silu_derivative_finite_difference():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.dsilu(z), fd, rtol=1e-7, atol=1e-9)


def small_params(seed=3):
    rng = np.random.default_rng(seed)
    return [[rng.standard_normal((o, i)) * np.sqrt(2.0 / i), rng.standard_normal(o) * 0.1]
            for i, o in zip(M.SIZES[:-1], M.SIZES[1:])]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    params = small_params()
    X = rng.standard_normal((17, 40))
    y = rng.standard_normal(17)
    _, grads = M.loss_and_grads(params, X, y, bf16_ops=False)
    h = 1e-6
    for k in range(4):
        for j in range(2):
            P = params[k][j]
            G = grads[k][j]
            idx = [tuple(rng.integers(0, s) for s in P.shape) for _ in range(6)]
            for ix in idx:
                old = P[ix]
                P[ix] = old + h
                lp, _ = M.loss_and_grads(params, X, y, bf16_ops=False)
                P[ix] = old - h
                lm, _ = M.loss_and_grads(params, X, y, bf16_ops=False)
                P[ix] = old
                fd = (lp - lm) / (2 * h)
                assert abs(G[ix] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, j, ix, G[ix], fd)


def test_bf16_gradients_close_to_exact():
    rng = np.random.default_rng(2)
    params = small_params(4)
    X = rng.standard_normal((64, 40))
    y = rng.standard_normal(64)
    _, g0 = M.loss_and_grads(params, X, y, bf16_ops=False)
    _, g1 = M.loss_and_grads(params, X, y, bf16_ops=True)
    for k in range(4):
        rel = np.linalg.norm(g1[k][0] - g0[k][0]) / np.linalg.norm(g0[k][0])
        assert rel < 3e-2


def test_adam_first_step_closed_form():
    """With zero moments, the bias-corrected first step is lr g / (|g| + eps)."""
    params = small_params(5)
    grads = [[np.full_like(W, 0.3), np.full_like(b, -2.0)] for W, b in params]
    before = [[W.copy(), b.copy()] for W, b in params]
    st = M.adam_state(params)
    M.adam_step(params, grads, st, lr=1e-3)
    for k in range(4):
        assert np.allclose(params[k][0] - before[k][0], -1e-3 * 0.3 / (0.3 + 1e-8), rtol=1e-12)
        assert np.allclose(params[k][1] - before[k][1], 1e-3 * 2.0 / (2.0 + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((256, 40))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    params = M.init_params(11)
    st = M.adam_state(params)
    l0, _ = M.loss_and_grads(params, X, y)
    for _ in range(60):
        _, g = M.loss_and_grads(params, X, y)
        M.adam_step(params, g, st, lr=3e-3)
    l1, _ = M.loss_and_grads(params, X, y)
    assert l1 < 0.3 * l0
