"""Drag-closure MLP on the GPU (bfloat16 MFMA, binary32 accumulation) against
the FP64 oracle that rounds the same operands to bfloat16.

Tolerances: the oracle accumulates in binary64, the GPU in binary32, so a
bfloat16 rounding of an activation can land on the other side of a tie in a
few elements; outputs agree to 2e-3 relative (max over rows, scaled by the
output range) and gradients norm-wise per tensor to 1e-2.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def params_and_data(n, seed):
    params = M.init_params(seed)
    rng = np.random.default_rng(seed)
    for W, b in params:
        b[:] = rng.standard_normal(b.shape) * 0.05
    X = rng.standard_normal((n, 40)).astype(np.float32).astype(np.float64)
    y = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2]).astype(np.float32).astype(np.float64)
    # the GPU holds binary32 masters
    params = [[W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)]
              for W, b in params]
    return params, X, y


@pytest.mark.parametrize("n", [1, 15, 1000, 4099])
def test_forward_matches_oracle(gpu_lib, n):
    params, X, _ = params_and_data(n, 21)
    say("mlp forward", n)
    m = gpu_lib.Mlp(max_batch=64)
    m.set_params(gpu_lib.mlp_pack(params))
    y_gpu = m.forward(X).cpu().numpy().astype(np.float64)
    y_ref, _ = M.forward(params, X, bf16_ops=True)
    scale = max(np.abs(y_ref).max(), 1e-3)
    err = np.abs(y_gpu - y_ref).max() / scale
    say("forward n=%d rel err %.2e" % (n, err))
    assert err < 2e-3


@pytest.mark.parametrize("n", [32, 300])
def test_gradients_match_oracle(gpu_lib, n):
    params, X, y = params_and_data(n, 22)
    say("mlp gradients", n)
    m = gpu_lib.Mlp(max_batch=512)
    m.set_params(gpu_lib.mlp_pack(params))
    g, loss = m.gradients(X, y)
    loss_ref, g_ref = M.loss_and_grads(params, X, y, bf16_ops=True)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref) + 1e-7
    got = gpu_lib.mlp_unpack(g)
    for k in range(4):
        for j in range(2):
            a, b = np.asarray(got[k][j], dtype=np.float64), np.asarray(g_ref[k][j]).reshape(np.shape(got[k][j]))
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            say("grad layer %d %s rel %.2e" % (k + 1, "W" if j == 0 else "b", rel))
            assert rel < 1e-2


def test_training_reduces_loss_and_tracks_oracle(gpu_lib):
    params, X, y = params_and_data(2048, 23)
    m = gpu_lib.Mlp(max_batch=2048)
    m.set_params(gpu_lib.mlp_pack(params))
    st = M.adam_state(params)
    losses = []
    for it in range(40):
        losses.append(m.train_step(X, y, 2e-3))
        _, g = M.loss_and_grads(params, X, y, bf16_ops=True)
        M.adam_step(params, g, st, lr=2e-3)
    say("gpu losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
    p_gpu = m.get_params().astype(np.float64)
    p_ref = gpu_lib.mlp_pack(params)
    rel = np.linalg.norm(p_gpu - p_ref) / np.linalg.norm(p_ref)
    say("params after 40 Adam steps: rel diff to oracle %.2e" % rel)
    assert rel < 1e-2
