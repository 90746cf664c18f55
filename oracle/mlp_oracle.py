"""FP64 oracle of the learned drag closure (test infrastructure only).

The closure is a multilayer perceptron 40 -> 128 -> 128 -> 128 -> 1 with SiLU
on the hidden layers, trained with mean-squared error by Adam (Kingma & Ba
2015).  The GPU kernels feed bfloat16 operands to matrix cores and accumulate
in binary32; this oracle takes the same steps in binary64, rounding every
matrix-product operand to bfloat16 (round to nearest even) at the same places
when `bf16=True`, so the two agree to binary32 accumulation error.  With
`bf16=False` it is the exact-arithmetic reference used for the finite-difference
pins.

Only tests and the benchmark's CPU leg may import this module.
"""
import numpy as np

SIZES = (40, 128, 128, 128, 1)


def bf16(x):
    """Round binary32 values to bfloat16, nearest even; NaN stays NaN."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed):
    """Seeded initial weights, drawn by the shared input generator."""
    from paper_1011_2613_amd import inputs as I
    return I.mlp_initial_params(seed, SIZES)


def _q(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, X, bf16_ops=True):
    """Returns the output [n] and the per-layer cache (inputs, pre-activations)."""
    h = np.asarray(X, dtype=np.float64)
    cache = []
    L = len(params)
    for k, (W, b) in enumerate(params):
        hq = _q(h, bf16_ops)
        Wq = _q(W, bf16_ops)
        z = hq @ Wq.T + b
        cache.append((hq, z))
        h = silu(z) if k < L - 1 else z
    return h[:, 0], cache


def loss_and_grads(params, X, y, bf16_ops=True):
    """Mean-squared error 1/n sum (out - y)^2 and its gradients."""
    out, cache = forward(params, X, bf16_ops)
    n = len(y)
    r = out - y
    loss = float(np.mean(r * r))
    g = (2.0 / n) * r[:, None]          # dL/dz of the output layer
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        W, b = params[k]
        hq, z = cache[k]
        gq = _q(g, bf16_ops)
        grads[k] = [gq.T @ hq, g.sum(axis=0)]
        if k > 0:
            gh = gq @ _q(W, bf16_ops)
            _, zprev = cache[k - 1]
            g = gh * dsilu(zprev)
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the binary32 master weights (state: t, m, v)."""
    state["t"] += 1
    t = state["t"]
    for k in range(len(params)):
        for j in range(2):
            g = grads[k][j]
            m = state["m"][k][j] = b1 * state["m"][k][j] + (1 - b1) * g
            v = state["v"][k][j] = b2 * state["v"][k][j] + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            params[k][j] = params[k][j] - lr * mh / (np.sqrt(vh) + eps)
    return params


def adam_state(params):
    return {"t": 0, "m": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params],
            "v": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]}
