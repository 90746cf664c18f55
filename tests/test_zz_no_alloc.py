"""mlp_gradients_noalloc, the allocation-free gradient entry point (its
intermediates live in a fixed device array of the library), against
mlp_gradients on a context that holds the same parameters.  Both run the same
kernels in the same order, so the gradient and the loss must agree bit for
bit.  Two calls in a row, the second with fewer rows (not a multiple of the
32-row padding) and other parameters, show that nothing the first call left in
the shared array reaches the second."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def problem(n, seed):
    rng = np.random.default_rng(seed)
    sizes = ((40, 128), (128, 128), (128, 128), (128, 1))
    p = []
    for fin, fout in sizes:
        p.append((rng.standard_normal((fout, fin)) / np.sqrt(fin)).ravel())
        p.append(rng.standard_normal(fout) * 0.05)
    params = np.concatenate(p).astype(np.float32)
    X = rng.standard_normal((n, 40)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2]).astype(np.float32)
    return params, X, y


def test_noalloc_gradients_equal_the_context_entry_point(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    m = gpu_lib.Mlp(max_batch=gpu_lib.MLP_NOALLOC_MAX_ROWS)
    for call, (n, seed) in enumerate(((gpu_lib.MLP_NOALLOC_MAX_ROWS, 31), (1000, 32))):
        say("mlp_gradients_noalloc call %d: n=%d seed=%d" % (call, n, seed))
        params, X, y = problem(n, seed)
        m.set_params(params)
        g_ref, loss_ref = m.gradients(X, y)
        P = torch.from_numpy(params).to(dev)
        Xd = torch.from_numpy(X).to(dev)
        yd = torch.from_numpy(y).to(dev)
        G = torch.full((gpu_lib.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device=dev)
        L = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        gpu_lib.mlp_gradients_noalloc(P, Xd, yd, G, L)
        torch.cuda.synchronize()
        g = G.cpu().numpy()
        diff = int(np.count_nonzero(g.view(np.uint32) != g_ref.view(np.uint32)))
        say("  differing gradient entries %d of %d, loss %r vs %r" % (diff, g.size, float(L.item()), loss_ref))
        assert diff == 0
        assert float(L.item()) == loss_ref
        # without a loss output the gradient is the same
        G2 = torch.full_like(G, float("nan"))
        gpu_lib.mlp_gradients_noalloc(P, Xd, yd, G2, None)
        torch.cuda.synchronize()
        assert np.array_equal(G2.cpu().numpy().view(np.uint32), g_ref.view(np.uint32))


def test_noalloc_rejects_sizes_beyond_its_array(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    lib = gpu_lib._load_mlp(gpu_lib.load())
    nmax = gpu_lib.MLP_NOALLOC_MAX_ROWS
    P = torch.zeros(gpu_lib.MLP_NPARAMS, dtype=torch.float32, device=dev)
    X = torch.zeros((nmax + 1, 40), dtype=torch.float32, device=dev)
    y = torch.zeros(nmax + 1, dtype=torch.float32, device=dev)
    G = torch.zeros(gpu_lib.MLP_NPARAMS, dtype=torch.float32, device=dev)
    vp = ctypes.c_void_p
    s = vp(torch.cuda.current_stream(dev).cuda_stream)
    for n in (0, -1, nmax + 1):
        rc = lib.mlp_gradients_noalloc(vp(P.data_ptr()), vp(X.data_ptr()), vp(y.data_ptr()), n,
                                       vp(G.data_ptr()), None, s)
        assert rc == -1, (n, rc)  # LBM_E_INVALID
    with pytest.raises(ValueError, match="1..%d rows" % nmax):
        gpu_lib.mlp_gradients_noalloc(P, X, y, G)
    assert torch.count_nonzero(G).item() == 0
