"""Drag-data ensemble and learned closure on top of the batched LB-IMB runs.

sample_boxes()   draws the periodic boxes of the ensemble (seeded);
autotune_cached() tile shape and launch mode per box edge, cached in JSON;
run_to_steady()  advances a Batch until every box's drag is steady or a step
                 cap is reached, retiring converged boxes early;
drag_dataset()   per-sphere closure inputs (computed on the device) and
                 normalised drag;
train_closure()  trains the BF16-MFMA MLP on (features, ln normalised drag);
evaluate()       compares closure, a Wen-Yu-type correlation and the resolved
                 drag on held-out boxes, with resolved drag as the fallback
                 outside the training envelope.

All lattice work runs in the HIP library (binding.Batch / binding.Mlp).
"""
import math
import time

import numpy as np

from . import binding
from . import inputs as I

EDGES = (32, 48, 64, 96)
NFEAT = 40


def _wen_yu_factor(phi, re):
    """Drag of a particle in a suspension over its Stokes drag at the same
    superficial velocity, Wen & Yu form (1 - phi)^-3.65 (1 + 0.15 Re^0.687)."""
    return (1.0 - phi) ** -3.65 * (1.0 + 0.15 * re ** 0.687)


def sample_boxes(n_boxes, seed, edges=EDGES, phi_range=(0.05, 0.4), r_range=(4.0, 8.0),
                 re_range=(0.1, 50.0), max_spheres=64, u_target=0.02, tau_range=(0.52, 2.0),
                 phi_cap=0.3):
    """Periodic boxes for the ensemble (seed -> identical boxes).

    Edge uniform over `edges`, solid fraction uniform in phi_range (capped at
    phi_cap, the random-sequential-addition limit used here), radius uniform
    in r_range, N = round(phi L^3 / (4/3 pi r^3)) kept if 1 <= N <= max_spheres,
    target particle Reynolds number log-uniform in re_range.  tau puts the
    superficial velocity near u_target (clamped to tau_range); the +x body
    force is the Wen-Yu estimate of the drag of N particles spread over the
    box, and the fluid starts at the superficial velocity that estimate
    targets, which shortens the approach to steady drag.  The achieved Re is
    measured after the run.
    """
    rs = I.Stream(seed)
    boxes = []
    b = 0
    draws = 0
    while len(boxes) < n_boxes:
        draws += 1
        if draws > 1000 * n_boxes:
            raise ValueError("sample_boxes: no box meets the limits (edge, radius, solid fraction, "
                             "max_spheres) in %d draws" % (draws - 1))
        u = rs.uniform(5)
        L = int(edges[min(int(u[0] * len(edges)), len(edges) - 1)])
        phi = phi_range[0] + u[1] * (phi_range[1] - phi_range[0])
        r = r_range[0] + u[2] * (r_range[1] - r_range[0])
        re = math.exp(math.log(re_range[0]) + u[3] * (math.log(re_range[1]) - math.log(re_range[0])))
        phi_eff = min(phi, phi_cap)
        n = int(round(phi_eff * L ** 3 / (4.0 / 3.0 * math.pi * r ** 3)))
        if n < 1 or n > max_spheres or 2 * r + 2 > L:
            continue
        d = 2.0 * r
        nu = min(max(u_target * d / re, (tau_range[0] - 0.5) / 3.0), (tau_range[1] - 0.5) / 3.0)
        tau = 0.5 + 3.0 * nu
        U = re * nu / d
        phi_box = n * 4.0 / 3.0 * math.pi * r ** 3 / L ** 3
        Fp = 3.0 * math.pi * nu * d * U * _wen_yu_factor(phi_box, re)
        g = n * Fp / L ** 3
        try:
            pos = I.place_particles(3, (L, L, L), r, n, seed * 100003 + b, max_tries=2000)
        except RuntimeError:
            b += 1
            continue
        boxes.append({"edge": L, "tau": tau, "fluid_force": (g, 0.0, 0.0), "pos": pos, "radius": r,
                      "init_velocity": (U, 0.0, 0.0), "re_target": re, "phi": phi_box,
                      "seed": seed * 100003 + b})
        b += 1
    return boxes


def autotune_cached(batch, path=None, steps=10):
    """Tile rows per box edge and launch mode for `batch`, from the JSON cache
    at `path` when it holds every edge of the batch for this device, else
    timed by the library's autotuner (which resets the batch to its initial
    state) and stored.  Returns {"rows": {edge: rows}, "mode", "cached"}."""
    import json
    import os
    import torch
    key = torch.cuda.get_device_name(batch.device) + "|fp32s"
    cache = {}
    if path and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    entry = cache.get(key, {})
    rows = entry.get("rows", {})
    edges = sorted(set(batch.edges))
    if "mode" in entry and all(str(e) in rows for e in edges):
        for e in edges:
            batch.set_tile_rows(e, int(rows[str(e)]))
        return {"rows": {e: int(rows[str(e)]) for e in edges}, "mode": int(entry["mode"]), "cached": True}
    res = batch.autotune(steps=steps)
    rows.update({str(e): r for e, r in res["rows"].items()})
    cache[key] = {"rows": rows, "mode": res["mode"]}
    if path:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    res["cached"] = False
    return res


def run_to_steady(batch, boxes, check_every=500, max_steps=20000, tol=1e-5, mode=None, log=None):
    """Advance until every box's drag changes by less than `tol` (max over its
    spheres of |dF| / mean |F|) between checks, or `max_steps`; the check and
    the retirement of converged boxes run on the device
    (lbm_batch_run_steady).  Returns the per-box steady flag and the step count
    at which each box stopped."""
    if mode is None:
        mode = binding.LBM_BATCH_PER_STEP
    t0 = batch.t
    steady, stop = batch.run_steady(max_steps, tol, check_every, mode)
    if log:
        log("  %d steps: %d of %d boxes steady" % (batch.t - t0, int(steady.sum()), len(boxes)))
    return steady, stop - t0


NNEIGH = 16  # nearest neighbours described by position in the closure inputs


def stokes_scale(boxes, U):
    """Per sphere, the Stokes drag 3 pi nu d |U| at the box's superficial
    velocity U (the drag normalisation of the closure)."""
    out = []
    for bi, b in enumerate(boxes):
        nu = (b["tau"] - 0.5) / 3.0
        umag = float(np.linalg.norm(np.asarray(U[bi])))
        out += [3.0 * math.pi * nu * 2.0 * b["radius"] * umag] * len(b["pos"])
    return np.asarray(out)


def drag_dataset(boxes, batch, steady, U):
    """The 40 closure inputs of every sphere (computed on the device,
    lbm_batch_get_drag), its normalised drag y = F . U/|U| / (3 pi nu d |U|),
    the box of each sphere and whether that box reached steady drag."""
    F, X = batch.get_drag()
    scale = stokes_scale(boxes, U)
    counts = [len(b["pos"]) for b in boxes]
    box_of = np.repeat(np.arange(len(boxes)), counts)
    e = np.asarray(U, dtype=np.float64)
    e = e / np.maximum(np.linalg.norm(e, axis=1, keepdims=True), 1e-300)
    y = np.einsum("ij,ij->i", F, e[box_of]) / scale
    return X.astype(np.float64), y, box_of, np.asarray(steady, dtype=bool)[box_of]


class Normaliser:
    """z-score of the inputs with training statistics; training envelope."""

    def __init__(self, X):
        self.mu = X.mean(axis=0)
        self.sd = X.std(axis=0) + 1e-12
        self.lo = X.min(axis=0)
        self.hi = X.max(axis=0)

    def __call__(self, X):
        return (X - self.mu) / self.sd

    def inside(self, X):
        return np.all((X >= self.lo) & (X <= self.hi), axis=1)


def train_closure(X, y, epochs=60, batch=2048, lr=2e-3, seed=5, device="cuda:0", log=None):
    """Train the MLP on z-scored X and ln y (mean squared error, Adam with a
    cosine-decayed learning rate, minibatches drawn by a seeded permutation).
    Returns (mlp, normaliser, per-epoch mean losses)."""
    norm = Normaliser(X)
    Xn = norm(X).astype(np.float32)
    t = np.log(np.maximum(y, 1e-6)).astype(np.float32)
    mlp = binding.Mlp(max_batch=batch, device=device)
    mlp.set_params(binding.mlp_pack(I.mlp_initial_params(seed)))
    n = len(Xn)
    steps_per_epoch = max(1, (n + batch - 1) // batch)
    total = epochs * steps_per_epoch
    import torch
    Xd = torch.as_tensor(Xn, device=device)
    td = torch.as_tensor(t, device=device)
    losses = []
    k = 0
    for ep in range(epochs):
        perm = np.argsort(I.uniform(seed + 1000 + ep, 0, n))
        el = []
        for s0 in range(0, n, batch):
            idx = torch.as_tensor(perm[s0:s0 + batch], device=device)
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * k / total))
            el.append(mlp.train_step(Xd[idx], td[idx], rate))
            k += 1
        losses.append(float(np.mean(el)))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log("epoch %d loss %.4e" % (ep, losses[-1]))
    mlp.set_normaliser(norm.mu, norm.sd, norm.lo, norm.hi)
    return mlp, norm, losses


def predict(mlp, X):
    """Normalised drag predicted by the closure on raw inputs X, and the rows
    outside the training envelope (mlp_infer)."""
    y, out = mlp.infer(np.asarray(X, dtype=np.float32))
    return np.exp(y.cpu().numpy().astype(np.float64)), out.cpu().numpy().astype(bool)


def evaluate(mlp, norm, X, y, box_of=None):
    """Closure vs resolved drag on held-out particles.

    The closure's error is reported on the rows inside the training envelope
    (mlp_rel_err_*) with the fraction of rows outside it, where the resolved
    drag is used instead (fallback_fraction); the error of the closure alone
    on every row is reported as well.  The Wen-Yu-type correlation (no
    learning) uses the local solid fraction (input 0, with the box value as
    floor) and the box Reynolds number.  With `box_of` (the box of each
    particle) the errors of the box means (mean predicted drag of a box's
    particles, resolved drag at the fallback rows, against their mean resolved
    drag) are reported as well."""
    PHI_BOX, LOG_RE = NFEAT - 3, 1
    pred, outside = predict(mlp, X)
    inside = ~outside
    err_mlp = np.abs(pred - y) / np.abs(y)
    phi = np.maximum(X[:, 0], X[:, PHI_BOX])
    wy = _wen_yu_factor(np.minimum(phi, 0.6), 10.0 ** X[:, LOG_RE])
    err_wy = np.abs(wy - y) / np.abs(y)
    Xd = mlp._dev(np.asarray(X, dtype=np.float32), (-1, NFEAT))
    mlp.infer(Xd)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mlp.infer(Xd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nan = float("nan")
    out = {"n": int(len(y)), "fallback_fraction": float(outside.mean()),
           "mlp_rel_err_mean": float(err_mlp[inside].mean()) if inside.any() else nan,
           "mlp_rel_err_median": float(np.median(err_mlp[inside])) if inside.any() else nan,
           "mlp_rel_err_p90": float(np.quantile(err_mlp[inside], 0.9)) if inside.any() else nan,
           "mlp_rel_err_mean_all_rows": float(err_mlp.mean()),
           "wen_yu_rel_err_mean": float(err_wy.mean()),
           "wen_yu_rel_err_mean_inside": float(err_wy[inside].mean()) if inside.any() else nan,
           "inference_s": t1 - t0}
    if box_of is not None:
        used = np.where(inside, pred, y)
        eb_mlp, eb_wy = [], []
        for b in np.unique(box_of):
            m = box_of == b
            ref = y[m].mean()
            eb_mlp.append(abs(used[m].mean() - ref) / abs(ref))
            eb_wy.append(abs(wy[m].mean() - ref) / abs(ref))
        out.update({"boxes": len(eb_mlp), "mlp_box_mean_rel_err": float(np.mean(eb_mlp)),
                    "mlp_box_max_rel_err": float(np.max(eb_mlp)),
                    "wen_yu_box_mean_rel_err": float(np.mean(eb_wy))})
    return out
