"""Drag-data ensemble and learned closure on top of the batched LB-IMB runs.

sample_boxes()   draws the periodic boxes of the ensemble (seeded);
autotune_cached() tile shape and launch mode per box edge, cached in JSON;
run_to_steady()  advances a Batch until every box's drag is steady or a step
                 cap is reached, retiring converged boxes early;
features()       the 40 per-particle inputs of the closure (local slip from
                 the library's shell velocity);
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
    while len(boxes) < n_boxes:
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
    spheres of |dF| / mean |F|) between checks, or `max_steps`.  Returns the
    per-box steady flag and the step count at which each box stopped."""
    if mode is None:
        mode = binding.LBM_BATCH_PER_STEP
    nb = len(boxes)
    counts = [len(b["pos"]) for b in boxes]
    offs = np.concatenate([[0], np.cumsum(counts)])
    active = np.ones(nb, dtype=np.uint8)
    steady = np.zeros(nb, dtype=bool)
    stop = np.full(nb, max_steps)
    prev = None
    t = 0
    while t < max_steps and active.any():
        k = min(check_every, max_steps - t)
        batch.run(k, mode)
        t += k
        F, _ = batch.forces()
        if prev is not None:
            for b in range(nb):
                if not active[b] or counts[b] == 0:
                    continue
                Fb, Pb = F[offs[b]:offs[b + 1]], prev[offs[b]:offs[b + 1]]
                scale = np.linalg.norm(Fb, axis=1).mean()
                if scale > 0 and np.abs(Fb - Pb).max() / scale < tol:
                    active[b] = 0
                    steady[b] = True
                    stop[b] = t
            batch.set_active(active)
        prev = F.copy()
        if log:
            log("  t=%d: %d of %d boxes still running" % (t, int(active.sum()), nb))
    return steady, stop


NNEIGH = 16  # nearest neighbours described by position in the closure inputs


def features(boxes, U, Us):
    """The 40 per-particle closure inputs and the normalising drag scale.

    Per particle: local solid fraction of the other spheres within 3R (from
    neighbour centres), log10 of the box Reynolds number Re = |U| d / nu with
    U the superficial mean velocity, the local slip (the mean fluid velocity
    in the shell [R + 1, 2R] around the sphere, Us; the spheres are at rest)
    in the flow-aligned frame over |U| (3), the positions of the 16 nearest
    neighbours (minimum image, nearest first) as the distance along the flow
    and the distance across it, both over d (32; the drag along the flow does
    not change under rotation about it; a box with fewer spheres pads with the
    box edge over d), the box solid fraction, d / L and the nearest surface
    gap / d.
    Returns X [n, 40] and the Stokes drag scale 3 pi nu d |U| [n].
    """
    rows, scale = [], []
    k = 0
    for bi, b in enumerate(boxes):
        pos, r, L = np.asarray(b["pos"]), b["radius"], b["edge"]
        n = len(pos)
        d = 2.0 * r
        nu = (b["tau"] - 0.5) / 3.0
        u = np.asarray(U[bi])
        umag = float(np.linalg.norm(u))
        re = umag * d / nu
        ex = u / umag if umag > 0 else np.array([1.0, 0.0, 0.0])
        phi_box = n * 4.0 / 3.0 * math.pi * r ** 3 / L ** 3
        for p in range(n):
            dvec = pos - pos[p]
            dvec -= L * np.round(dvec / L)
            dist = np.linalg.norm(dvec, axis=1)
            others = np.nonzero(np.arange(n) != p)[0]
            nearest = others[np.argsort(dist[others], kind="stable")][:NNEIGH]
            along = dvec[nearest] @ ex
            across = np.sqrt(np.maximum(dist[nearest] ** 2 - along ** 2, 0.0))
            nb = np.full(2 * NNEIGH, L / d)
            nb[0:2 * len(nearest):2] = along / d
            nb[1:2 * len(nearest):2] = across / d
            n_loc = int(np.count_nonzero(dist[others] < 3.0 * r))
            phi_loc = n_loc / 27.0
            gap = (dist[others].min() - d) / d if n > 1 else L / d
            us = np.asarray(Us[k]) / max(umag, 1e-300)
            ey = np.cross(ex, [0.0, 0.0, 1.0])
            if np.linalg.norm(ey) < 1e-8:
                ey = np.cross(ex, [0.0, 1.0, 0.0])
            ey /= np.linalg.norm(ey)
            ez = np.cross(ex, ey)
            rows.append([phi_loc, math.log10(max(re, 1e-6)), us @ ex, us @ ey, us @ ez, *nb,
                         phi_box, d / L, gap])
            scale.append(3.0 * math.pi * nu * d * umag)
            k += 1
    X = np.asarray(rows, dtype=np.float64)
    assert X.shape[1] == NFEAT
    return X, np.asarray(scale)


def drag_dataset(boxes, batch, steady, U):
    """Features, normalised drag y = F . U/|U| / (3 pi nu d |U|) and the box of
    each particle, for the steady boxes only."""
    F, _ = batch.forces()
    counts = [len(b["pos"]) for b in boxes]
    offs = np.concatenate([[0], np.cumsum(counts)])
    X, scale = features(boxes, U, batch.shell_velocity())
    y = np.empty(len(X))
    box_of = np.empty(len(X), dtype=int)
    k = 0
    for bi, b in enumerate(boxes):
        u = np.asarray(U[bi])
        e = u / max(np.linalg.norm(u), 1e-300)
        for p in range(counts[bi]):
            y[k] = (F[offs[bi] + p] @ e) / scale[k]
            box_of[k] = bi
            k += 1
    keep = steady[box_of]
    return X[keep], y[keep], box_of[keep]


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
    return mlp, norm, losses


def predict(mlp, norm, X):
    """Normalised drag predicted by the closure."""
    y = mlp.forward(norm(X).astype(np.float32)).cpu().numpy().astype(np.float64)
    return np.exp(y)


def evaluate(mlp, norm, X, y, box_of=None):
    """Closure vs resolved drag on held-out particles.  Particles outside the
    training envelope fall back to the resolved drag (zero error, counted).
    The Wen-Yu-type correlation (no learning) uses the local solid fraction
    (feature 0, with the box value as floor) and the box Reynolds number.
    With `box_of` (the box of each particle) the errors of the box means
    (mean predicted drag of a box's particles against their mean resolved
    drag) are reported as well."""
    PHI_BOX, LOG_RE = NFEAT - 3, 1
    inside = norm.inside(X)
    pred = predict(mlp, norm, X)
    err_mlp = np.abs(pred - y) / np.abs(y)
    err_used = np.where(inside, err_mlp, 0.0)
    phi = np.maximum(X[:, 0], X[:, PHI_BOX])
    wy = _wen_yu_factor(np.minimum(phi, 0.6), 10.0 ** X[:, LOG_RE])
    err_wy = np.abs(wy - y) / np.abs(y)
    t0 = time.perf_counter()
    _ = predict(mlp, norm, X)
    t1 = time.perf_counter()
    out = {"n": int(len(y)), "fallback_fraction": float(1.0 - inside.mean()),
           "mlp_mean_rel_err": float(err_used.mean()), "mlp_mean_rel_err_inside": float(err_mlp[inside].mean())
           if inside.any() else float("nan"),
           "mlp_median_rel_err": float(np.median(err_used)),
           "wen_yu_mean_rel_err": float(err_wy.mean()), "inference_s": t1 - t0}
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
