"""Plain numpy reference of the closure's 40 per-sphere inputs, the check for
the device kernel behind lbm_batch_get_drag (tests only).

Written from the inputs' definition, sphere by sphere, in binary64: the local
solid fraction from neighbour centres within 3R, the box Reynolds number, the
shell velocity in the flow-aligned frame, the 16 nearest neighbours (minimum
image, stable by distance) along and across the flow, the box solid fraction,
d / L and the nearest surface gap.
"""
import math

import numpy as np

NFEAT = 40
NNEIGH = 16


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
