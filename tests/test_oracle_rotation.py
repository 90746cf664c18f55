"""Pins of the oracle's rotational coupling and of its relaxation weight.

What is pinned, and against what (no test retypes an oracle formula):

- The solid velocity V_S = v + omega x r of the operator after Eq. 2 and the
  torque sum of Eq. 3.  On the first step from a fluid at rest (rho = 1,
  u = 0) every covered node exchanges q_n = beta_n rho (v + omega x r_n), so
  the force and torque on a lone particle are closed forms in the
  beta-weighted moments of its footprint, B = sum beta rho, M1 = sum beta rho r
  and M2 = sum beta rho r r^T:  F = -(B v + omega x M1) and
  T = -(M1 x v + tr(M2) omega - M2 omega) (the vector triple product
  r x (omega x r) = |r|^2 omega - (r . omega) r).  The counts come from brute
  force sample counting and beta from Eq. 2 (pinned by its special values).
  The particle straddles a periodic seam, so the minimum-image arms count.
- The Newton-Euler update: omega gains T / I with the textbook moments of
  inertia of a solid sphere (2/5 m R^2) and a disc of unit depth (1/2 m R^2);
  v gains F / m.
- Fully covered nodes (eps = 1, beta = 1) leave the collision with momentum
  rho (v + omega x r), read back after streaming from the neighbours the
  post-collision values moved to.
- A particle spinning in quiescent fluid feels a torque opposing omega whose
  magnitude approaches the rotlet value (8 pi rho nu R^3 omega for a sphere,
  4 pi rho nu R^2 omega for a disc, the exact Stokes torques) as R grows.
- The collision's second moment at a fully covered node,
  Pi_out = Pi_in + rho (V_S V_S - u u), which holds for any tau; at a
  partially covered node the relaxation weight (1 - beta)/tau appears in
  Pi_out = Pi_in - ((1 - beta)/tau) (Pi_in - rho (I/3 + u u))
           + beta rho (V_S V_S - u u),
  both from the lattice's second-moment isotropy (sum w c c = I/3).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

from test_oracle_pins import brute_counts, lattice


def _min_image(d, L):
    return np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))


def _footprint_moments(dim, box, xp, R, S, tau):
    """B, M1, M2 of the beta-weighted footprint (rho = 1 at the first step)."""
    counts = brute_counts(dim, box, xp, R, S)          # [z,] y, x
    Smax = S ** dim
    eps = np.minimum(counts, Smax) / Smax
    beta = np.vectorize(lambda e: O.beta(float(e), tau))(eps)
    grids = np.meshgrid(*[np.arange(n) for n in box], indexing="ij")
    r = np.zeros((3,) + grids[0].shape)
    for a in range(dim):
        r[a] = _min_image(grids[a] - xp[a], box[a])
    bw = beta.T                                         # to [x, y(, z)] order
    rho0 = O.feq(dim, 1.0, [0, 0, 0]).sum()             # rest density as the oracle holds it
    B = rho0 * bw.sum()
    M1 = rho0 * np.array([(bw * r[a]).sum() for a in range(3)])
    M2 = rho0 * np.array([[(bw * r[a] * r[b]).sum() for b in range(3)] for a in range(3)])
    return B, M1, M2


@pytest.mark.parametrize("dim", [2, 3])
def test_first_step_force_torque_and_update_closed_form(dim):
    S, R, tau, rho_s = (8, 5.0, 0.7, 3.0) if dim == 2 else (4, 3.5, 0.7, 3.0)
    box = [30, 26] if dim == 2 else [18, 16, 20]
    xp = np.zeros(3)
    xp[:dim] = [0.8, 24.6] if dim == 2 else [17.3, 0.45, 9.2]   # across periodic seams
    v = np.array([2e-3, -1.5e-3, 1e-3 if dim == 3 else 0.0])
    om = np.array([4e-4, -3e-4, 5e-4]) if dim == 3 else np.array([0.0, 0.0, 6e-4])
    sim = O.OracleSim(dim, box, tau, samples=S)
    sim.set_particles(xp[None], vel=v[None], omega=om[None], radius=[R], rho_s=[rho_s])
    sim.step(1)
    F, T = sim.forces()
    x1, v1, w1 = sim.particles()

    B, M1, M2 = _footprint_moments(dim, box, xp, R, S, tau)
    F_exp = -(B * v + np.cross(om, M1))
    T_exp = -(np.cross(M1, v) + np.trace(M2) * om - M2 @ om)
    if dim == 2:
        F_exp[2] = 0.0
        T_exp[:2] = 0.0
    assert np.abs(F[0] - F_exp).max() <= 1e-12 * np.abs(F_exp).max()
    assert np.abs(T[0] - T_exp).max() <= 1e-12 * np.abs(T_exp).max()
    # the torque opposes the spin (the footprint's inertia tensor is positive)
    assert T[0] @ om < 0

    # Newton-Euler with the textbook mass and moment of inertia
    if dim == 2:
        m = rho_s * math.pi * R ** 2
        inertia = 0.5 * m * R ** 2
    else:
        m = rho_s * 4.0 / 3.0 * math.pi * R ** 3
        inertia = 0.4 * m * R ** 3 / R
    assert np.allclose(v1[0], v + F_exp / m, rtol=0, atol=1e-15 * np.abs(v).max())
    assert np.allclose(w1[0], om + T_exp / inertia, rtol=0, atol=1e-14 * np.abs(om).max())
    x_exp = xp + v1[0]
    x_exp[:dim] = np.mod(x_exp[:dim], box)
    assert np.allclose(x1[0], x_exp, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_fully_covered_nodes_leave_with_rigid_momentum(dim):
    S, R = (8, 6.0) if dim == 2 else (4, 4.5)
    box = [28, 30] if dim == 2 else [20, 18, 16]
    xp = np.zeros(3)
    xp[:dim] = [27.1, 14.3] if dim == 2 else [0.6, 8.9, 15.2]
    v = np.array([1e-3, 2e-3, -1e-3 if dim == 3 else 0.0])
    om = np.array([3e-4, 2e-4, -4e-4]) if dim == 3 else np.array([0.0, 0.0, -5e-4])
    sim = O.OracleSim(dim, box, 0.9, samples=S)
    sim.set_particles(xp[None], vel=v[None], omega=om[None], radius=[R], rho_s=[2.0], fixed=[1])
    rho0 = O.feq(dim, 1.0, [0, 0, 0]).sum()
    sim.step(1)
    f = sim.get_f()                                     # f(x, t+1) = f*(x - c, t)
    c3, _ = lattice(dim)
    counts = brute_counts(dim, box, xp, R, S)
    full = np.argwhere(counts == S ** dim)
    assert len(full) > 20
    for idx in full:
        node = idx[::-1]                                # (x, y[, z])
        post = np.zeros(3)
        for i in range(len(c3)):
            tgt = tuple(((node[a] + int(c3[i, a])) % box[a]) for a in range(dim))
            post += c3[i] * f[(i,) + tgt[::-1]]
        r = np.zeros(3)
        r[:dim] = _min_image(node - xp[:dim], np.array(box))
        vs = v + np.cross(om, r)
        assert np.allclose(post, rho0 * vs, rtol=0, atol=2e-16)


def _rotlet_ratio(dim, R, tau, steps):
    S = 8 if dim == 2 else 4
    L = int(R * (12 if dim == 2 else 8))
    box = [L] * dim
    nu = (tau - 0.5) / 3.0
    sim = O.OracleSim(dim, box, tau, samples=S)
    xp = np.zeros(3)
    xp[:dim] = L / 2 + 0.23
    om = np.array([3e-5, -5e-5, 8e-5]) if dim == 3 else np.array([0.0, 0.0, 1e-4])
    sim.set_particles(xp[None], omega=om[None], radius=[R], rho_s=[2.0], fixed=[1])
    sim.step(steps)
    _, T = sim.forces()
    ref = -(8.0 * math.pi * nu * R ** 3 if dim == 3 else 4.0 * math.pi * nu * R ** 2) * om
    ratio = T[0] @ ref / (ref @ ref)
    perp = np.linalg.norm(T[0] - ratio * ref) / np.linalg.norm(ref)
    return ratio, perp


@pytest.mark.parametrize("dim,radii,steps,bounds", [
    (2, (3.0, 4.5, 6.0), 2000, (0.15, 0.06, 0.025)),
    (3, (2.5, 3.5, 5.0), 500, (0.35, 0.2, 0.1)),
])
def test_spinning_particle_torque_approaches_rotlet(dim, radii, steps, bounds):
    """Steady torque on a particle spinning in a periodic box of edge 12 R (2D)
    or 8 R (3D), tau = 1: it opposes omega, lies along it, and its ratio to the
    Stokes torque tends to 1 as the particle is resolved by more nodes."""
    errs = []
    for R, bound in zip(radii, bounds):
        ratio, perp = _rotlet_ratio(dim, R, 1.0, steps)
        assert 0.0 < ratio < 1.05
        assert perp < 2e-3
        assert 1.0 - ratio < bound
        errs.append(abs(1.0 - ratio))
    assert errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1]


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_second_moment_identities(dim):
    rng = np.random.default_rng(70 + dim)
    c3, w = lattice(dim)
    S = 4
    Smax = S ** dim
    I3 = np.eye(3)
    if dim == 2:
        I3[2, 2] = 0.0
    for trial in range(100):
        tau = float(rng.uniform(0.51, 2.0))
        fin = w * (1.0 + 0.05 * rng.standard_normal(len(w)))
        vs = np.zeros(3)
        vs[:dim] = 0.03 * rng.standard_normal(dim)
        rho = fin.sum()
        u = (fin @ c3) / rho
        Pin = np.einsum("i,ia,ib->ab", fin, c3, c3)
        dV = rho * (np.outer(vs, vs) - np.outer(u, u))
        # eps = 1: independent of tau
        fout, _ = O.collide_node(dim, tau, [0, 0, 0], S, fin, Smax, vs)
        Pout = np.einsum("i,ia,ib->ab", fout, c3, c3)
        assert np.allclose(Pout, Pin + dV, rtol=0, atol=4e-16 * len(w))
        # partial cover: relaxation weight (1 - beta)/tau
        count = int(rng.integers(1, Smax))
        eps = count / Smax
        beta = O.beta(eps, tau)
        fout, _ = O.collide_node(dim, tau, [0, 0, 0], S, fin, count, vs)
        Pout = np.einsum("i,ia,ib->ab", fout, c3, c3)
        Peq = rho * (I3 / 3.0 + np.outer(u, u))
        Pexp = Pin - (1.0 - beta) / tau * (Pin - Peq) + beta * dV
        assert np.allclose(Pout, Pexp, rtol=0, atol=4e-16 * len(w))
        # uncovered: plain BGK relaxation by 1/tau
        fout, _ = O.collide_node(dim, tau, [0, 0, 0], S, fin, 0, vs)
        Pout = np.einsum("i,ia,ib->ab", fout, c3, c3)
        assert np.allclose(Pout, Pin - (Pin - Peq) / tau, rtol=0, atol=4e-16 * len(w))
