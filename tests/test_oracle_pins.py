"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
conservation laws, brute force on tiny inputs, exact rational arithmetic, or
special cases with a known answer.  No test retypes an oracle formula.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1011_2613_amd import inputs as I


# ------------------------------------------------------------------ helpers
def lattice(dim):
    c, w = O.velocities(dim)
    c3 = np.zeros((len(w), 3))
    c3[:, :dim] = c
    return c3, w


def fluid_momentum(sim):
    """Total fluid momentum and mass, summed exactly (math.fsum) then rounded."""
    f = sim.get_f().reshape(sim.Q, -1)
    c3, _ = lattice(sim.dim)
    P = np.array([math.fsum((c3[:, a:a + 1] * f).ravel()) for a in range(3)])
    return P, math.fsum(f.ravel())


def particle_mass(dim, R, rho):
    return rho * (math.pi * R * R if dim == 2 else 4.0 / 3.0 * math.pi * R ** 3)


# ---------------------------------------------------------- lattice moments
@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments_closed_form(dim):
    """Sum f^eq = rho, sum f^eq c = rho u, sum f^eq c c = rho (I/3 + u u)."""
    rng = np.random.default_rng(11 + dim)
    c3, _ = lattice(dim)
    for _ in range(20):
        rho = 1.0 + 0.05 * rng.standard_normal()
        u = np.zeros(3)
        u[:dim] = 0.05 * rng.standard_normal(dim)
        fe = O.feq(dim, rho, u)
        assert abs(fe.sum() - rho) <= 4e-16 * rho * len(fe)
        assert np.allclose(fe @ c3, rho * u, rtol=0, atol=1e-16 * len(fe))
        P = np.einsum("i,ia,ib->ab", fe, c3, c3)
        Pexp = rho * (np.eye(3) / 3.0 + np.outer(u, u))
        if dim == 2:
            Pexp[2, :] = 0.0
            Pexp[:, 2] = 0.0
        assert np.allclose(P, Pexp, rtol=0, atol=2e-16 * len(fe))


def test_lattice_isotropy_fourth_moment():
    """Weights give sum w c_a c_b c_c c_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9."""
    for dim in (2, 3):
        c, w = O.velocities(dim)
        T = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
        d = np.eye(dim)
        E = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
             + np.einsum("ad,bc->abcd", d, d)) / 9.0
        assert np.allclose(T, E, atol=1e-15)


# ---------------------------------------------------------------- beta, Eq. 2
def test_beta_special_values():
    """beta(0) = 0, beta(1) = 1 for any tau; increasing in eps; hand values."""
    for tau in (0.51, 0.55, 0.6, 1.0, 2.0):
        assert O.beta(0.0, tau) == 0.0
        assert O.beta(1.0, tau) == 1.0
        vals = [O.beta(e / 64.0, tau) for e in range(65)]
        assert all(b > a for a, b in zip(vals, vals[1:]))
    # tau = 1: beta(1/2) = (1/2 * 1/2) / (1/2 + 1/2) = 1/4
    assert O.beta(0.5, 1.0) == 0.25
    # tau = 1.5: beta(1/4) = (1/4) / (3/4 + 1) = 1/7
    assert abs(O.beta(0.25, 1.5) - 1.0 / 7.0) <= 1e-16


# ------------------------------------------------------------------- Sum2
def test_sum2_against_exact_rational_sum():
    """Compensated sum equals the correctly rounded exact sum (ill-conditioned data)."""
    rng = np.random.default_rng(5)
    mismatches = 0
    for trial in range(300):
        n = int(rng.integers(2, 800))
        p = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        p = np.concatenate([p, -p[: n // 2] * (1 + 1e-9 * rng.standard_normal(n // 2))])
        rng.shuffle(p)
        exact = float(sum(Fraction(float(x)) for x in p))
        got = O.sum2(p)
        if got != exact:
            mismatches += 1
            assert abs(got - exact) <= 2.3e-16 * abs(exact) + 1e-300
    assert mismatches <= 3


# --------------------------------------------------- single-node IMB identities
@pytest.mark.parametrize("dim", [2, 3])
def test_node_collision_moments(dim):
    """Mass is conserved; momentum gains q + rho g; q = beta rho (V_S - u).

    The last identity follows from the solid collision operator: summing
    Omega_i c_i over the lattice leaves rho (V_S - u) because the lattice's
    velocity set is symmetric (c_{-i} = -c_i) and f^eq carries momentum rho u.
    """
    rng = np.random.default_rng(20 + dim)
    c3, w = lattice(dim)
    S = 4
    Smax = S ** dim
    tau = 0.6
    for trial in range(200):
        fin = w * (1.0 + 0.05 * rng.standard_normal(len(w)))
        count = int(rng.integers(0, Smax + 30))
        vs = np.zeros(3)
        vs[:dim] = 0.02 * rng.standard_normal(dim)
        g = np.zeros(3)
        g[:dim] = 1e-4 * rng.standard_normal(dim)
        fout, q = O.collide_node(dim, tau, g, S, fin, count, vs)
        rho = fin.sum()
        u = (fin @ c3) / rho
        eps = min(count, Smax) / Smax
        beta = eps * (tau - 0.5) / ((1 - eps) + (tau - 0.5))
        assert abs(fout.sum() - rho) <= 1e-15 * len(w)
        qexp = beta * rho * (vs - u) if count > 0 else np.zeros(3)
        assert np.allclose(q, qexp, rtol=1e-12, atol=1e-17)
        assert np.allclose(fout @ c3 - fin @ c3, q + rho * g, rtol=0, atol=1e-16 * len(w))


@pytest.mark.parametrize("dim", [2, 3])
def test_full_cover_takes_solid_velocity(dim):
    """eps = 1 gives beta = 1: the node's post-collision momentum is rho V_S."""
    rng = np.random.default_rng(3)
    c3, w = lattice(dim)
    for _ in range(20):
        fin = w * (1.0 + 0.05 * rng.standard_normal(len(w)))
        vs = np.zeros(3)
        vs[:dim] = 0.02 * rng.standard_normal(dim)
        fout, _ = O.collide_node(dim, 0.8, [0, 0, 0], 4, fin, 4 ** dim, vs)
        assert np.allclose(fout @ c3, fin.sum() * vs, atol=1e-16)


# ------------------------------------------------------------ footprint (eps)
def brute_counts(dim, box, xp, R, S):
    """Count sample points of every node inside the particle, by brute force."""
    offs = (np.arange(S) + 0.5) / S - 0.5
    shape = box[:dim]
    counts = np.zeros(tuple(reversed(shape)), dtype=int)
    axes = [np.arange(n) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    for idx in np.ndindex(*([S] * dim)):
        d2 = np.zeros(grids[0].shape)
        for a in range(dim):
            d = grids[a] - xp[a]
            d = np.where(d > box[a] / 2, d - box[a], np.where(d < -box[a] / 2, d + box[a], d))
            d = d + offs[idx[a]]
            d2 = d2 + d * d
        inside = d2 <= R * R
        counts += inside.T
    return counts


@pytest.mark.parametrize("dim,S,R", [(2, 8, 6.0), (2, 3, 2.5), (3, 4, 4.0), (3, 2, 3.0)])
def test_footprint_counts_brute_force(dim, S, R):
    rng = np.random.default_rng(int(R * 10) + dim)
    box = [24, 22, 20][:dim]
    sim = O.OracleSim(dim, box, 0.7, samples=S)
    for _ in range(4):
        xp = np.zeros(3)
        xp[:dim] = rng.uniform(0, 1, dim) * np.array(box)
        sim.set_particles(xp[None], radius=[R], rho_s=[2.0])
        got = sim.footprint_counts()
        exp = brute_counts(dim, box, xp, R, S)
        assert np.array_equal(got, exp)
        vol = math.pi * R * R if dim == 2 else 4.0 / 3.0 * math.pi * R ** 3
        assert abs(got.sum() / S ** dim - vol) / vol < 0.03


def test_footprint_translation_invariance():
    """An integer shift of the particle shifts its count pattern exactly."""
    box = [32, 30]
    sim = O.OracleSim(2, box, 0.7, samples=8)
    xp = np.array([10.37, 11.81, 0.0])
    sim.set_particles(xp[None], radius=[6.0], rho_s=[2.0])
    a = sim.footprint_counts()
    sim.set_particles((xp + [3, -2, 0])[None], radius=[6.0], rho_s=[2.0])
    b = sim.footprint_counts()
    assert np.array_equal(np.roll(np.roll(a, 3, axis=1), -2, axis=0), b)


def test_footprint_disc_area_converges():
    """eps summed over nodes approaches pi R^2 as the sampling is refined."""
    box = [40, 40]
    errs = []
    for S in (2, 4, 8, 16):
        sim = O.OracleSim(2, box, 0.7, samples=S)
        sim.set_particles(np.array([[19.3, 20.6, 0.0]]), radius=[7.0], rho_s=[1.0])
        errs.append(abs(sim.footprint_counts().sum() / S ** 2 - math.pi * 49.0))
    assert errs[-1] < errs[0]
    assert errs[-1] / (math.pi * 49.0) < 2e-3


# --------------------------------------------------- conservation over a run
@pytest.mark.parametrize("dim", [2, 3])
def test_mass_and_momentum_balance(dim):
    """Fully periodic box with free particles, fluid force and particle gravity:
    total mass is constant and fluid + particle momentum grows by exactly
    M g_f + sum_p m_p a_p per step (the IMB momentum exchange and the DEM pair
    forces cancel between fluid and particles)."""
    box = [40, 36] if dim == 2 else [20, 18, 16]
    R = 4.0 if dim == 2 else 3.0
    gf = np.array([2e-5, -1e-5, 0.5e-5 if dim == 3 else 0.0])
    ap = np.array([0.0, -3e-5, 0.0])
    sim = O.OracleSim(dim, box, 0.65, fluid_force=gf, particle_accel=ap,
                      samples=4, kn=200.0, restitution=0.8)
    pos = np.array([[10.0, 10.0, 8.0], [17.9, 10.4, 8.2], [25.0, 25.0, 4.0]])[:, :]
    if dim == 2:
        pos[:, 2] = 0.0
    else:
        pos = np.array([[5.0, 5.0, 8.0], [10.9, 5.3, 8.1], [14.0, 13.0, 3.0]])
    vel = np.array([[0.01, 0.0, 0.0], [-0.01, 0.002, 0.0], [0.0, 0.0, 0.0]])
    om = np.array([[0.0, 0.0, 1e-3], [0.0, 0.0, -2e-3], [0.0, 0.0, 0.0]])
    if dim == 3:
        om[:, 0] = [1e-3, 0.0, -1e-3]
    rho_s = np.array([3.0, 3.0, 3.0])
    sim.set_particles(pos, vel, om, [R] * 3, rho_s)
    m = particle_mass(dim, R, rho_s)
    P0, M0 = fluid_momentum(sim)
    _, v, _ = sim.particles()
    Pp0 = (m[:, None] * v).sum(axis=0)
    saw_contact = False
    for step in range(60):
        sim.step(1)
        P1, M1 = fluid_momentum(sim)
        _, v, _ = sim.particles()
        Pp1 = (m[:, None] * v).sum(axis=0)
        saw_contact |= bool(np.any(sim.contact_forces() != 0.0))
        expect = M0 * gf + (m[:, None] * ap).sum(axis=0)
        if dim == 2:
            expect[2] = 0.0
        # rounding floor: one ulp of every population per step, eps * total mass
        assert abs(M1 - M0) <= 1e-15 * M0
        assert np.allclose((P1 + Pp1) - (P0 + Pp0), expect, rtol=0, atol=2e-16 * M0)
        P0, M0, Pp0 = P1, M1, Pp1
    assert saw_contact


@pytest.mark.parametrize("wall", [False, True])
def test_rest_state_is_exact(wall):
    """No forces and particles at rest: the fluid stays at f^eq(1,0), the
    hydrodynamic forces vanish and the particles do not move -- up to rounding
    only (the rounded weights sum to 1 + 2^-52, so rho = 1 is not exact)."""
    sim = O.OracleSim(2, [30, 28], 0.6, wall_y=wall, samples=4, kn=100.0)
    pos = np.array([[8.2, 9.7, 0.0], [20.5, 17.1, 0.0]])
    sim.set_particles(pos, radius=[4.0, 3.5], rho_s=[5.0, 5.0])
    f0 = sim.get_f()
    sim.step(40)
    assert np.abs(sim.get_f() - f0).max() < 1e-15
    _, u = sim.macro()
    assert np.abs(u).max() < 1e-15
    F, T = sim.forces()
    assert np.abs(F).max() < 1e-14 and np.abs(T).max() < 1e-13
    x, v, w = sim.particles()
    assert np.abs(x - pos).max() < 1e-14 and np.abs(v).max() < 1e-16


def test_moving_particle_feels_drag():
    """A disc moving through quiescent fluid is decelerated (force opposes
    motion) and the fluid gains momentum along the motion."""
    sim = O.OracleSim(2, [48, 40], 0.7, samples=4)
    sim.set_particles(np.array([[20.0, 20.0, 0.0]]), vel=[[0.01, 0.0, 0.0]], radius=[5.0],
                      rho_s=[4.0])
    sim.step(5)
    F, _ = sim.forces()
    assert F[0, 0] < 0.0 and abs(F[0, 1]) < 1e-3 * abs(F[0, 0])
    P, _ = fluid_momentum(sim)
    assert P[0] > 0.0


def test_mirror_symmetry():
    """A configuration mirrored in x gives the mirrored flow and forces."""
    box = [36, 30]
    def run(mirror):
        sim = O.OracleSim(2, box, 0.7, wall_y=True, fluid_force=[0.0, -1e-5], samples=4, kn=100.0)
        xs = np.array([10.3, 21.9])
        if mirror:
            xs = (box[0] - 1) - xs
        pos = np.array([[xs[0], 9.4, 0.0], [xs[1], 15.2, 0.0]])
        vel = np.array([[0.004, 0.001, 0.0], [-0.003, 0.0, 0.0]]) * ([-1, 1, 1] if mirror else 1)
        sim.set_particles(pos, vel, radius=[4.0, 4.0], rho_s=[3.0, 3.0])
        sim.step(30)
        return sim.macro(), sim.forces(), sim.particles()
    (r0, u0), (F0, T0), (x0, v0, w0) = run(False)
    (r1, u1), (F1, T1), (x1, v1, w1) = run(True)
    assert np.allclose(r0, r1[:, ::-1], rtol=0, atol=1e-13)
    assert np.allclose(u0[0], -u1[0][:, ::-1], rtol=0, atol=1e-13)
    assert np.allclose(u0[1], u1[1][:, ::-1], rtol=0, atol=1e-13)
    assert np.allclose(F0[:, 0], -F1[:, 0], atol=1e-14)
    assert np.allclose(F0[:, 1], F1[:, 1], atol=1e-14)
    assert np.allclose(T0[:, 2], -T1[:, 2], atol=1e-14)


# ----------------------------------------------------------- Poiseuille (P4)
def poiseuille(N, tau, g):
    """Steady body-force channel flow between halfway bounce-back walls with the
    simple forcing F_i = 3 w_i rho c_i.g and u = sum f c / rho:
    u(j) = g/(2 nu) (j + 1/2)(N - 1/2 - j) + g (16 tau^2 - 20 tau + 3) / (4 (2 tau - 1))."""
    nu = (tau - 0.5) / 3.0
    j = np.arange(N)
    return g / (2 * nu) * (j + 0.5) * (N - 0.5 - j) + g * (16 * tau * tau - 20 * tau + 3) / (4 * (2 * tau - 1))


@pytest.mark.parametrize("dim,N,tau", [(2, 12, 1.0), (2, 10, 0.6), (2, 8, 1.7), (3, 12, 0.8), (3, 9, 0.55)])
def test_poiseuille_closed_form(dim, N, tau):
    g = 1e-6
    shape = [1, N] if dim == 2 else [1, N, 1]
    sim = O.OracleSim(dim, shape, tau, wall_y=True, fluid_force=[g, 0, 0])
    nu = (tau - 0.5) / 3.0
    steps = int(40 * N * N / (math.pi ** 2 * nu)) + 200
    sim.step(steps)
    _, u = sim.macro()
    ux = u[0].reshape(-1)
    exp = poiseuille(N, tau, g)
    assert np.allclose(ux, exp, rtol=1e-10, atol=0)
    # transverse velocity is a rounding mode only
    assert np.abs(u[1]).max() < 1e-8 * np.abs(exp).max()


# ------------------------------------------------- periodic-array drag (P5)
def test_hasimoto_square_array_drag_2d():
    """Stokes drag on a fixed disc in a square periodic array (Hasimoto 1959,
    Sangani & Acrivos 1982): F / (rho nu U) = 4 pi / (-ln(c)/2 - 0.738 + c - 0.887 c^2),
    c the solid area fraction, U the superficial velocity.  At steady state the
    drag also balances the total body force on the fluid exactly."""
    L, R, tau, g = 40, 5.0, 1.0, 1e-7
    sim = O.OracleSim(2, [L, L], tau, fluid_force=[g, 0.0], samples=8)
    sim.set_particles(np.array([[19.5, 19.5, 0.0]]), radius=[R], rho_s=[1.0], fixed=[1])
    sim.step(12000)
    rho, u = sim.macro()
    F, _ = sim.forces()
    nu = (tau - 0.5) / 3.0
    mass = rho.sum()
    assert abs(F[0, 0] - g * mass) / (g * mass) < 1e-5
    U = (rho * u[0]).sum() / L ** 2
    c = math.pi * R * R / L ** 2
    K_th = 4 * math.pi / (-0.5 * math.log(c) - 0.738 + c - 0.887 * c * c)
    K = F[0, 0] / (nu * U)
    assert abs(K - K_th) / K_th < 0.05


@pytest.mark.slow
def test_hasimoto_cubic_array_drag_3d():
    """Stokes drag on a fixed sphere in a simple cubic periodic array (Hasimoto 1959):
    F / (6 pi rho nu R U) = 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2)."""
    L, R, tau, g = 32, 4.0, 1.0, 1e-7
    sim = O.OracleSim(3, [L, L, L], tau, fluid_force=[g, 0.0, 0.0], samples=4)
    sim.set_particles(np.array([[15.5, 15.5, 15.5]]), radius=[R], rho_s=[1.0], fixed=[1])
    sim.step(1500)
    rho, u = sim.macro()
    F, _ = sim.forces()
    nu = (tau - 0.5) / 3.0
    U = (rho * u[0]).sum() / L ** 3
    c = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
    K_th = 1.0 / (1 - 1.7601 * c ** (1 / 3) + c - 1.5593 * c * c)
    K = F[0, 0] / (6 * math.pi * nu * R * U)
    assert abs(K - K_th) / K_th < 0.08


# ----------------------------------------------------------------- DEM (P6)
def contact_recurrence(delta0, w0, k, eta, meff, n):
    """Symplectic-Euler map of a linear spring-dashpot contact, w the approach
    speed and delta the overlap:  w' = w - (k delta + eta w)/m_eff,
    delta' = delta + w'."""
    M = np.array([[1 - k / meff, 1 - eta / meff], [-k / meff, 1 - eta / meff]])
    return np.linalg.matrix_power(M, n) @ np.array([delta0, w0])


@pytest.mark.parametrize("tc", [10.0, 40.0, 160.0])
def test_dem_head_on_pair(tc):
    e = 0.9
    R, rho = 5.0, 1.0
    m = rho * math.pi * R * R
    meff = m / 2
    le = math.log(e)
    k = (math.pi ** 2 + le ** 2) * meff / tc ** 2
    eta = -2 * le * math.sqrt(meff * k) / math.sqrt(math.pi ** 2 + le ** 2)
    sim = O.OracleSim(2, [80, 24], 0.7, samples=2, kn=k, restitution=e)
    sim.set_coupling(False)
    v0 = 0.03
    sim.set_particles(np.array([[30.0, 12.0, 0.0], [40.5, 12.0, 0.0]]),
                      vel=[[v0, 0, 0], [-v0, 0, 0]], radius=[R, R], rho_s=[rho, rho])
    traj = []
    for _ in range(int(3 * tc) + 60):
        x, v, _ = sim.particles()
        traj.append((x[1, 0] - x[0, 0], v[0, 0] - v[1, 0]))
        sim.step(1)
    traj = np.array(traj)
    s, w = traj[:, 0], traj[:, 1]
    first = int(np.argmax(2 * R - s > 0))
    last = first + int(np.argmax(2 * R - s[first:] <= 0))
    for n in range(first, last):
        got = np.array([2 * R - s[n], w[n]])
        exp = contact_recurrence(2 * R - s[first], w[first], k, eta, meff, n - first)
        assert np.allclose(got, exp, rtol=1e-9, atol=1e-12)
    e_eff = -w[last + 1] / w[first - 1]
    # symplectic Euler converges to the continuous restitution as tc grows
    assert abs(e_eff - e) < 3.0 / tc
    assert abs((last - first) - tc) <= 0.1 * tc + 2
    # momentum of the pair is conserved exactly by the antisymmetric force
    x, v, _ = sim.particles()
    assert abs(v[0, 0] + v[1, 0]) < 1e-17


def test_dem_wall_bounce():
    """A disc falling onto the lower wall plane y = -1/2 rebounds with the
    same recurrence as a pair, with m_eff = m."""
    e, R, rho, tc = 0.9, 4.0, 2.0, 40.0
    m = rho * math.pi * R * R
    le = math.log(e)
    k = (math.pi ** 2 + le ** 2) * m / tc ** 2
    sim = O.OracleSim(2, [24, 40], 0.7, wall_y=True, samples=2, kn=k, restitution=e)
    sim.set_coupling(False)
    sim.set_particles(np.array([[12.0, 4.0, 0.0]]), vel=[[0, -0.02, 0]], radius=[R], rho_s=[rho])
    ys, vs = [], []
    for _ in range(200):
        x, v, _ = sim.particles()
        ys.append(x[0, 1]); vs.append(v[0, 1])
        sim.step(1)
    ys, vs = np.array(ys), np.array(vs)
    assert ys.min() > -0.5  # never passes the wall plane
    assert vs[-1] > 0 and abs(vs[-1] / 0.02 - e) < 3.0 / tc


def test_dem_forces_pairs_antisymmetric_and_periodic():
    """Pair forces are equal and opposite bitwise, also across a periodic seam."""
    x = np.array([[0.5, 5.0, 0.0], [15.8, 5.2, 0.0], [8.0, 1.0, 0.0]])
    v = np.array([[0.01, 0.0, 0.0], [-0.02, 0.003, 0.0], [0.0, 0.0, 0.0]])
    Fc = O.dem_forces(2, x, v, [1.0, 1.0, 1.0], [3.0, 5.0, 4.0], 50.0, 0.9, [16.0, 16.0])
    assert Fc[0, 0] > 0  # particle 0 is pushed away from 1 across the seam (+x)
    assert np.array_equal(Fc[0], -Fc[1])
    assert np.all(Fc[2] == 0.0)


# -------------------------------------------------------- input generators
def test_placement_non_overlapping_and_in_bounds():
    for dim, box, wall in ((2, (64, 48), True), (3, (24, 30, 20), True), (2, (40, 40), False)):
        pos = I.place_particles(dim, box, 3.0, 20, seed=7, wall_y=wall)
        for i in range(len(pos)):
            for j in range(i):
                d = pos[i] - pos[j]
                for a in range(dim):
                    if not (wall and a == 1):
                        d[a] -= box[a] * round(d[a] / box[a])
                assert np.linalg.norm(d[:dim]) > 6.0
        if wall:
            assert np.all(pos[:, 1] >= -0.5 + 3.0) and np.all(pos[:, 1] <= box[1] - 0.5 - 3.0)


def test_splitmix64_reference_vector():
    """First outputs of SplitMix64 seeded with 0 (published reference values)."""
    out = I.splitmix64(0, 0, 2)
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


# ------------------------------------------------ Table 2 printed values
def _table2():
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_dem.txt")
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                vals[line[0]] = (float(line[1]), float(line[2]))
    return vals


@pytest.mark.parametrize("col,dim", [(0, 2), (1, 3)])
def test_table2_masses_and_contact_time(col, dim):
    """The oracle fed with Table 2's solid density, diameter, stiffness and
    restitution: (i) its particle mass (disc of unit depth in 2D, sphere in
    3D) reproduces the printed mass, seen through the duration of a head-on
    contact, which must match the printed contact-time formula (about 10
    steps) to within one step; (ii) the pair rebounds with a restitution near
    the printed 0.9 (symplectic Euler at 10 steps per contact)."""
    t = _table2()
    rho, d, m_print, k, e = (t[n][col] for n in ("rho_s", "d", "m_s", "k_n", "e"))
    R = d / 2
    m_formula = rho * (math.pi * R * R if dim == 2 else 4.0 / 3.0 * math.pi * R ** 3)
    assert abs(m_formula - m_print) / m_print < 5e-5          # printed to 5 digits
    tc = math.sqrt((math.pi ** 2 + math.log(e) ** 2) * (m_print / 2) / k)
    assert abs(tc - 10.0) < 0.01
    shape = [60, 24] if dim == 2 else [60, 24, 24]
    sim = O.OracleSim(dim, shape, 0.7, samples=1, kn=k, restitution=e)
    sim.set_coupling(False)
    v0 = 0.05
    z = 12.0 if dim == 3 else 0.0
    sim.set_particles(np.array([[20.0, 12.0, z], [30.6, 12.0, z]]), vel=[[v0, 0, 0], [-v0, 0, 0]],
                      radius=[R, R], rho_s=[rho, rho])
    gaps, rel = [], []
    for _ in range(60):
        x, v, _ = sim.particles()
        gaps.append(x[1, 0] - x[0, 0] - d)
        rel.append(v[0, 0] - v[1, 0])
        sim.step(1)
    gaps = np.array(gaps)
    contact = np.nonzero(gaps < 0)[0]
    assert len(contact) > 0
    steps_in_contact = contact[-1] - contact[0] + 1
    assert abs(steps_in_contact - tc) <= 1.0
    e_eff = -rel[-1] / rel[0]
    assert abs(e_eff - e) < 0.01


# ---------------------------------------------- eps by table lookup (Eq. 6)
def _fine_coverage(dim, R, d, M=32):
    """Coverage of the unit cell at displacement d from the centre by M^D
    points, written out here (not the oracle's sampling routine)."""
    o = (np.arange(M) + 0.5) / M - 0.5
    if dim == 2:
        X, Y = np.meshgrid(d[0] + o, d[1] + o, indexing="ij")
        return float(((X * X + Y * Y) <= R * R).mean())
    X, Y, Z = np.meshgrid(d[0] + o, d[1] + o, d[2] + o, indexing="ij")
    return float(((X * X + Y * Y + Z * Z) <= R * R).mean())


@pytest.mark.parametrize("dim,S", [(2, 8), (3, 4)])
def test_eps_table_planar_limit(dim, S):
    """For a radius much larger than the cell the surface is a plane: a cell
    at signed distance rho along an axis is covered 1/2 - rho, along the 2D
    diagonal (1/sqrt(2) - rho)^2 ... (piecewise quadratic).  The table is
    within its bin width plus its reference resolution (1/16) of that."""
    R = 1000.0
    Smax = S ** dim
    for rho in np.linspace(-0.48, 0.48, 25):
        d = [R + rho, 0.0, 0.0]
        cov = O.eps_table_count(dim, S, R, d) / Smax
        assert abs(cov - (0.5 - rho)) <= 0.05, (rho, cov)
    if dim == 2:
        for rho in np.linspace(-0.68, 0.68, 25):
            u = (R + rho) / math.sqrt(2.0)
            cov = O.eps_table_count(2, S, R, [u, u]) / Smax
            s = -rho      # cell points with n.x <= s are inside
            h = 1.0 / math.sqrt(2.0)
            exact = (s + h) ** 2 if s <= 0 else 1.0 - (h - s) ** 2
            assert abs(cov - exact) <= 0.06, (rho, cov, exact)


@pytest.mark.parametrize("dim,S,R", [(2, 8, 6.0), (3, 4, 4.0)])
def test_eps_table_total_volume(dim, S, R):
    """The counts of all nodes around a particle add up to its area/volume
    (pi R^2, 4/3 pi R^3) within 1 %."""
    c = np.array([0.37, -0.21, 0.13])[:dim]
    n = int(R) + 2
    tot = 0
    rng = range(-n, n + 1)
    for ix in rng:
        for iy in rng:
            for iz in (rng if dim == 3 else [0]):
                d = np.array([ix, iy, iz][:dim], dtype=float) - c
                tot += O.eps_table_count(dim, S, R, list(d))
    vol = tot / S ** dim
    exact = math.pi * R * R if dim == 2 else 4.0 / 3.0 * math.pi * R ** 3
    assert abs(vol - exact) / exact < 0.01, (vol, exact)


@pytest.mark.parametrize("dim,S,R", [(2, 8, 5.0), (3, 4, 4.0)])
def test_eps_table_vs_fine_coverage(dim, S, R):
    """Near the surface the table agrees with a 32^D-point coverage within
    0.06 per node and 0.01 on average: half a rho bin (sqrt(D)/64) times the
    slope of the coverage, the 1/16 reference grid and the rounding to the
    S^D scale bound it.  Sub-cell sampling with S points per axis is printed
    beside it for comparison."""
    rs = np.random.default_rng(3)
    et, es = [], []
    sim = O.OracleSim(dim, [32] * dim, 0.8, samples=S)
    for _ in range(150):
        u = rs.normal(size=dim)
        u /= np.linalg.norm(u)
        d = u * (R + rs.uniform(-0.85, 0.85))
        fine = _fine_coverage(dim, R, d)
        tab = O.eps_table_count(dim, S, R, list(d)) / S ** dim
        c = (16.0 - d) if dim == 3 else np.append(16.0 - d, 0.0)
        sim.set_particles([list(c)], radius=[R], rho_s=[1.0])
        smp = sim.particle_node_count(0, 16, 16, 16 if dim == 3 else 0) / S ** dim
        et.append(abs(tab - fine))
        es.append(abs(smp - fine))
    sim.close()
    print("eps error vs 32^D coverage: table mean %.4f max %.4f, sampling mean %.4f max %.4f"
          % (np.mean(et), np.max(et), np.mean(es), np.max(es)))
    assert max(et) <= 0.06 and np.mean(et) <= 0.01
