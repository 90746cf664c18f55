"""Seeded synthetic inputs for the LB-IMB-DEM path.

This module only draws data: random numbers (SplitMix64, Steele, Lea & Flood
2014, counter form), non-overlapping particle placements by random sequential
addition, initial particle velocities and small population perturbations.  It
holds none of the method's arithmetic and imports nothing from the library or
from the oracle; both sides receive the arrays it returns.

The workload recipes mirror the paper's suspensions: monodisperse discs of
diameter 10 (2D) or spheres (3D) at random positions, an initial random
particle velocity of magnitude 5e-3 (Section "Simulation results"), periodic
boxes or walls in y.
"""
from dataclasses import dataclass, field
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, start, count):
    """Outputs start .. start+count-1 of the SplitMix64 stream of `seed`.

    Output k is mix(seed + (k + 1) * golden) with the published mixing
    function, so any slice of the stream can be drawn independently.
    """
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, start, count):
    """Uniform doubles in [0, 1): (x >> 11) * 2^-53."""
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential reader over one SplitMix64 stream."""

    def __init__(self, seed):
        self.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.pos = 0

    def uniform(self, count):
        out = uniform(self.seed, self.pos, count)
        self.pos += count
        return out


def place_particles(dim, box, radius, count, seed, wall_y=False, max_tries=10**6):
    """Random sequential addition of `count` equal particles.

    A candidate is accepted when its distance to every accepted centre exceeds
    the sum of radii (minimum image on periodic axes) and, with walls in y, its
    clearance to the wall planes y = -1/2 and y = ny - 1/2 is at least R.
    Returns positions [count, 3] (2D: z = 0).
    """
    box = [float(b) for b in box] + [1.0] * (3 - len(box))
    R = float(radius)
    rs = Stream(seed)
    cell = 2.0 * R
    ncell = [max(1, int(box[a] // cell)) for a in range(3)]
    grid = {}
    pos = np.zeros((count, 3))
    accepted = 0
    tries = 0
    lo_y, span_y = (-0.5 + R, box[1] - 1.0 - 2.0 * R) if wall_y else (0.0, box[1])
    while accepted < count:
        tries += 1
        if tries > max_tries * max(count, 1):
            raise RuntimeError("random sequential addition did not converge")
        u = rs.uniform(3)
        c = np.array([u[0] * box[0], lo_y + u[1] * span_y, u[2] * box[2] if dim == 3 else 0.0])
        key = [int(c[a] / box[a] * ncell[a]) % ncell[a] if (a < dim) else 0 for a in range(3)]
        if wall_y:
            key[1] = min(max(int((c[1] + 0.5) / box[1] * ncell[1]), 0), ncell[1] - 1)
        ok = True
        rng = [range(-1, 2) if a < dim else range(0, 1) for a in range(3)]
        for dz in rng[2]:
            for dy in rng[1]:
                for dx in rng[0]:
                    kk = [key[0] + dx, key[1] + dy, key[2] + dz]
                    if wall_y and not (0 <= kk[1] < ncell[1]):
                        continue
                    kk = tuple(kk[a] % ncell[a] for a in range(3))
                    for j in grid.get(kk, ()):
                        d = c - pos[j]
                        for a in range(dim):
                            if wall_y and a == 1:
                                continue
                            d[a] -= box[a] * round(d[a] / box[a])
                        if float(d @ d) <= (2.0 * R) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        pos[accepted] = c
        grid.setdefault(tuple(key[a] % ncell[a] for a in range(3)), []).append(accepted)
        accepted += 1
    return pos


def random_velocities(dim, count, speed, seed):
    """Velocities of magnitude `speed` in uniformly random directions."""
    rs = Stream(seed)
    u = rs.uniform(2 * count).reshape(count, 2)
    v = np.zeros((count, 3))
    if dim == 2:
        th = 2.0 * math.pi * u[:, 0]
        v[:, 0] = np.cos(th)
        v[:, 1] = np.sin(th)
    else:
        z = 2.0 * u[:, 0] - 1.0
        ph = 2.0 * math.pi * u[:, 1]
        s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        v[:, 0] = s * np.cos(ph)
        v[:, 1] = s * np.sin(ph)
        v[:, 2] = z
    return v * speed


def perturbation(Q, N, amplitude, seed):
    """Uniform noise in [-amplitude, amplitude), shape [Q, N], counter-based."""
    return (uniform(seed, 0, Q * N).reshape(Q, N) * 2.0 - 1.0) * amplitude


def mlp_initial_params(seed, sizes=(40, 128, 128, 128, 1)):
    """Seeded Kaiming-uniform weights (bound sqrt(6 / fan_in)) and zero biases
    of the drag-closure MLP, as [[W, b], ...] with W [fan_out, fan_in]; the
    values are binary32-representable."""
    params = []
    pos = 0
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        bound = math.sqrt(6.0 / fin)
        u = uniform(seed, pos, fin * fout)
        pos += fin * fout
        W = ((u * 2.0 - 1.0) * bound).reshape(fout, fin).astype(np.float32).astype(np.float64)
        params.append([W, np.zeros(fout)])
    return params


def solid_fraction_count(dim, box, radius, phi, wall_y=False):
    """Particle count for a target solid fraction of the fluid box."""
    vol = float(np.prod(box[:dim]))
    pv = math.pi * radius ** 2 if dim == 2 else 4.0 / 3.0 * math.pi * radius ** 3
    return int(round(phi * vol / pv))


@dataclass
class Workload:
    """A named synthetic LB-IMB-DEM workload.

    `fluid_force` is the body force on the fluid, `particle_accel` the
    acceleration applied to particles (gravity with buoyancy), both in
    lattice units.
    """
    name: str
    dim: int
    shape: tuple
    tau: float
    wall_y: bool
    radius: float
    count: int
    rho_ratio: float
    samples: int
    kn: float
    restitution: float
    steps: int
    seed: int
    v0: float = 0.0
    fluid_force: tuple = (0.0, 0.0, 0.0)
    particle_accel: tuple = (0.0, 0.0, 0.0)
    fixed: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def nodes(self):
        return int(np.prod(self.shape))

    def particles(self):
        """(pos, vel, omega, radius, rho_s, fixed) arrays for this workload."""
        pos = place_particles(self.dim, self.shape, self.radius, self.count, self.seed,
                              wall_y=self.wall_y)
        n = self.count
        vel = (random_velocities(self.dim, n, self.v0, self.seed + 0x5EED)
               if self.v0 else np.zeros((n, 3)))
        om = np.zeros((n, 3))
        rad = np.full(n, float(self.radius))
        rho = np.full(n, float(self.rho_ratio))
        fixed = np.full(n, 1 if self.fixed else 0, dtype=np.uint8)
        return pos, vel, om, rad, rho, fixed


def _c2_c3_gravity(nu, rho_r, d):
    """Gravity that keeps the paper's 2D terminal particle Reynolds number.

    Table 2 gives V_t d / nu = 3.14496e-3 * 10 / 0.1231 = 0.2555 at
    nu = 0.1231, rho_r = 692.3, d = 10; Stokes-like scaling g ~ nu^2/(rho_r d^3)
    carries that Re_p over to another (nu, rho_r, d).
    """
    g_ref = 1.176e-7
    return g_ref * (nu / 0.1231) ** 2 * (692.3 / rho_r) * (10.0 / d) ** 3


def _kn_for_contact_time(dim, rho_r, radius, restitution, tc=10.0):
    """Stiffness for a contact time of `tc` steps between two equal particles.

    Table 2's stiffnesses give exactly this: sqrt((pi^2 + ln^2 e) m_eff / k)
    evaluates to 10.0 time steps in both 2D and 3D.
    """
    m = rho_r * (math.pi * radius ** 2 if dim == 2 else 4.0 / 3.0 * math.pi * radius ** 3)
    meff = 0.5 * m
    le = math.log(restitution)
    return (math.pi ** 2 + le ** 2) * meff / tc ** 2


def workload(name):
    """The named workloads.

    C1  D2Q9 256x256 periodic, tau 0.6, fluid force 1e-6 along +x, 16 discs
        R = 6 at rest, density ratio 10, 8x8 sampling, k = 1e3, e = 0.9.
    C2  D2Q9 8192x2048, periodic x, walls y, tau 0.55, discs d = 10 at solid
        fraction 0.1, density ratio 1000, gravity along -y, 8x8 sampling.
    C3  D3Q19 192x756x192, periodic x/z, walls y, tau 0.6, spheres R = 4 at
        solid fraction 0.08, density ratio 1000, gravity along -y, 4^3 sampling.
    P3  The paper's 3D suspension at full size (simulation section, Table 2
        3D column): D3Q19 512x2016x512 periodic on every axis, 129,024
        spheres d = 10 (solid fraction 0.128), nu 0.2462 (tau 1.2386),
        density ratio 692.3, gravity 4.704e-7 along -y on the particles and
        the body force 4.04e-5 along +y on the fluid that balances it,
        k = 17892, e = 0.9, initial particle speed 5e-3, 4^3 sampling.
    P2  The paper's 2D suspension at full size (simulation section, Table 2
        2D column): D2Q9 15360x61440 periodic on both axes, 1,166,400 discs
        d = 10 (solid fraction 0.097), nu 0.1231 (tau 0.8693), density ratio
        692.3, gravity 1.176e-7 along -y on the particles and the body force
        8.753e-6 along +y on the fluid that balances it, k = 2686, e = 0.9,
        initial particle speed 5e-3, 8x8 sampling.
    """
    if name == "C1":
        return Workload("C1", 2, (256, 256), 0.6, False, 6.0, 16, 10.0, 8, 1.0e3, 0.9, 1000,
                        seed=1, fluid_force=(1.0e-6, 0.0, 0.0))
    if name in ("C2", "C2dense"):
        tau, rr, d = 0.55, 1000.0, 10.0
        nu = (tau - 0.5) / 3.0
        g = _c2_c3_gravity(nu, rr, d)
        shape = (8192, 2048)
        n = 40000 if name == "C2dense" else solid_fraction_count(2, shape, 5.0, 0.1)
        return Workload(name, 2, shape, tau, True, 5.0, n, rr, 8,
                        _kn_for_contact_time(2, rr, 5.0, 0.9), 0.9, 5000, seed=2, v0=5.0e-3,
                        particle_accel=(0.0, -(1.0 - 1.0 / rr) * g, 0.0))
    if name in ("C3", "C3dense"):
        tau, rr, d = 0.6, 1000.0, 8.0
        nu = (tau - 0.5) / 3.0
        g = _c2_c3_gravity(nu, rr, d)
        shape = (192, 756, 192)
        n = 16000 if name == "C3dense" else solid_fraction_count(3, shape, 4.0, 0.08)
        return Workload(name, 3, shape, tau, True, 4.0, n, rr, 4,
                        _kn_for_contact_time(3, rr, 4.0, 0.9), 0.9, 2000, seed=3, v0=5.0e-3,
                        particle_accel=(0.0, -(1.0 - 1.0 / rr) * g, 0.0))
    if name == "P3":
        nu, rr, g = 0.2462, 692.3, 4.704e-7
        return Workload("P3", 3, (512, 2016, 512), 0.5 + 3.0 * nu, False, 5.0, 129024, rr, 4,
                        17892.0, 0.9, 2000, seed=4, v0=5.0e-3, fluid_force=(0.0, 4.04e-5, 0.0),
                        particle_accel=(0.0, -(1.0 - 1.0 / rr) * g, 0.0))
    if name == "P2":
        nu, rr, g = 0.1231, 692.3, 1.176e-7
        return Workload("P2", 2, (15360, 61440), 0.5 + 3.0 * nu, False, 5.0, 1166400, rr, 8,
                        2686.0, 0.9, 2000, seed=5, v0=5.0e-3, fluid_force=(0.0, 8.753e-6, 0.0),
                        particle_accel=(0.0, -(1.0 - 1.0 / rr) * g, 0.0))
    raise KeyError(name)
