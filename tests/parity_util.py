"""Helpers that run one scenario through the oracle and the HIP library."""
import numpy as np

from oracle import oracle as O


def rel_err(a, b):
    """max |a - b| / max |b| (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def make_pair(binding, dim, shape, tau, wall_y=False, fluid_force=(0, 0, 0),
              particle_accel=(0, 0, 0), samples=4, kn=0.0, restitution=0.9,
              particles=None, f0=None, storage="fp64", max_radius=0.0, eps="sampling"):
    """Oracle and GPU simulations with identical inputs."""
    orc = O.OracleSim(dim, shape, tau, wall_y=wall_y, fluid_force=fluid_force,
                      particle_accel=particle_accel, samples=samples, kn=kn, restitution=restitution,
                      eps=eps)
    n = 0 if particles is None else len(particles[0])
    gpu = binding.Simulation(dim, shape, tau, storage=storage, wall_y=wall_y,
                             fluid_force=fluid_force, particle_accel=particle_accel,
                             samples=samples, kn=kn, restitution=restitution,
                             max_particles=max(n, 1), max_radius=max_radius, eps=eps)
    if particles is not None and n > 0:
        orc.set_particles(*particles)
        gpu.set_particles(*particles)
    else:
        gpu.set_particles()
    if f0 is not None:
        orc.set_f(f0)
        gpu.set_f(f0)
    return orc, gpu


def compare(orc, gpu, with_f=True):
    """Relative errors of every field of the two simulations."""
    out = {}
    r0, u0 = orc.macro()
    r1, u1 = gpu.macro()
    out["rho"] = rel_err(r1 - 1.0, r0 - 1.0)
    out["u"] = rel_err(u1, u0)
    if with_f:
        out["f"] = rel_err(gpu.get_f(), orc.get_f())
    if orc.np_:
        F0, T0 = orc.forces()
        F1, T1 = gpu.forces()
        out["F"] = rel_err(F1, F0)
        out["T"] = rel_err(T1, T0)
        out["Fc"] = rel_err(gpu.contact_forces(), orc.contact_forces())
        x0, v0, w0 = orc.particles()
        x1, v1, w1 = gpu.particles()
        out["x"] = rel_err(x1, x0)
        out["v"] = rel_err(v1, v0)
        out["w"] = rel_err(w1, w0)
    return out


def seeded_f(dim, N, amplitude, seed):
    from paper_1011_2613_amd import inputs as I
    _, w = O.velocities(dim)
    Q = len(w)
    return w[:, None] * (1.0 + I.perturbation(Q, N, amplitude, seed))
