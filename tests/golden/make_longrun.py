"""Write long-run FP64 reference data for the full-size suspension workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators
(paper_1011_2613_amd/inputs.py, which hold none of the method's arithmetic).
The oracle runs with every host core; its threaded loops give the serial
program's results bit for bit (tests/test_oracle_threads.py).

    python tests/golden/make_longrun.py C3 2000
    python tests/golden/make_longrun.py C2 5000

writes tests/golden/longrun_<workload>_<steps>.npz holding:

  every CHECK steps (and at the end)
    cp_step            step index t
    cp_mass            total fluid mass sum_n sum_i f_i
    cp_fluid_mom[3]    total fluid momentum sum_n sum_i c_i f_i
    cp_x/v/w/F/T/Fc    state, hydrodynamic force and torque, contact force of
                       SAMPLE_P seeded particles (indices in cp_pidx)
  at the end
    x, v, w, F, T, Fc  every particle
    node_idx           seeded node sample (flat index x + nx (y + ny z)):
                       SAMPLE_N uniform nodes plus the bounding boxes of four
                       seeded particles at their final positions
    node_f[Q, k]       pre-collision populations f(x, t) at those nodes
    node_rho, node_u   their moments (u = sum f c / rho)
  meta: workload, steps, threads, host cores, oracle seconds per step
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1011_2613_amd import inputs as I  # noqa: E402

CHECK = 100
SAMPLE_P = 64
SAMPLE_N = 4096
SEED_P, SEED_N = 0x5A3D, 0x9A1E


def particle_sample(n):
    """SAMPLE_P distinct seeded particle indices (sorted)."""
    u = I.uniform(SEED_P, 0, 4 * SAMPLE_P)
    idx = []
    for k in (u * n).astype(np.int64):
        if k not in idx:
            idx.append(int(k))
        if len(idx) == min(SAMPLE_P, n):
            break
    return np.array(sorted(idx), dtype=np.int64)


def node_sample(w, x_final):
    nx, ny = w.shape[0], w.shape[1]
    nz = w.shape[2] if w.dim == 3 else 1
    N = nx * ny * nz
    idx = set((I.uniform(SEED_N, 0, SAMPLE_N) * N).astype(np.int64).tolist())
    # bounding boxes (radius + 1 node) of four seeded particles
    for p in (I.uniform(SEED_N + 1, 0, 4) * w.count).astype(np.int64):
        c = x_final[p]
        r = int(np.ceil(w.radius)) + 1
        rng = [range(int(np.floor(c[a])) - r, int(np.floor(c[a])) + r + 2) for a in range(w.dim)]
        zs = rng[2] if w.dim == 3 else [0]
        for z in zs:
            for y in rng[1]:
                if w.wall_y and not (0 <= y < ny):
                    continue
                for x in rng[0]:
                    idx.add((x % nx) + nx * ((y % ny) + ny * (z % nz)))
    return np.array(sorted(idx), dtype=np.int64)


def lattice_c(dim):
    c, _ = O.velocities(dim)
    c3 = np.zeros((c.shape[0], 3))
    c3[:, :dim] = c
    return c3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("steps", type=int)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    w = I.workload(args.workload)
    threads = O.set_threads(args.threads)
    pos, vel, om, rad, rho, fixed = w.particles()
    sim = O.OracleSim(w.dim, w.shape, w.tau, wall_y=w.wall_y, fluid_force=w.fluid_force,
                      particle_accel=w.particle_accel, samples=w.samples, kn=w.kn,
                      restitution=w.restitution)
    sim.set_particles(pos, vel, om, rad, rho, fixed)
    pidx = particle_sample(w.count)
    c3 = lattice_c(w.dim)
    cp = {k: [] for k in ("step", "mass", "fluid_mom", "x", "v", "w", "F", "T", "Fc")}
    step_s = 0.0
    t = 0
    print("%s: %d steps on %d threads" % (w.name, args.steps, threads), flush=True)
    while t < args.steps:
        k = min(CHECK, args.steps - t)
        t0 = time.perf_counter()
        sim.step(k)
        step_s += time.perf_counter() - t0
        t += k
        f = sim.get_f().reshape(sim.Q, -1)
        x, v, om_, = sim.particles()
        F, T = sim.forces()
        Fc = sim.contact_forces()
        cp["step"].append(t)
        cp["mass"].append(float(f.sum()))
        cp["fluid_mom"].append([float((c3[:, a] @ f).sum()) for a in range(3)])
        for name, arr in (("x", x), ("v", v), ("w", om_), ("F", F), ("T", T), ("Fc", Fc)):
            cp[name].append(arr[pidx])
        del f
        print("  t = %d  mass %.17g  %.2f s/step" % (t, cp["mass"][-1], step_s / t), flush=True)
    x, v, om_ = sim.particles()
    F, T = sim.forces()
    Fc = sim.contact_forces()
    nidx = node_sample(w, x)
    f = sim.get_f().reshape(sim.Q, -1)
    node_f = f[:, nidx].copy()
    del f
    rho_, u_ = sim.macro()
    node_rho = rho_.reshape(-1)[nidx].copy()
    node_u = u_.reshape(w.dim, -1)[:, nidx].copy()
    del rho_, u_
    out = args.out or os.path.join(HERE, "longrun_%s_%d.npz" % (w.name, args.steps))
    np.savez_compressed(
        out, workload=w.name, steps=args.steps, threads=threads, host_cores=os.cpu_count(),
        oracle_s_per_step=step_s / args.steps, nodes=w.nodes, particles=w.count,
        cp_pidx=pidx, cp_step=np.array(cp["step"]), cp_mass=np.array(cp["mass"]),
        cp_fluid_mom=np.array(cp["fluid_mom"]),
        **{"cp_" + k: np.array(cp[k]) for k in ("x", "v", "w", "F", "T", "Fc")},
        x=x, v=v, w=om_, F=F, T=T, Fc=Fc, node_idx=nidx, node_f=node_f, node_rho=node_rho,
        node_u=node_u)
    print("wrote %s (%.1f MB, oracle %.2f s/step on %d threads)"
          % (out, os.path.getsize(out) / 1e6, step_s / args.steps, threads), flush=True)


if __name__ == "__main__":
    main()
