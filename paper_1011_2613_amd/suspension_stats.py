"""Time series of the suspension-wide statistics of a workload ("Simulation
results": the temporal evolution of the area-averaged inter-phase slip velocity
V_ry and drag force F_dy, Figs. 5 and 7), read from the library with
lbm_get_stats every `every` steps.

    python -m paper_1011_2613_amd.suspension_stats --workload P2 --steps 3000 \
        --every 100 --out series.json

Each record holds the time step, the fluid-phase and particle-phase mean
velocities, their difference (the slip velocity), the mean hydrodynamic force
per particle (the drag), the total fluid mass and the solid fraction, in
lattice units; `velocity_scale` converts lattice velocities to m/s with the
paper's lattice spacing and time step (Table 2), and `drag_scale` forces to
newtons per particle (per metre of depth in 2D).
"""
import argparse
import json
import sys
import time

from . import binding
from . import inputs as I

# Table 2: lattice spacing 7.5e-6 m; time step 3e-7 s (2D) / 6e-7 s (3D);
# gas density 1.3 kg/m^3 is the lattice density 1
LATTICE_M = 7.5e-6
STEP_S = {2: 3e-7, 3: 6e-7}
GAS_KG_M3 = 1.3


def series(workload, steps, every, storage="fp64", log=None, block=None):
    """Runs `workload` from its seeded initial state for `steps` steps and
    returns the lbm_get_stats records taken every `every` steps (and at 0)."""
    w = I.workload(workload)
    sim = binding.simulation_for(w, storage)
    if block is not None:
        sim.set_lattice_block(*block)
    recs = []
    t0 = time.perf_counter()

    def take():
        st = sim.stats()
        rec = {"t": int(st["t"]), "mass": float(st["mass"]), "solid_fraction": float(st["solid_fraction"]),
               "fluid_velocity": [float(x) for x in st["fluid_velocity"]],
               "particle_velocity": [float(x) for x in st["particle_velocity"]],
               "slip_velocity": [float(x) for x in st["slip_velocity"]],
               "mean_drag": [float(x) for x in st["mean_drag"]]}
        recs.append(rec)
        if log:
            log("t=%d slip_y %.4e drag_y %.4e mass %.15g (%.1f s)"
                % (rec["t"], rec["slip_velocity"][1], rec["mean_drag"][1], rec["mass"],
                   time.perf_counter() - t0))

    take()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        sim.step(k)
        done += k
        take()
    sim.close()
    dim = w.dim
    vscale = LATTICE_M / STEP_S[dim]
    # force in lattice units: rho_lattice l^D / dt^2 (per unit depth in 2D)
    fscale = GAS_KG_M3 * LATTICE_M ** dim / STEP_S[dim] ** 2
    return {"workload": w.name, "storage": storage, "nodes": w.nodes, "particles": w.count,
            "steps": steps, "every": every, "velocity_scale": vscale, "drag_scale": fscale,
            "records": recs}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="P2")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--storage", default="fp64", choices=["fp64", "fp32s", "fp16s"])
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    out = series(args.workload, args.steps, args.every, args.storage,
                 log=lambda *a: print(*a, flush=True))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    main()
    sys.exit(0)
