"""Resolution study: gravity-driven flow past a fixed sphere in a periodic cube.

The paper validates its LB-IMB code with a fixed sphere in a cube driven by a
body force, at particle diameters d/l = 4 ... 50 and particle Reynolds numbers
0.2 and 2 (validation section, Table 1), and reports the error of the gas
velocity falling with resolution.  The cube size and forcing of that study are
not given, so here the cube edge is L = 2.5 d (solid fraction 0.0335 at every
resolution), the sphere centre sits at the same offset (0.3, 0.3, 0.3) from a
node at every resolution, and the body force is set from the Stokes drag of a
simple cubic array (Hasimoto 1959) for the requested Reynolds number.

Each run goes to steady drag in FP64 through the library; the result is the
superficial velocity U (total fluid momentum over total mass), the drag F on
the sphere and K = F / (3 pi nu d U).  The error at each resolution is taken
against the value extrapolated from the finest three (K = K_inf + a d^-p);
Hasimoto's Stokes-limit K is listed beside it.

    python -m paper_1011_2613_amd.validation --dl 4,6,8,10,12,16,20,24,32 --re 0.2,2

(The paper goes to d/l = 50.  One sphere that large is footprinted by one
workgroup and summed by one wavefront, which are latency-bound at about 1 ms
per step for d/l = 50, so the sweep here stops at 32.)
"""
import argparse
import json
import math
import sys
import time


def hasimoto_K(c):
    """Stokes drag of a simple cubic sphere array over 3 pi mu d U
    (Hasimoto 1959, series in the solid fraction c)."""
    return 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)


def fixed_sphere(binding, dl, Re, box_ratio=2.5, tau=None, offset=0.3, check_every=None,
                 tol=1e-7, max_steps=400000, storage="fp64", log=None):
    """One steady run; returns a dict of the measured quantities.  `log`
    receives a progress line about every 20 s of a long run."""
    import torch
    d = float(dl)
    L = int(round(box_ratio * d))
    if tau is None:
        tau = 1.0 if Re <= 1.0 else 0.8
    nu = (tau - 0.5) / 3.0
    c = math.pi * d ** 3 / 6.0 / L ** 3
    K0 = hasimoto_K(c)
    U_target = Re * nu / d
    # drag = body force on every node at steady state: g L^3 = 3 pi nu d U K
    g = 3.0 * math.pi * nu * d * U_target * K0 / L ** 3
    sim = binding.Simulation(3, (L, L, L), tau, storage=storage, fluid_force=(g, 0.0, 0.0),
                             samples=4, max_particles=1, max_radius=d / 2.0)
    ctr = L // 2 + offset
    sim.set_particles([[ctr, ctr, ctr]], radius=[d / 2.0], rho_s=[1.0], fixed=[1])
    if check_every is None:
        # a few hundred checks over the slowest viscous decay time L^2 / (4 pi^2 nu)
        check_every = max(50, int(L * L / (4.0 * math.pi ** 2 * nu) / 8))
    steps, prev, F = 0, None, 0.0
    t_last = time.perf_counter()
    while steps < max_steps:
        sim.step(check_every)
        steps += check_every
        F = float(sim.forces()[0][0, 0])
        if prev is not None and abs(F - prev) <= tol * abs(F):
            break
        if log and time.perf_counter() - t_last > 20.0:
            t_last = time.perf_counter()
            log("  d/l %g Re %g: step %d, F %.8g, change %.1e" % (dl, Re, steps, F,
                                                               abs(F - prev) / abs(F) if prev else 1.0))
        prev = F
    rho, u = sim.macro_device()
    U = float((rho * u[0]).sum() / rho.sum())
    mass = float(rho.sum())
    del rho, u
    sim.close()
    torch.cuda.empty_cache()
    K = F / (3.0 * math.pi * nu * d * U)
    return {"dl": dl, "L": L, "tau": tau, "Re_target": Re, "Re": U * d / nu, "U": U, "F": F,
            "K": K, "K_hasimoto": K0, "solid_fraction": c, "steps": steps,
            "steady": steps < max_steps, "force_balance": abs(F - g * mass) / (g * mass)}


def extrapolate(ds, Ks):
    """K_inf and p of K = K_inf + a d^-p through the last three points (Aitken);
    None when the three are not monotone."""
    (d1, d2, d3), (k1, k2, k3) = ds[-3:], Ks[-3:]
    if not ((k1 - k2) * (k2 - k3) > 0):
        return None, None
    # solve for p with the three points, then K_inf
    def resid(p):
        return (k1 - k2) / (k2 - k3) - (d1 ** -p - d2 ** -p) / (d2 ** -p - d3 ** -p)
    lo, hi = 0.05, 6.0
    if resid(lo) * resid(hi) > 0:
        return None, None
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if resid(lo) * resid(mid) <= 0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    a = (k2 - k3) / (d2 ** -p - d3 ** -p)
    return k3 - a * d3 ** -p, p


def sweep(binding, dls, Res, log=None):
    out = []
    for Re in Res:
        rows = []
        for dl in dls:
            t0 = time.perf_counter()
            r = fixed_sphere(binding, dl, Re, log=log)
            r["seconds"] = round(time.perf_counter() - t0, 2)
            rows.append(r)
            if log:
                log("d/l %g Re %g: K %.5f (Hasimoto %.5f), Re %.3f, %d steps, %.1f s"
                    % (dl, Re, r["K"], r["K_hasimoto"], r["Re"], r["steps"], r["seconds"]))
        Kinf, p = extrapolate([r["dl"] for r in rows], [r["K"] for r in rows])
        for r in rows:
            r["K_extrapolated"] = Kinf
            r["order"] = p
            r["rel_err_vs_extrapolated"] = None if Kinf is None else abs(r["K"] - Kinf) / Kinf
            r["rel_err_vs_hasimoto"] = abs(r["K"] - r["K_hasimoto"]) / r["K_hasimoto"]
        out.extend(rows)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dl", default="4,6,8,10,12,16,20,24,32")
    ap.add_argument("--re", default="0.2,2")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    from paper_1011_2613_amd import binding
    binding.load()
    dls = [float(x) for x in args.dl.split(",") if x]
    Res = [float(x) for x in args.re.split(",") if x]
    rows = sweep(binding, dls, Res, log=lambda s: print(s, file=sys.stderr, flush=True))
    text = json.dumps(rows)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
