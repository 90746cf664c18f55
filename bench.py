"""Benchmark: D3Q19 LB-IMB-DEM throughput (MLUPS) on one MI355X.

One step = the whole hot path: particle footprint / solid fraction, fused pull
stream + LBGK/IMB collision, per-particle hydrodynamic force and torque, DEM
cell list + contacts, particle integration.  The headline workload is the
D3Q19 suspension 192x756x192 (periodic x/z, walls y, 8317 spheres R = 4 at
solid fraction 0.08, density ratio 1000, tau 0.6, gravity along -y), in FP64;
the FP32-shifted and FP16-storage variants are timed on the same input.

Prints ONE JSON line.  value = FP64 MLUPS (lattice nodes x steps / wall s).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "D3Q19 LB-IMB MLUPS (FP64 vs FP32-shifted) and % of HBM roofline"
BYTES_PER_VALUE = {"fp64": 8, "fp32s": 4, "fp16s": 2}
DTYPE = {"fp64": "f64", "fp32s": "f32", "fp16s": "f16-storage/f32"}


def kernel_source_sha():
    with open(os.path.join(ROOT, "paper_1011_2613_amd", "csrc", "lb_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(storage, workload, width):
    """HBM bytes per launch of the lattice kernel from the committed rocprofv3
    counter runs, if they were taken on the current kernel source at the
    launch shape in use (a record, or a list of records for several shapes)."""
    path = os.path.join(ROOT, "profiles", "lb_kernel_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    recs = d.get("%s_%s" % (workload, storage))
    for rec in recs if isinstance(recs, list) else [recs]:
        if (rec and rec.get("kernel_source_sha") == kernel_source_sha()
                and rec.get("lattice_block") == width):
            return rec.get("bytes_per_launch")
    return None


def parse_shape(text):
    """"256", "256/xcd", "192/cu3" or "256/xcd/cu4" -> (width, order, cu_groups)."""
    parts = text.split("/")
    order, cap = "linear", 0
    for p in parts[1:]:
        if p == "xcd":
            order = "xcd"
        elif p.startswith("cu"):
            cap = int(p[2:])
        else:
            raise ValueError("bad launch shape %r" % text)
    return int(parts[0]), order, cap


def parse_blocks(spec):
    """--lattice-block: "auto", one launch shape for every variant, or per
    variant ("fp64=256/xcd/cu3,fp32s=64")."""
    if spec == "auto":
        return {}
    if "=" not in spec:
        return {v: parse_shape(spec) for v in BYTES_PER_VALUE}
    return {k: parse_shape(x) for k, x in (item.split("=") for item in spec.split(",") if item)}


def shape_text(shape):
    width, order, cap = shape
    return "%d%s%s" % (width, "/xcd" if order == "xcd" else "", "/cu%d" % cap if cap else "")


def run_variant(binding, inputs, w, parts, storage, steps, warmup, eps="sampling", block=None, pipeline=None):
    import torch
    sim = binding.Simulation(w.dim, w.shape, w.tau, storage=storage, wall_y=w.wall_y,
                             fluid_force=w.fluid_force, particle_accel=w.particle_accel,
                             samples=w.samples, kn=w.kn, restitution=w.restitution,
                             max_particles=w.count, max_radius=w.radius, eps=eps)
    if pipeline is not None:
        sim.set_pipeline(pipeline)
    sim.set_particles(*parts)
    # the lattice kernel's workgroup width: measured per workload and storage
    # (part of the warm-up), or as given
    tune_ms = None
    if block is None:
        _, tune_ms = sim.autotune_lattice_block(steps=20)
    else:
        sim.set_lattice_block(*block)
    width = shape_text(sim.lattice_block)
    sim.step(warmup)
    # timed region: HIP events around the lattice kernel only (on the stream
    # it runs on), the other kernels launched as in normal operation
    sim.set_timing(True, lattice_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat_ms, lat_n = sim.get_timing()["lattice"]
    sim.set_timing(False)
    # per-phase breakdown from a short separate pass with events around every phase
    phase_steps = min(steps, 50)
    sim.set_timing(True)
    sim.step(phase_steps)
    phases = sim.get_timing()
    sim.set_timing(False)
    slabs = sim.pipeline
    wall = t1 - t0
    mlups = w.nodes * steps / wall / 1e6
    # one launch of the lattice kernel updates the whole lattice, or one slab
    # of it when the slab pipeline is on (lat_n = steps x slabs)
    avg_ms = lat_ms / max(lat_n, 1)
    launch_nodes = w.nodes * steps / max(lat_n, 1)
    Q = 9 if w.dim == 2 else 19
    bpn = 2 * Q * BYTES_PER_VALUE[storage]
    achieved = bpn * launch_nodes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(storage, w.name, width) if slabs == 1 else None
    step_gbs = bpn * mlups / 1e3
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {
        "mlups": mlups, "ms_per_step": wall / steps * 1e3, "wall_s": wall,
        "lattice_kernel_ms": lat_ms / steps, "lattice_launch_ms": avg_ms, "lattice_launches_per_step": lat_n / steps,
        "pipeline_slabs": slabs, "bytes_per_node": bpn,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "roofline_step": {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                          "basis": "whole step: MLUPS x %d B/node" % bpn},
        "phase_ms_per_step": {k: round(v[0] / phase_steps, 4) for k, v in phases.items() if v[1] > 0},
        "lattice_block": width,
        "lattice_block_tuning_ms": None if tune_ms is None else {
            shape_text(k): round(v, 4) for k, v in tune_ms.items() if math.isfinite(v)},
    }


def precision_report(binding, w, parts, steps=500, window=100):
    """FP32-shifted and FP16 storage against the FP64 GPU run of the same
    workload from the same state, `steps` steps: the per-particle drag error
    |F_low - F_64| / |F_64| averaged over particles and the last `window`
    steps (and its largest value), the error of the suspension-mean drag
    (lbm_get_stats) over the same window, the velocity error
    max |u_low - u_64| / max |u_64| over all nodes at the end, and for FP16 the
    fraction of stored values g_i / w_i that are binary16 subnormals (nonzero
    and below 2^-14 in magnitude)."""
    import numpy as np
    import torch
    Q = 9 if w.dim == 2 else 19
    wts = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4) if w.dim == 2 else \
        np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    ref = {}
    out = {}
    for storage in ("fp64", "fp32s", "fp16s"):
        sim = binding.Simulation(w.dim, w.shape, w.tau, storage=storage, wall_y=w.wall_y,
                                 fluid_force=w.fluid_force, particle_accel=w.particle_accel,
                                 samples=w.samples, kn=w.kn, restitution=w.restitution,
                                 max_particles=w.count, max_radius=w.radius)
        sim.set_particles(*parts)
        sim.step(steps - window)
        F, md = [], []
        for _ in range(window):
            sim.step(1)
            F.append(sim.forces()[0])
            md.append(sim.stats()["mean_drag"])
        F, md = np.array(F), np.array(md)
        _, u = sim.macro_device()
        if storage == "fp64":
            ref = {"F": F, "md": md, "u": u}
        else:
            e = np.linalg.norm(F - ref["F"], axis=2) / np.linalg.norm(ref["F"], axis=2)
            emd = np.linalg.norm(md - ref["md"], axis=1) / np.linalg.norm(ref["md"], axis=1)
            uerr = float((u - ref["u"]).abs().max() / ref["u"].abs().max())
            rec = {"steps": steps, "window": window, "drag_rel_err_mean": float(e.mean()),
                   "drag_rel_err_max": float(e.max()), "mean_drag_rel_err": float(emd.mean()),
                   "velocity_rel_err_inf": uerr}
            if storage == "fp16s":
                f = sim.get_f_device().reshape(Q, -1)
                sub = 0
                for q in range(Q):  # one direction at a time: the paper-scale lattices are large
                    h = (f[q] - wts[q]) / wts[q]
                    sub += ((h != 0) & (h.abs() < 2.0 ** -14)).sum().item()
                    del h
                rec["fp16_subnormal_fraction"] = sub / f.numel()
                del f
            out[storage] = rec
        del u
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


def ensemble_bench(binding, nbox=512, steps=200, check_every=100):
    """Batched drag ensemble at the drag-data size: 512 boxes (edges 32-96,
    1-64 spheres of radius 4-8), autotuned tile shape and launch mode, FP32
    shifted storage, advanced by lbm_batch_run_steady (chunks of check_every
    steps replayed as one captured graph with the device-side steady check;
    the tolerance is set so that no box retires, which times every box);
    lattice updates per second over all boxes."""
    import torch
    from paper_1011_2613_amd import ensemble as E
    boxes = E.sample_boxes(nbox, 4)
    t0 = time.perf_counter()
    b = binding.Batch(boxes, samples=4)
    setup = time.perf_counter() - t0
    tune = b.autotune(steps=5)
    b.run_steady(check_every, 1e-300, check_every, tune["mode"])  # warm-up: captures the chunk graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steady, _ = b.run_steady(steps, 1e-300, check_every, tune["mode"])
    t1 = time.perf_counter()
    assert not steady.any()
    nodes = sum(x["edge"] ** 3 for x in boxes)
    mlups = nodes * steps / (t1 - t0) / 1e6
    gbs = mlups * 1e6 * 152 / 1e9
    b.close()
    torch.cuda.empty_cache()
    return {"value": round(mlups, 1), "unit": "MLUPS", "boxes": nbox, "nodes": nodes,
            "spheres": int(sum(len(x["pos"]) for x in boxes)), "steps": steps, "check_every": check_every,
            "path": "lbm_batch_run_steady (captured chunk graph, device steady check)",
            "mode": "persistent" if tune["mode"] == 1 else "per-step", "tile_rows": tune["rows"],
            "setup_s": round(setup, 2),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def closure_bench(binding, rows=1 << 20, reps=10):
    """MLP drag closure inference (bfloat16 MFMA, binary32 accumulate)."""
    import torch
    from paper_1011_2613_amd import inputs
    m = binding.Mlp(max_batch=64)
    m.set_params(binding.mlp_pack(inputs.mlp_initial_params(3)))
    X = torch.randn(rows, 40, device="cuda:0")
    m.forward(X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m.forward(X)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    flops = 2.0 * (40 * 128 + 128 * 128 * 2 + 128) * rows
    tf = flops / dt / 1e12
    m.close()
    return {"value": round(rows / dt / 1e6, 2), "unit": "M rows/s", "rows": rows,
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": round(tf / 2500.0, 4)}}


def host_cpu():
    """Host facts for the CPU baseline: usable cores and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(w, parts, budget_s=15.0, max_steps=20):
    """The FP64 CPU oracle on the same workload: on every usable host core
    (OpenMP over nodes and particles; results equal the serial program bit for
    bit) for whole steps until `budget_s` has passed or `max_steps` steps, and
    for one step on one thread (the paper's one-core comparison)."""
    from oracle import oracle as O
    out = {}
    cores = len(os.sched_getaffinity(0))
    try:  # the host's CPU share for this process, when the environment states one
        cores = max(1, min(cores, int(os.environ.get("OMP_NUM_THREADS", cores))))
    except ValueError:
        pass
    for label, threads in (("all", cores), ("one", 1)):
        used = O.set_threads(threads)
        orc = O.OracleSim(w.dim, w.shape, w.tau, wall_y=w.wall_y, fluid_force=w.fluid_force,
                          particle_accel=w.particle_accel, samples=w.samples, kn=w.kn,
                          restitution=w.restitution)
        orc.set_particles(*parts)
        steps, dt = 0, 0.0
        while steps < (max_steps if label == "all" else 1) and (steps == 0 or dt < budget_s):
            t0 = time.perf_counter()
            orc.step(1)
            dt += time.perf_counter() - t0
            steps += 1
        orc.close()
        out[label] = (used, steps, dt)
    used, steps, dt = out["all"]
    u1, s1, d1 = out["one"]
    host = host_cpu()
    return {"value": round(w.nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": used,
            "kind": "oracle",
            "sample": "%d steps of the full %s lattice (%d nodes, %d particles) on %d threads, %.1f s"
                      % (steps, w.name, w.nodes, w.count, used, dt),
            "one_thread": {"value": round(w.nodes * s1 / d1 / 1e6, 3), "unit": "MLUPS", "steps": s1,
                           "seconds": round(d1, 2)},
            "host": host}


def copy_calibration(gib=2.0, reps=10):
    """A plain device-to-device copy of known size: the reference for scaling
    the HBM byte counters and the achievable copy bandwidth."""
    import torch
    n = int(gib * 2 ** 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    moved = 2 * n * 8
    print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8,
                      "copy_GBps": round(moved / dt / 1e9, 1), "launches": reps + 1}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--variants", default="fp64,fp32s,fp16s")
    ap.add_argument("--eps", default="sampling", choices=["sampling", "table"],
                    help="solid fraction by sub-cell sampling or by the paper's table lookup")
    ap.add_argument("--lattice-block", default="auto",
                    help='lattice kernel launch shape: "auto" (measured per variant), a width '
                         '64/128/192/256 with an optional "/xcd" workgroup order and "/cuN" cap of '
                         'N workgroups per CU, or per variant, e.g. "fp64=256/xcd/cu3,fp32s=64"')
    ap.add_argument("--pipeline", type=int, default=None,
                    help="slab pipeline: 0 automatic, 1 off, 2..8 slabs (default: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32s / FP16 error measurement against the FP64 run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-ensemble and closure measurements")
    ap.add_argument("--closure-only", action="store_true",
                    help="only time the closure's inference kernel (4 M rows; for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.closure_only:
        from paper_1011_2613_amd import binding
        binding.load()
        print(json.dumps({"closure": closure_bench(binding, rows=1 << 22)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1011_2613_amd import binding, inputs
    binding.load()
    w = inputs.workload(args.workload)
    parts = w.particles()
    variants = [v for v in args.variants.split(",") if v]
    if "fp64" not in variants:
        variants = ["fp64"] + variants
    blocks = parse_blocks(args.lattice_block)
    res = {}
    for v in variants:
        res[v] = run_variant(binding, inputs, w, parts, v, args.steps, args.warmup, eps=args.eps,
                             block=blocks.get(v), pipeline=args.pipeline)
        print("# %s: %.1f MLUPS, lattice kernel %.3f ms per step (%d slabs), %.1f GB/s, workgroup %s"
              % (v, res[v]["mlups"], res[v]["lattice_kernel_ms"], res[v]["pipeline_slabs"],
                 res[v]["roofline"]["achieved"], res[v]["lattice_block"]), file=sys.stderr, flush=True)
    base = res["fp64"]
    out = {
        "metric": METRIC,
        "value": round(base["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(base["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE["fp64"],
        "data": "synthetic (seeded random sphere placement, fluid at rest)",
        "config": {"workload": "%s: %s %s, %s, %d %s R=%g, tau %g, density ratio %g"
                   % (w.name, "D3Q19" if w.dim == 3 else "D2Q9", "x".join(str(e) for e in w.shape),
                      "walls y" if w.wall_y else "periodic", w.count,
                      "spheres" if w.dim == 3 else "discs", w.radius, round(w.tau, 4), w.rho_ratio),
                   "nodes": w.nodes, "particles": w.count, "storage": "fp64", "eps": args.eps,
                   "lattice_block": base["lattice_block"], "pipeline_slabs": base["pipeline_slabs"],
                   "lattice_block_tuning_ms": base["lattice_block_tuning_ms"]},
        "roofline": base["roofline"],
        "roofline_step": base["roofline_step"],
        "phase_ms_per_step": base["phase_ms_per_step"],
        "variants": {v: {"value": round(r["mlups"], 1), "unit": "MLUPS", "dtype": DTYPE[v],
                         "ms_per_step": round(r["ms_per_step"], 4),
                         "roofline": r["roofline"], "roofline_step": r["roofline_step"],
                         "phase_ms_per_step": r["phase_ms_per_step"],
                         "lattice_block": r["lattice_block"], "pipeline_slabs": r["pipeline_slabs"],
                         "lattice_block_tuning_ms": r["lattice_block_tuning_ms"],
                         "speedup_vs_fp64": round(r["mlups"] / base["mlups"], 3)}
                     for v, r in res.items() if v != "fp64"},
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_precision:
        prec = precision_report(binding, w, parts)
        for v, rec in prec.items():
            if v in out["variants"]:
                out["variants"][v]["errors_vs_fp64"] = rec
        print("# precision: %s" % prec, file=sys.stderr, flush=True)
    if not args.no_extras:
        out["ensemble"] = ensemble_bench(binding)
        print("# ensemble: %s" % out["ensemble"], file=sys.stderr, flush=True)
        out["closure"] = closure_bench(binding)
        print("# closure: %s" % out["closure"], file=sys.stderr, flush=True)
    # the oracle times whole steps of the workload (C3: about 3 s per step on
    # 8 cores, 9 s on one); a lattice much larger than that is not timed on the host
    if not args.no_cpu_baseline and w.nodes <= 10 ** 8:
        out["cpu_baseline"] = cpu_baseline(w, parts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
