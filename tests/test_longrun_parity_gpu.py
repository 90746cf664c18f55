"""FP64 parity at the full suspension workloads over their stated step counts.

The reference data (tests/golden/longrun_*.npz) were written by
tests/golden/make_longrun.py, which runs only the CPU oracle (with every host
core; its threaded loops equal the serial program bit for bit).  The GPU runs
the same seeded workload in the launch shape the benchmark keeps for it and is
compared every 100 steps on 64 seeded particles (position, velocity, angular
velocity, hydrodynamic force and torque, contact force) and the total fluid
mass, and at the end on every particle and on a seeded node sample (the
pre-collision populations and their moments).  Bar: 1e-12 relative per field
(max |gpu - oracle| / max |oracle|; positions as displacements from the start,
minimum image; populations as deviations from the rest weights).  The first
checkpoint that misses the bar is reported.
"""
import os

import numpy as np
import pytest

from paper_1011_2613_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12


def say(*a):
    print(*a, flush=True)


def _rel(a, b, den=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if den is None else den
    num = np.abs(a - b).max()
    return float(num / den) if den > 0 else float(num)


def _disp_err(x, xref, x0, w):
    """Error of positions relative to the largest displacement, minimum image
    on the periodic axes."""
    L = np.array(list(w.shape) + [1] * (3 - len(w.shape)), dtype=np.float64)
    per = np.array([True, not w.wall_y, w.dim == 3])

    def mi(d):
        d = d.copy()
        d[:, per] -= L[per] * np.round(d[:, per] / L[per])
        return d

    return float(np.abs(mi(x - xref)).max() / max(np.abs(mi(xref - x0)).max(), 1e-300))


@pytest.mark.parametrize("name,steps,shape", [
    ("C3", 2000, (256, "xcd", 4)),
    ("C2", 5000, (256, "linear", 4)),
])
def test_longrun_fp64_parity(gpu_lib, name, steps, shape):
    path = os.path.join(HERE, "golden", "longrun_%s_%d.npz" % (name, steps))
    if not os.path.exists(path):
        pytest.skip("reference data not written yet: python tests/golden/make_longrun.py %s %d"
                    % (name, steps))
    d = np.load(path, allow_pickle=False)
    w = I.workload(name)
    assert int(d["steps"]) == steps and int(d["particles"]) == w.count
    say("long run %s, %d steps, launch shape %s" % (name, steps, shape))
    sim = gpu_lib.simulation_for(w, "fp64")
    sim.set_lattice_block(*shape)
    x0 = w.particles()[0]
    pidx = d["cp_pidx"]
    first_bad = None
    worst = {}
    for k, t in enumerate(d["cp_step"]):
        sim.step(int(t) - sim.t)
        x, v, om = sim.particles()
        F, T = sim.forces()
        Fc = sim.contact_forces()
        st = sim.stats()
        errs = {
            "x": _disp_err(x[pidx], d["cp_x"][k], x0[pidx], w),
            "v": _rel(v[pidx], d["cp_v"][k]),
            "w": _rel(om[pidx], d["cp_w"][k]),
            "F": _rel(F[pidx], d["cp_F"][k]),
            "T": _rel(T[pidx], d["cp_T"][k]),
            "Fc": _rel(Fc[pidx], d["cp_Fc"][k]) if np.abs(d["cp_Fc"][k]).max() > 0
            else float(np.abs(Fc[pidx]).max()),
            "mass": abs(st["mass"] - float(d["cp_mass"][k])) / float(d["cp_mass"][k]),
        }
        for key, e in errs.items():
            worst[key] = max(worst.get(key, 0.0), e)
        bad = {key: e for key, e in errs.items() if not e <= TOL}
        if bad and first_bad is None:
            first_bad = (int(t), bad)
        say("  t=%d %s" % (t, " ".join("%s %.1e" % kv for kv in errs.items())))
    assert first_bad is None, "first checkpoint beyond %g: t=%d %s" % (TOL, first_bad[0], first_bad[1])
    # every particle at the end
    x, v, om = sim.particles()
    F, T = sim.forces()
    Fc = sim.contact_forces()
    fin = {"x": _disp_err(x, d["x"], x0, w), "v": _rel(v, d["v"]), "w": _rel(om, d["w"]),
           "F": _rel(F, d["F"]), "T": _rel(T, d["T"]), "Fc": _rel(Fc, d["Fc"])}
    # a seeded node sample: populations, density, velocity
    nidx = d["node_idx"]
    f = sim.get_f().reshape(sim.Q, -1)[:, nidx]
    rho, u = sim.macro()
    rho = rho.reshape(-1)[nidx]
    u = u.reshape(w.dim, -1)[:, nidx]
    _, wts = _weights(w.dim)
    fin["f"] = _rel(f, d["node_f"], np.abs(d["node_f"] - wts[:, None]).max())
    fin["rho"] = _rel(rho, d["node_rho"], np.abs(d["node_rho"] - 1.0).max())
    fin["u"] = _rel(u, d["node_u"])
    say("  final %s" % " ".join("%s %.1e" % kv for kv in fin.items()))
    say("  worst over checkpoints %s" % " ".join("%s %.1e" % kv for kv in worst.items()))
    bad = {k: e for k, e in fin.items() if not e <= TOL}
    assert not bad, "final fields beyond %g: %s" % (TOL, bad)


def _weights(dim):
    if dim == 2:
        return None, np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return None, np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
