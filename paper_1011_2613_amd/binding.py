"""Thin ctypes binding of liblbimb.so (C ABI in include/lbimb.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies the device workspace and the HIP stream.  The
binding fails loudly when the native library has not been built; there is no
fallback implementation.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbimb.so")

LBM_OK = 0
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_FP64, LBM_FP32_SHIFTED, LBM_FP16_STORE = 0, 1, 2
LBM_HOST, LBM_DEVICE = 0, 1
LBM_NPHASES = 6
PHASES = ("footprint", "lattice", "force", "cells", "dem", "integrate")
STORAGE = {"fp64": LBM_FP64, "fp32s": LBM_FP32_SHIFTED, "fp16s": LBM_FP16_STORE}
EPS_MODES = {"sampling": 0, "table": 1}
ERRORS = {-1: "LBM_E_INVALID", -2: "LBM_E_NOMEM", -3: "LBM_E_HIP", -4: "LBM_E_NONFINITE",
          -5: "LBM_E_SLOT_OVERFLOW", -6: "LBM_E_STATE", -7: "LBM_E_IO",
          -8: "LBM_E_CELL_OVERFLOW", -9: "LBM_E_CONTACT_OVERFLOW"}


class lbm_config(C.Structure):
    _fields_ = [("lattice", C.c_int), ("storage", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int), ("wall_y", C.c_int), ("tau", C.c_double),
                ("fluid_force", C.c_double * 3), ("particle_accel", C.c_double * 3),
                ("eps_samples", C.c_int), ("kn", C.c_double), ("restitution", C.c_double),
                ("max_particles", C.c_int), ("max_radius", C.c_double), ("eps_mode", C.c_int)]


class lbm_stats(C.Structure):
    _fields_ = [("t", C.c_int64), ("np", C.c_int64), ("nodes", C.c_int64), ("mass", C.c_double),
                ("fluid_momentum", C.c_double * 3), ("solid_fraction", C.c_double),
                ("fluid_velocity", C.c_double * 3), ("particle_momentum", C.c_double * 3),
                ("particle_velocity", C.c_double * 3), ("mean_particle_velocity", C.c_double * 3),
                ("slip_velocity", C.c_double * 3), ("mean_drag", C.c_double * 3)]


class LbmError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "error"), code, msg))


_lib = None
_SYMBOLS = ("lbm_workspace_bytes", "lbm_create", "lbm_destroy", "lbm_set_particles",
            "lbm_set_distributions", "lbm_get_distributions", "lbm_step", "lbm_get_forces",
            "lbm_get_contact_forces", "lbm_get_particles", "lbm_get_macro", "lbm_get_q",
            "lbm_time", "lbm_particle_count", "lbm_set_timing", "lbm_get_timing", "lbm_save", "lbm_load",
            "lbm_set_lattice_block", "lbm_get_lattice_block", "lbm_autotune_lattice_block", "lbm_get_stats",
            "lbm_set_neighbour_list", "lbm_get_neighbour_list", "lbm_set_pipeline", "lbm_get_pipeline",
            "lbm_error_string", "lbm_last_error",
            "mlp_workspace_bytes", "mlp_create", "mlp_destroy", "mlp_set_params", "mlp_get_params",
            "mlp_forward", "mlp_gradients", "mlp_train_step", "mlp_gradients_noalloc",
            "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_destroy", "lbm_batch_set_tile_rows",
            "lbm_batch_run", "lbm_batch_set_active", "lbm_batch_forces", "lbm_batch_mean_velocity",
            "lbm_batch_get_distributions", "lbm_batch_autotune", "lbm_batch_time", "lbm_batch_shell_velocity",
            "lbm_batch_run_steady", "lbm_batch_get_drag", "mlp_set_normaliser", "mlp_infer")


def load():
    """Load liblbimb.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbimb.so is not built: run `python -m paper_1011_2613_amd.build` "
                           "(or __graft_entry__.build()) first")
    # PyTorch-ROCm carries its own HIP runtime (soname libamdhip64.so.7).  Load
    # it first so that the library binds to that same runtime: one runtime per
    # process, so torch's streams and device memory are valid handles here.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.lbm_workspace_bytes.argtypes = [C.POINTER(lbm_config), C.POINTER(C.c_size_t)]
    L.lbm_create.argtypes = [C.POINTER(lbm_config), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_set_particles.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.c_int]
    L.lbm_set_distributions.argtypes = [vp, vp, C.c_int]
    L.lbm_get_distributions.argtypes = [vp, vp, C.c_int]
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_get_forces.argtypes = [vp, vp, vp, C.c_int]
    L.lbm_get_contact_forces.argtypes = [vp, vp, C.c_int]
    L.lbm_get_particles.argtypes = [vp, vp, vp, vp, C.c_int]
    L.lbm_get_macro.argtypes = [vp, vp, vp, C.c_int]
    L.lbm_get_q.argtypes = [vp, vp, C.c_int]
    L.lbm_time.argtypes = [vp]
    L.lbm_time.restype = i64
    L.lbm_particle_count.argtypes = [vp]
    L.lbm_particle_count.restype = i64
    L.lbm_set_timing.argtypes = [vp, C.c_int]
    L.lbm_get_timing.argtypes = [vp, dp, C.POINTER(i64)]
    ip = C.POINTER(C.c_int)
    L.lbm_set_lattice_block.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.lbm_get_lattice_block.argtypes = [vp, ip, ip, ip]
    L.lbm_autotune_lattice_block.argtypes = [vp, C.c_int, ip, ip, ip, dp]
    L.lbm_get_stats.argtypes = [vp, C.POINTER(lbm_stats)]
    L.lbm_set_neighbour_list.argtypes = [vp, C.c_int, C.c_double]
    L.lbm_get_neighbour_list.argtypes = [vp, ip, dp, C.POINTER(i64)]
    L.lbm_set_pipeline.argtypes = [vp, C.c_int]
    L.lbm_get_pipeline.argtypes = [vp, ip]
    L.lbm_save.argtypes = [vp, C.c_char_p]
    L.lbm_load.argtypes = [vp, C.c_char_p]
    L.lbm_error_string.argtypes = [C.c_int]
    L.lbm_error_string.restype = C.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    for name in _SYMBOLS:
        if name.startswith("lbm_") and not name.startswith("lbm_batch_") and name not in (
                "lbm_destroy", "lbm_time", "lbm_particle_count", "lbm_error_string", "lbm_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def exported_symbols():
    return _SYMBOLS


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


class Simulation:
    """One LB-IMB-DEM context on one GPU (see include/lbimb.h for semantics).

    shape is (nx, ny) for D2Q9 and (nx, ny, nz) for D3Q19.  Host-side getters
    return numpy arrays shaped like the lattice ([.., nz, ny, nx]).
    """

    def __init__(self, dim, shape, tau, storage="fp64", wall_y=False, fluid_force=(0, 0, 0),
                 particle_accel=(0, 0, 0), samples=4, kn=0.0, restitution=0.9,
                 max_particles=1, max_radius=0.0, eps="sampling", device="cuda:0"):
        import torch
        self._torch = torch
        L = load()
        self.dim = dim
        self.Q = 9 if dim == 2 else 19
        nx, ny = int(shape[0]), int(shape[1])
        nz = int(shape[2]) if dim == 3 else 1
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        cfg = lbm_config()
        cfg.lattice = LBM_D2Q9 if dim == 2 else LBM_D3Q19
        cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.wall_y = int(bool(wall_y))
        cfg.tau = float(tau)
        ff = list(fluid_force) + [0.0] * (3 - len(fluid_force))
        pa = list(particle_accel) + [0.0] * (3 - len(particle_accel))
        for a in range(3):
            cfg.fluid_force[a] = float(ff[a])
            cfg.particle_accel[a] = float(pa[a])
        cfg.eps_samples = int(samples)
        cfg.kn = float(kn)
        cfg.restitution = float(restitution)
        cfg.max_particles = int(max_particles)
        cfg.max_radius = float(max_radius)
        cfg.eps_mode = EPS_MODES[eps]
        self.cfg = cfg
        nbytes = C.c_size_t(0)
        self._check(L.lbm_workspace_bytes(C.byref(cfg), C.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        self._ctx = None
        self._check(L.lbm_create(C.byref(cfg), C.c_void_p(aligned), C.c_size_t(int(nbytes.value)),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._ctx = h
        self.np_ = 0

    # ----------------------------------------------------------- plumbing
    def _check(self, rc):
        if rc != LBM_OK:
            msg = ""
            msg = load().lbm_last_error(getattr(self, "_ctx", None)).decode()
            raise LbmError(rc, msg)

    def close(self):
        if getattr(self, "_ctx", None):
            load().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def field_shape(self):
        return (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)

    def synchronize(self):
        self.stream.synchronize()

    # ----------------------------------------------------------------- ABI
    def set_particles(self, pos=None, vel=None, omega=None, radius=None, rho_s=None, fixed=None):
        """Replaces the particle set; no arguments (or an empty pos) sets a
        fluid without particles, which must still precede the first step."""
        pos = _f64(np.zeros((0, 3)) if pos is None else pos, (-1, 3))
        n = pos.shape[0]
        vel = _f64(np.zeros((n, 3)) if vel is None else vel, (n, 3))
        omega = _f64(np.zeros((n, 3)) if omega is None else omega, (n, 3))
        radius = _f64(np.zeros(n) if radius is None and n == 0 else radius, (n,))
        rho_s = _f64(np.zeros(n) if rho_s is None and n == 0 else rho_s, (n,))
        fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.uint8).reshape(n))
        self._check(load().lbm_set_particles(self._ctx, n, _ptr(pos), _ptr(vel), _ptr(omega),
                                             _ptr(radius), _ptr(rho_s), _ptr(fx), LBM_HOST))
        self.np_ = n

    def set_f(self, f):
        f = _f64(f, (self.Q, self.N))
        self._check(load().lbm_set_distributions(self._ctx, _ptr(f), LBM_HOST))

    def get_f(self):
        f = np.empty((self.Q,) + self.field_shape)
        self._check(load().lbm_get_distributions(self._ctx, _ptr(f), LBM_HOST))
        return f

    def get_f_device(self):
        """Pre-collision populations [Q][...] binary64 as a device tensor,
        converted from the storage format on the library's stream."""
        torch = self._torch
        f = torch.empty((self.Q,) + self.field_shape, dtype=torch.float64, device=self.device)
        self._check(load().lbm_get_distributions(self._ctx, _ptr(f), LBM_DEVICE))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return f

    def step(self, n=1):
        self._check(load().lbm_step(self._ctx, int(n)))

    @property
    def t(self):
        return int(load().lbm_time(self._ctx))

    def macro(self):
        rho = np.empty(self.field_shape)
        u = np.empty((self.dim,) + self.field_shape)
        self._check(load().lbm_get_macro(self._ctx, _ptr(rho), _ptr(u), LBM_HOST))
        return rho, u

    def macro_device(self):
        """(rho, u) as device tensors, computed on the library's stream."""
        torch = self._torch
        rho = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        u = torch.empty((self.dim,) + self.field_shape, dtype=torch.float64, device=self.device)
        self._check(load().lbm_get_macro(self._ctx, _ptr(rho), _ptr(u), LBM_DEVICE))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return rho, u

    def q(self):
        q = np.empty((self.dim,) + self.field_shape)
        self._check(load().lbm_get_q(self._ctx, _ptr(q), LBM_HOST))
        return q

    def forces(self):
        n = max(self.np_, 1)
        F = np.zeros((n, 3)); T = np.zeros((n, 3))
        self._check(load().lbm_get_forces(self._ctx, _ptr(F), _ptr(T), LBM_HOST))
        return F[: self.np_], T[: self.np_]

    def contact_forces(self):
        Fc = np.zeros((max(self.np_, 1), 3))
        self._check(load().lbm_get_contact_forces(self._ctx, _ptr(Fc), LBM_HOST))
        return Fc[: self.np_]

    def particles(self):
        n = max(self.np_, 1)
        x = np.zeros((n, 3)); v = np.zeros((n, 3)); w = np.zeros((n, 3))
        self._check(load().lbm_get_particles(self._ctx, _ptr(x), _ptr(v), _ptr(w), LBM_HOST))
        return x[: self.np_], v[: self.np_], w[: self.np_]

    def stats(self):
        """Suspension-wide sums (lbm_get_stats) as a dict of floats / 3-vectors."""
        st = lbm_stats()
        self._check(load().lbm_get_stats(self._ctx, C.byref(st)))
        out = {}
        for name, typ in lbm_stats._fields_:
            v = getattr(st, name)
            out[name] = np.array(list(v)) if hasattr(v, "__len__") else v
        return out

    def set_timing(self, on, lattice_only=False):
        mode = 0 if not on else (2 if lattice_only else 1)
        self._check(load().lbm_set_timing(self._ctx, mode))

    def get_timing(self):
        ms = (C.c_double * LBM_NPHASES)()
        n = (C.c_int64 * LBM_NPHASES)()
        self._check(load().lbm_get_timing(self._ctx, ms, n))
        return {PHASES[k]: (ms[k], n[k]) for k in range(LBM_NPHASES)}

    LATTICE_BLOCKS = (64, 128, 192, 256)
    LATTICE_ORDERS = ("linear", "xcd")
    LATTICE_CAPS = (0, 4, 3)

    def set_neighbour_list(self, every, skin=1.0):
        """DEM neighbour search: every = 0 the per-step cell list, else lists
        within R_i + R_j + skin rebuilt after `every` steps or when a particle
        moved 0.49 skin (lbm_set_neighbour_list)."""
        self._check(load().lbm_set_neighbour_list(self._ctx, int(every), float(skin)))

    @property
    def neighbour_list(self):
        """(every, skin, builds so far)."""
        e, s, b = C.c_int(0), C.c_double(0.0), C.c_int64(0)
        self._check(load().lbm_get_neighbour_list(self._ctx, C.byref(e), C.byref(s), C.byref(b)))
        return e.value, s.value, b.value

    def set_pipeline(self, slabs):
        """Slab pipeline: 0 automatic, 1 off, 2..8 slabs (lbm_set_pipeline)."""
        self._check(load().lbm_set_pipeline(self._ctx, int(slabs)))

    @property
    def pipeline(self):
        """Slabs in use (1: the plain step)."""
        k = C.c_int(0)
        self._check(load().lbm_get_pipeline(self._ctx, C.byref(k)))
        return k.value

    def set_lattice_block(self, threads, order="linear", cu_groups=0):
        """Launch shape of the lattice kernel: workgroup width (0: built-in
        rule), workgroup order ("linear" or "xcd") and the most workgroups
        resident on one CU (0: no cap, else 3..8)."""
        self._check(load().lbm_set_lattice_block(self._ctx, int(threads),
                                                 self.LATTICE_ORDERS.index(order), int(cu_groups)))

    @property
    def lattice_block(self):
        """(width, order, cu_groups) of the lattice kernel's launches."""
        w, o, g = C.c_int(0), C.c_int(0), C.c_int(0)
        self._check(load().lbm_get_lattice_block(self._ctx, C.byref(w), C.byref(o), C.byref(g)))
        return w.value, self.LATTICE_ORDERS[o.value], g.value

    def autotune_lattice_block(self, steps=20):
        """Time the lattice kernel at each launch shape over real steps (the
        state advances by up to 48 (steps + 1) steps) and keep the fastest.
        Returns ((width, order, cu_groups), {shape: mean ms per lattice
        launch})."""
        w, o, g = C.c_int(0), C.c_int(0), C.c_int(0)
        ms = (C.c_double * 24)()
        self._check(load().lbm_autotune_lattice_block(self._ctx, int(steps), C.byref(w), C.byref(o),
                                                      C.byref(g), ms))
        table = {(self.LATTICE_BLOCKS[k % 4], self.LATTICE_ORDERS[(k // 4) % 2],
                  self.LATTICE_CAPS[k // 8]): ms[k] for k in range(24)}
        return (w.value, self.LATTICE_ORDERS[o.value], g.value), table

    def save(self, path):
        self._check(load().lbm_save(self._ctx, str(path).encode()))

    def load_state(self, path):
        self._check(load().lbm_load(self._ctx, str(path).encode()))
        self.np_ = int(load().lbm_particle_count(self._ctx))


def simulation_for(workload, storage="fp64", device="cuda:0", with_particles=True):
    """A Simulation set up for an inputs.Workload (particles placed, fluid at rest)."""
    w = workload
    sim = Simulation(w.dim, w.shape, w.tau, storage=storage, wall_y=w.wall_y,
                     fluid_force=w.fluid_force, particle_accel=w.particle_accel,
                     samples=w.samples, kn=w.kn, restitution=w.restitution,
                     max_particles=max(w.count, 1), max_radius=w.radius, device=device)
    if with_particles and w.count > 0:
        pos, vel, om, rad, rho, fixed = w.particles()
        sim.set_particles(pos, vel, om, rad, rho, fixed)
    return sim


# ------------------------------------------------------------ drag closure
MLP_NIN, MLP_NPARAMS = 40, 38401


def _load_mlp(L):
    if getattr(L, "_mlp_ready", False):
        return L
    vp, i64 = C.c_void_p, C.c_int64
    L.mlp_workspace_bytes.argtypes = [i64, C.POINTER(C.c_size_t)]
    L.mlp_create.argtypes = [i64, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.mlp_destroy.argtypes = [vp]
    L.mlp_destroy.restype = None
    L.mlp_set_params.argtypes = [vp, vp, C.c_int]
    L.mlp_get_params.argtypes = [vp, vp, C.c_int]
    L.mlp_forward.argtypes = [vp, vp, i64, vp]
    L.mlp_gradients.argtypes = [vp, vp, vp, i64, vp, vp, C.c_int]
    L.mlp_train_step.argtypes = [vp, vp, vp, i64, C.c_float, vp]
    L.mlp_gradients_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.mlp_set_normaliser.argtypes = [vp, vp, vp, vp, vp, C.c_int]
    L.mlp_infer.argtypes = [vp, vp, i64, vp, vp]
    for n in ("mlp_workspace_bytes", "mlp_create", "mlp_set_params", "mlp_get_params", "mlp_forward",
              "mlp_gradients", "mlp_train_step", "mlp_gradients_noalloc", "mlp_set_normaliser", "mlp_infer"):
        getattr(L, n).restype = C.c_int
    L._mlp_ready = True
    return L


class Mlp:
    """The drag-closure MLP on one GPU (include/mlp_closure.h).  Inputs and
    outputs are torch tensors on the context's device (binary32)."""

    def __init__(self, max_batch=4096, device="cuda:0"):
        import torch
        self._torch = torch
        L = _load_mlp(load())
        nbytes = C.c_size_t(0)
        rc = L.mlp_workspace_bytes(int(max_batch), C.byref(nbytes))
        if rc:
            raise LbmError(rc, "mlp_workspace_bytes")
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        rc = L.mlp_create(int(max_batch), C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream),
                          C.byref(h))
        if rc:
            raise LbmError(rc, "mlp_create")
        self._ctx = h

    def close(self):
        if getattr(self, "_ctx", None):
            load().mlp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_in(self):
        self.stream.wait_stream(self._torch.cuda.current_stream(self.device))

    def _sync_out(self):
        self._torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(MLP_NPARAMS))
        rc = load().mlp_set_params(self._ctx, _ptr(p), LBM_HOST)
        if rc:
            raise LbmError(rc, "mlp_set_params")

    def get_params(self):
        p = np.empty(MLP_NPARAMS, dtype=np.float32)
        rc = load().mlp_get_params(self._ctx, _ptr(p), LBM_HOST)
        if rc:
            raise LbmError(rc, "mlp_get_params")
        return p

    def _dev(self, a, shape):
        t = self._torch.as_tensor(a, dtype=self._torch.float32, device=self.device)
        return t.reshape(shape).contiguous()

    def forward(self, X):
        X = self._dev(X, (-1, MLP_NIN))
        y = self._torch.empty(X.shape[0], dtype=self._torch.float32, device=self.device)
        self._sync_in()
        rc = load().mlp_forward(self._ctx, _ptr(X), X.shape[0], _ptr(y))
        if rc:
            raise LbmError(rc, "mlp_forward")
        self._sync_out()
        return y

    def set_normaliser(self, mu, sd, lo, hi):
        a = [np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(MLP_NIN)) for v in (mu, sd, lo, hi)]
        rc = load().mlp_set_normaliser(self._ctx, *[_ptr(v) for v in a], LBM_HOST)
        if rc:
            raise LbmError(rc, "mlp_set_normaliser")

    def infer(self, X):
        """mlp_infer on raw inputs: (y [n] device tensor, out_of_envelope [n] device uint8 tensor)."""
        X = self._dev(X, (-1, MLP_NIN))
        n = X.shape[0]
        y = self._torch.empty(n, dtype=self._torch.float32, device=self.device)
        flag = self._torch.empty(n, dtype=self._torch.uint8, device=self.device)
        self._sync_in()
        rc = load().mlp_infer(self._ctx, _ptr(X), n, _ptr(y), _ptr(flag))
        if rc:
            raise LbmError(rc, "mlp_infer")
        self._sync_out()
        return y, flag

    def gradients(self, X, y):
        X = self._dev(X, (-1, MLP_NIN))
        y = self._dev(y, (-1,))
        g = np.empty(MLP_NPARAMS, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        self._sync_in()
        rc = load().mlp_gradients(self._ctx, _ptr(X), _ptr(y), X.shape[0], _ptr(g), _ptr(loss), LBM_HOST)
        if rc:
            raise LbmError(rc, "mlp_gradients")
        return g, float(loss[0])

    def train_step(self, X, y, lr):
        X = self._dev(X, (-1, MLP_NIN))
        y = self._dev(y, (-1,))
        loss = np.empty(1, dtype=np.float32)
        self._sync_in()
        rc = load().mlp_train_step(self._ctx, _ptr(X), _ptr(y), X.shape[0], C.c_float(lr), _ptr(loss))
        if rc:
            raise LbmError(rc, "mlp_train_step")
        return float(loss[0])


MLP_NOALLOC_MAX_ROWS = 4096


def mlp_gradients_noalloc(params, X, y, grads, loss=None, stream=None):
    """mlp_gradients_noalloc on device tensors (binary32, contiguous, on the
    current GPU): params [MLP_NPARAMS], X [n][40], y [n], grads [MLP_NPARAMS]
    out, loss [1] out or None.  Queued on `stream` (a torch stream; None: the
    current one); nothing is allocated."""
    import torch
    n = int(X.shape[0])
    for t in (params, X, y, grads) + ((loss,) if loss is not None else ()):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("mlp_gradients_noalloc takes contiguous binary32 device tensors")
    if params.numel() != MLP_NPARAMS or grads.numel() != MLP_NPARAMS or X.shape[1:] != (MLP_NIN,) \
            or y.numel() != n:
        raise ValueError("mlp_gradients_noalloc: shapes params [%d], X [n][%d], y [n], grads [%d]"
                         % (MLP_NPARAMS, MLP_NIN, MLP_NPARAMS))
    if not 1 <= n <= MLP_NOALLOC_MAX_ROWS:
        raise ValueError("mlp_gradients_noalloc takes 1..%d rows, got %d" % (MLP_NOALLOC_MAX_ROWS, n))
    s = stream if stream is not None else torch.cuda.current_stream(X.device)
    rc = _load_mlp(load()).mlp_gradients_noalloc(
        C.c_void_p(params.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()), n,
        C.c_void_p(grads.data_ptr()), C.c_void_p(loss.data_ptr() if loss is not None else None),
        C.c_void_p(s.cuda_stream))
    if rc:
        raise LbmError(rc, "mlp_gradients_noalloc")


def mlp_unpack(p):
    """Packed parameter vector -> [[W1, b1], ..., [W4, b4]] (views)."""
    p = np.asarray(p)
    out, o = [], 0
    for fin, fout in ((40, 128), (128, 128), (128, 128), (128, 1)):
        W = p[o:o + fin * fout].reshape(fout, fin); o += fin * fout
        b = p[o:o + fout]; o += fout
        out.append([W, b])
    return out


def mlp_pack(params):
    return np.concatenate([np.concatenate([np.asarray(W).ravel(), np.asarray(b).ravel()]) for W, b in params])


# ------------------------------------------------------ batched ensemble
class lbm_box(C.Structure):
    _fields_ = [("edge", C.c_int), ("tau", C.c_double), ("fluid_force", C.c_double * 3),
                ("nspheres", C.c_int), ("pos", C.POINTER(C.c_double)), ("radius", C.c_double),
                ("init_velocity", C.c_double * 3)]


LBM_BATCH_PER_STEP, LBM_BATCH_PERSISTENT = 0, 1


def _load_batch(L):
    if getattr(L, "_batch_ready", False):
        return L
    vp, i64 = C.c_void_p, C.c_int64
    bp = C.POINTER(lbm_box)
    L.lbm_batch_workspace_bytes.argtypes = [bp, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.lbm_batch_create.argtypes = [bp, C.c_int, C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_batch_set_tile_rows.argtypes = [vp, C.c_int, C.c_int]
    L.lbm_batch_run.argtypes = [vp, i64, C.c_int]
    L.lbm_batch_set_active.argtypes = [vp, vp]
    L.lbm_batch_forces.argtypes = [vp, vp, vp, C.c_int]
    L.lbm_batch_mean_velocity.argtypes = [vp, vp, C.c_int]
    L.lbm_batch_shell_velocity.argtypes = [vp, vp, C.c_int]
    L.lbm_batch_get_distributions.argtypes = [vp, C.c_int, vp, C.c_int]
    L.lbm_batch_autotune.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.lbm_batch_time.argtypes = [vp]
    L.lbm_batch_time.restype = i64
    L.lbm_batch_run_steady.argtypes = [vp, i64, C.c_double, C.c_int, C.c_int, vp, vp]
    L.lbm_batch_get_drag.argtypes = [vp, vp, vp, C.c_int]
    for n in ("lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_set_tile_rows", "lbm_batch_run",
              "lbm_batch_set_active", "lbm_batch_forces", "lbm_batch_mean_velocity",
              "lbm_batch_shell_velocity", "lbm_batch_get_distributions", "lbm_batch_autotune",
              "lbm_batch_run_steady", "lbm_batch_get_drag"):
        getattr(L, n).restype = C.c_int
    L._batch_ready = True
    return L


class Batch:
    """Batched ensemble of periodic D3Q19 boxes with fixed spheres (shifted
    FP32).  boxes: list of dicts with keys edge, tau, fluid_force (3),
    pos ([n, 3] array), radius and optionally init_velocity (3)."""

    def __init__(self, boxes, samples=4, device="cuda:0"):
        import torch
        self._torch = torch
        L = _load_batch(load())
        self.nbox = len(boxes)
        self._pos = []
        arr = (lbm_box * self.nbox)()
        self.edges = []
        self.counts = []
        for b, d in enumerate(boxes):
            pos = np.ascontiguousarray(np.asarray(d.get("pos", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3))
            self._pos.append(pos)
            arr[b].edge = int(d["edge"])
            arr[b].tau = float(d["tau"])
            ff = list(d.get("fluid_force", (0, 0, 0))) + [0.0] * 3
            for a in range(3):
                arr[b].fluid_force[a] = float(ff[a])
            arr[b].nspheres = pos.shape[0]
            arr[b].pos = pos.ctypes.data_as(C.POINTER(C.c_double)) if pos.shape[0] else None
            arr[b].radius = float(d.get("radius", 1.0))
            u0 = list(d.get("init_velocity", (0, 0, 0))) + [0.0] * 3
            for a in range(3):
                arr[b].init_velocity[a] = float(u0[a])
            self.edges.append(int(d["edge"]))
            self.counts.append(pos.shape[0])
        self._arr = arr
        self.nsph = int(sum(self.counts))
        nbytes = C.c_size_t(0)
        rc = L.lbm_batch_workspace_bytes(arr, self.nbox, int(samples), C.byref(nbytes))
        if rc:
            raise LbmError(rc, "lbm_batch_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        rc = L.lbm_batch_create(arr, self.nbox, int(samples), C.c_void_p(aligned), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise LbmError(rc, "lbm_batch_create")
        self._ctx = h

    def close(self):
        if getattr(self, "_ctx", None):
            load().lbm_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc:
            raise LbmError(rc, what)

    @property
    def t(self):
        return int(load().lbm_batch_time(self._ctx))

    def set_tile_rows(self, edge, rows):
        self._chk(load().lbm_batch_set_tile_rows(self._ctx, int(edge), int(rows)), "set_tile_rows")

    def run(self, nsteps, mode=LBM_BATCH_PER_STEP):
        self._chk(load().lbm_batch_run(self._ctx, int(nsteps), int(mode)), "lbm_batch_run")

    def run_steady(self, max_steps, tol, check_every, mode=LBM_BATCH_PER_STEP):
        """lbm_batch_run_steady: returns (steady [nbox] bool, stop_step [nbox])."""
        st = np.zeros(self.nbox, dtype=np.uint8)
        stop = np.zeros(self.nbox, dtype=np.int64)
        self._chk(load().lbm_batch_run_steady(self._ctx, int(max_steps), float(tol), int(check_every), int(mode),
                                              _ptr(st), _ptr(stop)), "lbm_batch_run_steady")
        return st.astype(bool), stop

    def get_drag(self, features=True):
        """lbm_batch_get_drag: (F [nsph, 3] binary64, X [nsph, 40] binary32 or None)."""
        n = max(self.nsph, 1)
        F = np.zeros((n, 3))
        X = np.zeros((n, 40), dtype=np.float32) if features else None
        if self.nsph:
            self._chk(load().lbm_batch_get_drag(self._ctx, _ptr(F), _ptr(X), LBM_HOST), "lbm_batch_get_drag")
        return F[: self.nsph], (X[: self.nsph] if features else None)

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8).reshape(self.nbox))
        self._chk(load().lbm_batch_set_active(self._ctx, _ptr(a)), "set_active")

    def forces(self):
        n = max(self.nsph, 1)
        F = np.zeros((n, 3)); T = np.zeros((n, 3))
        self._chk(load().lbm_batch_forces(self._ctx, _ptr(F), _ptr(T), LBM_HOST), "forces")
        return F[: self.nsph], T[: self.nsph]

    def mean_velocity(self):
        U = np.zeros((self.nbox, 3))
        self._chk(load().lbm_batch_mean_velocity(self._ctx, _ptr(U), LBM_HOST), "mean_velocity")
        return U

    def shell_velocity(self):
        """Mean fluid velocity in the shell [R + 1, 2R] around each sphere, [nsph, 3]."""
        u = np.zeros((self.nsph, 3))
        if self.nsph:
            self._chk(load().lbm_batch_shell_velocity(self._ctx, _ptr(u), LBM_HOST), "shell_velocity")
        return u

    def get_f(self, box):
        L = self.edges[box]
        f = np.empty((19, L, L, L))
        self._chk(load().lbm_batch_get_distributions(self._ctx, int(box), _ptr(f), LBM_HOST), "get_f")
        return f

    def autotune(self, steps=20):
        ne = len(set(self.edges))
        edges = np.zeros(ne, dtype=np.int32); rows = np.zeros(ne, dtype=np.int32)
        mode = np.zeros(1, dtype=np.int32); ms = np.zeros(1)
        self._chk(load().lbm_batch_autotune(self._ctx, int(steps), _ptr(edges), _ptr(rows), _ptr(mode), _ptr(ms)),
                  "autotune")
        return {"rows": {int(e): int(r) for e, r in zip(edges, rows)}, "mode": int(mode[0]),
                "ms_per_step": float(ms[0])}
