"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It never imports the HIP library or its binding.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbimb_oracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: WPS433  (gcc is part of the image)
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        up = C.POINTER(C.c_ubyte)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                 dp, dp, C.c_int, C.c_double, C.c_double]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_coupling.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_particles.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp, dp, up]
        L.orc_set_particles.restype = C.c_int
        for name in ("orc_set_f", "orc_get_f", "orc_get_q", "orc_get_contact_forces"):
            getattr(L, name).argtypes = [C.c_void_p, dp]
            getattr(L, name).restype = C.c_int
        L.orc_get_macro.argtypes = [C.c_void_p, dp, dp]
        L.orc_get_forces.argtypes = [C.c_void_p, dp, dp]
        L.orc_get_particles.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_long
        L.orc_footprint_counts.argtypes = [C.c_void_p, ip]
        L.orc_particle_node_count.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_particle_node_count.restype = C.c_int
        L.orc_collide_node.argtypes = [C.c_int, C.c_double, dp, C.c_int, dp, C.c_int, dp, dp, dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_dem_forces.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, C.c_double, C.c_double,
                                     dp, C.c_int, dp]
        L.orc_sum2.argtypes = [dp, C.c_long]
        L.orc_sum2.restype = C.c_double
        L.orc_beta.argtypes = [C.c_double, C.c_double]
        L.orc_beta.restype = C.c_double
        L.orc_set_eps_mode.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_eps_mode.restype = C.c_int
        L.orc_eps_table_count.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_eps_table_count.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_set_parallel_minimum.argtypes = [C.c_long, C.c_long]
        L.orc_set_parallel_minimum.restype = None
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (n <= 0: every
    core); returns the number in effect.  Results do not depend on it."""
    return lib().orc_set_threads(int(n))


def set_parallel_minimum(nodes=32768, particles=256):
    """Smallest node loop and particle loop that run on several threads (the
    defaults keep small lattices on one thread).  Results do not depend on it."""
    lib().orc_set_parallel_minimum(int(nodes), int(particles))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleSim:
    """FP64 LB-IMB-DEM simulation on the CPU.

    Lattice fields are [.., nz, ny, nx] (x fastest); populations f[Q, nz, ny, nx].
    Particle arrays are [np, 3] (2D: z components zero; omega uses z).
    """

    def __init__(self, dim, shape, tau, wall_y=False, fluid_force=(0, 0, 0),
                 particle_accel=(0, 0, 0), samples=4, kn=0.0, restitution=0.9, eps="sampling"):
        nx, ny = shape[0], shape[1]
        nz = shape[2] if dim == 3 else 1
        self.dim, self.nx, self.ny, self.nz = dim, nx, ny, nz
        self.Q = 9 if dim == 2 else 19
        self.N = nx * ny * nz
        self.np_ = 0
        gf = _f64(list(fluid_force) + [0.0] * (3 - len(fluid_force)))
        ap = _f64(list(particle_accel) + [0.0] * (3 - len(particle_accel)))
        h = lib().orc_create(dim, nx, ny, nz, int(bool(wall_y)), float(tau), _dp(gf), _dp(ap),
                             int(samples), float(kn), float(restitution))
        if not h:
            raise ValueError("oracle rejected the configuration")
        self._h = h
        if eps not in ("sampling", "table"):
            raise ValueError("eps must be 'sampling' or 'table'")
        self._eps = 1 if eps == "table" else 0

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def field_shape(self):
        return (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)

    def set_coupling(self, on):
        lib().orc_set_coupling(self._h, int(bool(on)))

    def set_particles(self, pos, vel=None, omega=None, radius=None, rho_s=None, fixed=None):
        pos = _f64(pos).reshape(-1, 3)
        n = pos.shape[0]
        vel = _f64(np.zeros((n, 3)) if vel is None else vel, (n, 3))
        omega = _f64(np.zeros((n, 3)) if omega is None else omega, (n, 3))
        radius = _f64(radius, (n,))
        rho_s = _f64(rho_s, (n,))
        fx = np.ascontiguousarray(np.zeros(n) if fixed is None else fixed, dtype=np.uint8).reshape(n)
        if n == 0:
            pos = np.zeros((1, 3)); vel = np.zeros((1, 3)); omega = np.zeros((1, 3))
            radius = np.zeros(1); rho_s = np.zeros(1); fx = np.zeros(1, np.uint8)
        rc = lib().orc_set_particles(self._h, n, _dp(pos), _dp(vel), _dp(omega), _dp(radius),
                                     _dp(rho_s), fx.ctypes.data_as(C.POINTER(C.c_ubyte)))
        if rc != 0:
            raise ValueError("oracle rejected the particles")
        self.np_ = n
        if self._eps == 1 and lib().orc_set_eps_mode(self._h, 1) != 0:
            raise ValueError("table lookup needs one particle radius of at least 1")

    def set_f(self, f):
        f = _f64(f).reshape(self.Q, self.N)
        lib().orc_set_f(self._h, _dp(f))

    def get_f(self):
        f = np.empty((self.Q,) + self.field_shape)
        lib().orc_get_f(self._h, _dp(f))
        return f

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def t(self):
        return lib().orc_time(self._h)

    def macro(self):
        rho = np.empty(self.field_shape)
        u = np.empty((self.dim,) + self.field_shape)
        lib().orc_get_macro(self._h, _dp(rho), _dp(u))
        return rho, u

    def q(self):
        q = np.empty((3,) + self.field_shape)
        lib().orc_get_q(self._h, _dp(q))
        return q

    def forces(self):
        F = np.zeros((max(self.np_, 1), 3)); T = np.zeros((max(self.np_, 1), 3))
        lib().orc_get_forces(self._h, _dp(F), _dp(T))
        return F[: self.np_], T[: self.np_]

    def contact_forces(self):
        Fc = np.zeros((max(self.np_, 1), 3))
        lib().orc_get_contact_forces(self._h, _dp(Fc))
        return Fc[: self.np_]

    def particles(self):
        n = max(self.np_, 1)
        x = np.zeros((n, 3)); v = np.zeros((n, 3)); w = np.zeros((n, 3))
        lib().orc_get_particles(self._h, _dp(x), _dp(v), _dp(w))
        return x[: self.np_], v[: self.np_], w[: self.np_]

    def footprint_counts(self):
        c = np.empty(self.field_shape, dtype=np.int32)
        lib().orc_footprint_counts(self._h, c.ctypes.data_as(C.POINTER(C.c_int)))
        return c

    def particle_node_count(self, p, ix, iy, iz=0):
        return lib().orc_particle_node_count(self._h, int(p), int(ix), int(iy), int(iz))


def collide_node(dim, tau, gf, samples, fin, count, vs):
    Q = 9 if dim == 2 else 19
    fin = _f64(fin, (Q,))
    gf = _f64(list(gf) + [0.0] * (3 - len(gf)))
    vs = _f64(list(vs) + [0.0] * (3 - len(vs)))
    fout = np.empty(Q); q = np.empty(3)
    lib().orc_collide_node(dim, float(tau), _dp(gf), int(samples), _dp(fin), int(count), _dp(vs),
                           _dp(fout), _dp(q))
    return fout, q


def feq(dim, rho, u):
    Q = 9 if dim == 2 else 19
    u = _f64(list(u) + [0.0] * (3 - len(u)))
    out = np.empty(Q)
    lib().orc_feq(dim, float(rho), _dp(u), _dp(out))
    return out


def dem_forces(dim, x, v, R, m, kn, restitution, box, wall_y=False):
    x = _f64(x).reshape(-1, 3); n = x.shape[0]
    v = _f64(v, (n, 3)); R = _f64(R, (n,)); m = _f64(m, (n,))
    box = _f64(list(box) + [1.0] * (3 - len(box)))
    Fc = np.empty((n, 3))
    lib().orc_dem_forces(dim, n, _dp(x), _dp(v), _dp(R), _dp(m), float(kn), float(restitution),
                         _dp(box), int(bool(wall_y)), _dp(Fc))
    return Fc


def sum2(p):
    p = _f64(p).ravel()
    return lib().orc_sum2(_dp(p), p.size)


def beta(eps, tau):
    return lib().orc_beta(float(eps), float(tau))


# lattice constants, restated here for test bookkeeping (velocity sets of the
# paper's D2Q9 / D3Q19 schemes; same ordering as the C oracle)
D2Q9_C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
D2Q9_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
D3Q19_C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                    [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
D3Q19_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def velocities(dim):
    return (D2Q9_C, D2Q9_W) if dim == 2 else (D3Q19_C, D3Q19_W)


def eps_table_count(dim, samples, radius, d):
    """Count on the samples^dim scale that the eps lookup table gives a node
    at displacement d = (dx, dy, dz) from the centre of a particle of the
    given radius."""
    d = list(d) + [0.0] * (3 - len(d))
    return lib().orc_eps_table_count(int(dim), int(samples), float(radius), float(d[0]), float(d[1]),
                                     float(d[2]))
