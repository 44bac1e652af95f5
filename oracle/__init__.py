"""ctypes access to the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  The product path (the GPU library and its binding)
never imports this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.

Every function here is argument marshalling around the C oracle in
``dgbgk_oracle.c``; the arithmetic lives there.
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PERIODIC = 0
DIFFUSE_WALL = 1

_dp = C.POINTER(C.c_double)


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("y0", C.c_double), ("lx", C.c_double), ("ly", C.c_double),
        ("p", C.c_int), ("q", C.c_int),
        ("ex", _dp), ("ey", _dp), ("w", _dp),
        ("theta", C.c_double), ("tau", C.c_double),
        ("bc", C.c_int * 4), ("wall_u", (C.c_double * 2) * 4),
    ]


_lib = None


def lib():
    """Load liboracle.so, building it first if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    L.oracle_gauss_hermite.argtypes = [C.c_int, _dp, _dp]
    L.oracle_newton_cotes.argtypes = [C.c_int, C.c_double, _dp, _dp]
    L.oracle_tensor_set.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
    L.oracle_second_moment.argtypes = [C.c_int, _dp, _dp]
    L.oracle_second_moment.restype = C.c_double
    L.oracle_tau_from_kn.argtypes = [C.c_double, C.c_double, C.c_int]
    L.oracle_tau_from_kn.restype = C.c_double
    L.oracle_gll_nodes.argtypes = [C.c_int, _dp]
    L.oracle_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    L.oracle_create.argtypes = [C.POINTER(_Problem)]
    L.oracle_create.restype = C.c_void_p
    L.oracle_destroy.argtypes = [C.c_void_p]
    L.oracle_set_threads.argtypes = [C.c_int]
    L.oracle_num_threads.restype = C.c_int
    L.oracle_sizes.argtypes = [C.c_void_p] + [C.POINTER(C.c_int)] * 4
    L.oracle_operator.argtypes = [C.c_void_p, C.c_int, _dp]
    L.oracle_node_coords.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_stable_dt.argtypes = [C.c_void_p, C.c_double, _dp]
    L.oracle_set_state.argtypes = [C.c_void_p, _dp]
    L.oracle_get_state.argtypes = [C.c_void_p, _dp]
    L.oracle_init_equilibrium.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
    L.oracle_equilibrium.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, _dp]
    L.oracle_rhs.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_rhs_parts.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.oracle_wall_density.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_rk4.argtypes = [C.c_void_p, C.c_long, C.c_double]
    L.oracle_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.oracle_residual.argtypes = [C.c_void_p, _dp]
    L.oracle_total_mass.argtypes = [C.c_void_p]
    L.oracle_total_mass.restype = C.c_double
    L.oracle_couette_ux.argtypes = [C.c_double] * 5
    L.oracle_couette_ux.restype = C.c_double
    L.oracle_l2_error_couette.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
    L.oracle_l2_error_couette.restype = C.c_double
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# velocity sets
# --------------------------------------------------------------------------

def gauss_hermite(n):
    """1-D n-point Gauss-Hermite rule (standard normal weight, sum w = 1)."""
    x = np.zeros(n)
    w = np.zeros(n)
    rc = lib().oracle_gauss_hermite(n, _ptr(x), _ptr(w))
    if rc:
        raise ValueError(f"oracle_gauss_hermite({n}) failed: {rc}")
    return x, w


def newton_cotes(m, vmax):
    """1-D m-point composite Newton-Cotes rule on [-vmax, vmax], Maxwellian weighted."""
    x = np.zeros(m)
    w = np.zeros(m)
    rc = lib().oracle_newton_cotes(m, vmax, _ptr(x), _ptr(w))
    if rc:
        raise ValueError(f"oracle_newton_cotes({m}) failed: {rc}")
    return x, w


def tensor_set(x1, w1):
    n = len(x1)
    ex = np.zeros(n * n)
    ey = np.zeros(n * n)
    w = np.zeros(n * n)
    lib().oracle_tensor_set(n, _ptr(_f64(x1)), _ptr(_f64(w1)), _ptr(ex), _ptr(ey), _ptr(w))
    return ex, ey, w


def second_moment(ex, w):
    ex = _f64(ex)
    w = _f64(w)
    return lib().oracle_second_moment(len(ex), _ptr(ex), _ptr(w))


def velocity_set(spec):
    """(ex, ey, w, theta) for a velocity-set spec: ("gh", n) or ("nc", m, vmax),
    or ("custom", ex, ey, w, theta)."""
    kind = spec[0]
    if kind == "gh":
        x1, w1 = gauss_hermite(spec[1])
        ex, ey, w = tensor_set(x1, w1)
        return ex, ey, w, 1.0
    if kind == "nc":
        x1, w1 = newton_cotes(spec[1], spec[2])
        ex, ey, w = tensor_set(x1, w1)
        return ex, ey, w, second_moment(ex, w)
    if kind == "custom":
        return _f64(spec[1]), _f64(spec[2]), _f64(spec[3]), float(spec[4])
    raise ValueError(spec)


def tau_from_kn(kn, L=1.0, convention=1):
    return lib().oracle_tau_from_kn(kn, L, convention)


def gll_nodes(p):
    r = np.zeros(p + 1)
    if lib().oracle_gll_nodes(p, _ptr(r)):
        raise ValueError(p)
    return r


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().oracle_gauss_legendre(n, _ptr(x), _ptr(w))
    return x, w


def couette_ux(y, L, kn, u_top, u_bot):
    return lib().oracle_couette_ux(float(y), float(L), float(kn), float(u_top), float(u_bot))


def set_threads(n):
    lib().oracle_set_threads(int(n))


def num_threads():
    return lib().oracle_num_threads()


# --------------------------------------------------------------------------
# solver
# --------------------------------------------------------------------------

class Oracle:
    """One DG-BGK problem on the CPU oracle.  State layout f[q][k][n], FP64."""

    def __init__(self, nx, ny, p, velset, tau, bc, wall_u, x0=0.0, y0=0.0, lx=1.0, ly=1.0):
        ex, ey, w, theta = velocity_set(velset)
        self.ex, self.ey, self.w, self.theta = ex, ey, w, theta
        self.tau = float(tau)
        pb = _Problem()
        pb.nx, pb.ny, pb.p, pb.q = nx, ny, p, len(ex)
        pb.x0, pb.y0, pb.lx, pb.ly = x0, y0, lx, ly
        pb.ex, pb.ey, pb.w = _ptr(ex), _ptr(ey), _ptr(w)
        pb.theta = theta
        pb.tau = self.tau
        for s in range(4):
            pb.bc[s] = int(bc[s])
            pb.wall_u[s][0] = float(wall_u[s][0])
            pb.wall_u[s][1] = float(wall_u[s][1])
        h = lib().oracle_create(C.byref(pb))
        if not h:
            raise ValueError("oracle_create rejected the problem")
        self._h = h
        K, Np, Nfp, Q = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        lib().oracle_sizes(h, C.byref(K), C.byref(Np), C.byref(Nfp), C.byref(Q))
        self.K, self.Np, self.Nfp, self.Q = K.value, Np.value, Nfp.value, Q.value
        self.nx, self.ny, self.p = nx, ny, p
        self.lx, self.ly = lx, ly

    @classmethod
    def from_spec(cls, spec):
        tau = spec.tau if spec.tau is not None else tau_from_kn(spec.kn, spec.kn_length,
                                                                spec.kn_convention)
        return cls(spec.nx, spec.ny, spec.p, spec.velset, tau, spec.bc, spec.wall_u,
                   spec.x0, spec.y0, spec.lx, spec.ly)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.Q, self.K, self.Np)

    def operator(self, which):
        n1 = self.p + 1
        sizes = {0: self.Np * self.Np, 1: self.Np * self.Np, 2: self.Np * self.Np,
                 3: self.Np * 4 * self.Nfp, 4: n1, 5: n1 * n1, 6: 4, 7: 4 * self.K}
        out = np.zeros(sizes[which])
        if lib().oracle_operator(self._h, which, _ptr(out)):
            raise ValueError(which)
        shapes = {0: (self.Np, self.Np), 1: (self.Np, self.Np), 2: (self.Np, self.Np),
                  3: (self.Np, 4 * self.Nfp), 4: (n1,), 5: (n1, n1), 6: (4,), 7: (self.K, 4)}
        return out.reshape(shapes[which])

    def node_coords(self):
        x = np.zeros(self.K * self.Np)
        y = np.zeros(self.K * self.Np)
        lib().oracle_node_coords(self._h, _ptr(x), _ptr(y))
        return x.reshape(self.K, self.Np), y.reshape(self.K, self.Np)

    def stable_dt(self, cfl):
        dt = C.c_double()
        if lib().oracle_stable_dt(self._h, cfl, C.byref(dt)):
            raise ValueError(cfl)
        return dt.value

    def set_state(self, f):
        f = _f64(f).reshape(-1)
        assert f.size == self.Q * self.K * self.Np
        lib().oracle_set_state(self._h, _ptr(f))

    def get_state(self):
        f = np.zeros(self.Q * self.K * self.Np)
        lib().oracle_get_state(self._h, _ptr(f))
        return f.reshape(self.shape)

    def init_equilibrium(self, rho0=1.0, ux0=0.0, uy0=0.0):
        lib().oracle_init_equilibrium(self._h, rho0, ux0, uy0)

    def equilibrium(self, rho, ux, uy):
        out = np.zeros(self.Q)
        lib().oracle_equilibrium(self._h, rho, ux, uy, _ptr(out))
        return out

    def rhs(self, f=None):
        k = np.zeros(self.Q * self.K * self.Np)
        keep = _f64(f).reshape(-1) if f is not None else None
        fp = _ptr(keep) if keep is not None else None
        lib().oracle_rhs(self._h, fp, _ptr(k))
        return k.reshape(self.shape)

    def rhs_parts(self, f=None):
        n = self.Q * self.K * self.Np
        v, s, c = np.zeros(n), np.zeros(n), np.zeros(n)
        keep = _f64(f).reshape(-1) if f is not None else None
        fp = _ptr(keep) if keep is not None else None
        lib().oracle_rhs_parts(self._h, fp, _ptr(v), _ptr(s), _ptr(c))
        return v.reshape(self.shape), s.reshape(self.shape), c.reshape(self.shape)

    def wall_density(self, f=None):
        out = np.zeros(self.K * 4 * self.Nfp)
        keep = _f64(f).reshape(-1) if f is not None else None
        fp = _ptr(keep) if keep is not None else None
        lib().oracle_wall_density(self._h, fp, _ptr(out))
        return out.reshape(self.K, 4, self.Nfp)

    def rk4(self, nsteps, dt):
        if lib().oracle_rk4(self._h, int(nsteps), float(dt)):
            raise ValueError("oracle_rk4 failed")

    def moments(self):
        n = self.K * self.Np
        rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().oracle_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy))
        return (rho.reshape(self.K, self.Np), ux.reshape(self.K, self.Np),
                uy.reshape(self.K, self.Np))

    def residual(self):
        r = C.c_double()
        rc = lib().oracle_residual(self._h, C.byref(r))
        return r.value, rc

    def total_mass(self):
        return lib().oracle_total_mass(self._h)

    def l2_error_couette(self, kn, u_top, u_bot):
        return lib().oracle_l2_error_couette(self._h, kn, u_top, u_bot)


def couette_kn_eff(tau, L=1.0):
    """Knudsen number of eq. (7) for a given tau: Kn = sqrt(3) tau / L."""
    return math.sqrt(3.0) * tau / L
