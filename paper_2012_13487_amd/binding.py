"""ctypes binding of ``libdgbgk.so`` (C ABI: include/dgbgk.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch is used, when asked, only to provide device memory
(``dgbgk_bind_buffers``) and the HIP stream the library enqueues on.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgbgk.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_DIFFUSE_WALL = 0, 1
FP64, FP32, FP32_BF16MMA, FP32_REF, FP32_BF16MMA_REF = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32_bf16mma": FP32_BF16MMA, "fp32_ref": FP32_REF,
              "fp32_bf16mma_ref": FP32_BF16MMA_REF}

_dp = C.POINTER(C.c_double)


class DgbgkError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"dgbgk error {code}: {message}")
        self.code = code


class Problem(C.Structure):
    """Mirror of dgbgk_problem."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("x0", C.c_double), ("y0", C.c_double), ("lx", C.c_double), ("ly", C.c_double),
        ("p", C.c_int32), ("q", C.c_int32),
        ("ex", _dp), ("ey", _dp), ("w", _dp),
        ("theta", C.c_double), ("tau", C.c_double),
        ("bc", C.c_int32 * 4), ("wall_u", (C.c_double * 2) * 4),
    ]


class ServerOptions(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_active", C.c_int32), ("precision", C.c_int32),
                ("residual_target", C.c_double), ("check_every", C.c_int32),
                ("max_steps", C.c_int64), ("cfl", C.c_double), ("use_graph", C.c_int32),
                ("polish_below", C.c_double)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("arrival_s", C.c_double), ("admit_s", C.c_double),
                ("finish_s", C.c_double), ("steps", C.c_int64), ("residual", C.c_double),
                ("dof", C.c_int64), ("K", C.c_int64), ("Np", C.c_int64),
                ("steps_fp64", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("wall_s", C.c_double),
                ("dof_updates", C.c_double), ("latency_p50_s", C.c_double),
                ("latency_p99_s", C.c_double), ("batch_rebuilds", C.c_int64),
                ("chunks", C.c_int64), ("peak_active", C.c_int32), ("peak_bytes", C.c_size_t),
                ("precision_switches", C.c_int64), ("dof_updates_all", C.c_double),
                ("admitted", C.c_int64)]


class ImplicitOptions(C.Structure):
    """Mirror of dgbgk_implicit_options."""
    _fields_ = [("max_newton", C.c_int32), ("newton_rtol", C.c_double),
                ("newton_atol", C.c_double), ("restart", C.c_int32), ("max_krylov", C.c_int32),
                ("krylov_rtol", C.c_double), ("krylov_fp32", C.c_int32)]


class ImplicitReport(C.Structure):
    """Mirror of dgbgk_implicit_report."""
    _fields_ = [("newton_iterations", C.c_int32), ("krylov_iterations", C.c_int32),
                ("rhs_evaluations", C.c_int32), ("max_final_residual", C.c_double),
                ("converged", C.c_int32)]


BACKWARD_EULER, SDIRK2, SDIRK4 = 0, 1, 2
SCHEMES = {"backward_euler": BACKWARD_EULER, "sdirk2": SDIRK2, "sdirk4": SDIRK4}

REQ_WAITING, REQ_RUNNING, REQ_CONVERGED, REQ_STOPPED, REQ_FAILED = 0, 1, 2, 3, 4

# name -> (restype, argtypes) for every function declared in include/dgbgk.h
SIGNATURES = {
    "dgbgk_velset_gh": (C.c_int, [C.c_int32, _dp, _dp, _dp, _dp]),
    "dgbgk_velset_nc": (C.c_int, [C.c_int32, C.c_double, _dp, _dp, _dp, _dp]),
    "dgbgk_tau_from_kn": (C.c_int, [C.c_double, C.c_double, C.c_int32, _dp]),
    "dgbgk_required_bytes": (C.c_int, [C.POINTER(Problem), C.c_int32, C.POINTER(C.c_size_t)]),
    "dgbgk_create": (C.c_int, [C.POINTER(Problem), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dgbgk_bind_buffers": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "dgbgk_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dgbgk_destroy": (None, [C.c_void_p]),
    "dgbgk_last_error": (C.c_char_p, [C.c_void_p]),
    "dgbgk_version": (C.c_char_p, []),
    "dgbgk_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dgbgk_stable_dt": (C.c_int, [C.c_void_p, C.c_double, _dp]),
    "dgbgk_node_coords": (C.c_int, [C.c_void_p, _dp, _dp]),
    "dgbgk_get_operator": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "dgbgk_init_equilibrium": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double]),
    "dgbgk_init_moments": (C.c_int, [C.c_void_p, _dp, _dp, _dp, C.c_size_t]),
    "dgbgk_set_state": (C.c_int, [C.c_void_p, _dp, C.c_size_t]),
    "dgbgk_get_state": (C.c_int, [C.c_void_p, _dp, C.c_size_t]),
    "dgbgk_state_device_ptr": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "dgbgk_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_double]),
    "dgbgk_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "dgbgk_rhs": (C.c_int, [C.c_void_p, _dp, _dp, C.c_size_t]),
    "dgbgk_implicit_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_double,
                                      C.POINTER(ImplicitOptions), C.POINTER(ImplicitReport)]),
    "dgbgk_implicit_step_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_double,
                                              C.POINTER(ImplicitOptions),
                                              C.POINTER(ImplicitReport)]),
    "dgbgk_wall_density": (C.c_int, [C.c_void_p, _dp, _dp, C.c_size_t]),
    "dgbgk_residual": (C.c_int, [C.c_void_p, _dp]),
    "dgbgk_residual_async": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dgbgk_moments": (C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    "dgbgk_synchronize": (C.c_int, [C.c_void_p]),
    "dgbgk_fold": (C.c_int, [C.c_void_p]),
    "dgbgk_set_tiling": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "dgbgk_get_tiling": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]),
    "dgbgk_steps_taken": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "dgbgk_set_block_elements": (C.c_int, [C.c_void_p, C.c_int32]),
    "dgbgk_autotune": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "dgbgk_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "dgbgk_batch_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "dgbgk_batch_step": (C.c_int, [C.c_void_p, C.c_int64, _dp]),
    "dgbgk_batch_residuals": (C.c_int, [C.c_void_p, _dp]),
    "dgbgk_batch_launches_per_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "dgbgk_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "dgbgk_batch_destroy": (None, [C.c_void_p]),
    "dgbgk_server_create": (C.c_int, [C.POINTER(ServerOptions), C.c_void_p, C.POINTER(C.c_void_p)]),
    "dgbgk_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Problem), C.c_double,
                                      C.POINTER(C.c_int64)]),
    "dgbgk_server_run": (C.c_int, [C.c_void_p, C.c_double]),
    "dgbgk_server_result": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(RequestResult)]),
    "dgbgk_server_moments": (C.c_int, [C.c_void_p, C.c_int64, _dp, _dp, _dp]),
    "dgbgk_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "dgbgk_server_last_error": (C.c_char_p, [C.c_void_p]),
    "dgbgk_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch ships its own HIP runtime with the same soname as ROCm's; load it
        # first so that the library binds to that copy and the process keeps a
        # single HIP runtime (device pointers and streams are then shared).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _check(rc, handle=None):
    if rc != OK:
        msg = lib().dgbgk_last_error(handle).decode(errors="replace")
        raise DgbgkError(rc, msg)


def _bcheck(rc, handle=None):
    if rc != OK:
        msg = lib().dgbgk_batch_last_error(handle).decode(errors="replace")
        raise DgbgkError(rc, msg)


def version():
    return lib().dgbgk_version().decode()


def velset_gh(n1d):
    q = n1d * n1d
    ex, ey, w, th = np.zeros(q), np.zeros(q), np.zeros(q), C.c_double()
    _check(lib().dgbgk_velset_gh(n1d, _p(ex), _p(ey), _p(w), C.byref(th)))
    return ex, ey, w, th.value


def velset_nc(m1d, vmax):
    q = m1d * m1d
    ex, ey, w, th = np.zeros(q), np.zeros(q), np.zeros(q), C.c_double()
    _check(lib().dgbgk_velset_nc(m1d, vmax, _p(ex), _p(ey), _p(w), C.byref(th)))
    return ex, ey, w, th.value


def velocity_set(spec):
    """(ex, ey, w, theta) for ("gh", n) | ("nc", m, vmax) | ("custom", ex, ey, w, theta)."""
    if spec[0] == "gh":
        return velset_gh(spec[1])
    if spec[0] == "nc":
        return velset_nc(spec[1], spec[2])
    if spec[0] == "custom":
        return (np.ascontiguousarray(spec[1], float), np.ascontiguousarray(spec[2], float),
                np.ascontiguousarray(spec[3], float), float(spec[4]))
    raise ValueError(spec)


def tau_from_kn(kn, L=1.0, convention=1):
    t = C.c_double()
    _check(lib().dgbgk_tau_from_kn(kn, L, convention, C.byref(t)))
    return t.value


def _problem(nx, ny, p, vel, tau, bc, wall_u, x0, y0, lx, ly):
    ex, ey, w, theta = vel
    pb = Problem()
    pb.nx, pb.ny, pb.p, pb.q = int(nx), int(ny), int(p), len(ex)
    pb.x0, pb.y0, pb.lx, pb.ly = x0, y0, lx, ly
    pb.ex, pb.ey, pb.w = _p(ex), _p(ey), _p(w)
    pb.theta, pb.tau = float(theta), float(tau)
    for s in range(4):
        pb.bc[s] = int(bc[s])
        pb.wall_u[s][0], pb.wall_u[s][1] = float(wall_u[s][0]), float(wall_u[s][1])
    return pb


def required_bytes(nx, ny, p, vel, tau, bc, wall_u, x0=0.0, y0=0.0, lx=1.0, ly=1.0,
                   precision=FP64):
    pb = _problem(nx, ny, p, vel, tau, bc, wall_u, x0, y0, lx, ly)
    n = C.c_size_t()
    _check(lib().dgbgk_required_bytes(C.byref(pb), _prec(precision), C.byref(n)))
    return n.value


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


class Solver:
    """One DG-BGK problem on the GPU.  Host state arrays f[q][k][n], FP64.

    ``stream``: a HIP stream handle (int) or "torch" for torch's current
    stream; ``torch_memory``: take device memory from a torch tensor;
    ``precision``: FP64, FP32, FP32_BF16MMA, FP32_REF or FP32_BF16MMA_REF (or
    "fp64", "fp32", "fp32_bf16mma", "fp32_ref", "fp32_bf16mma_ref")."""

    def __init__(self, nx, ny, p, velset, tau, bc, wall_u, x0=0.0, y0=0.0, lx=1.0, ly=1.0,
                 stream=None, torch_memory=False, precision=FP64):
        self.precision = _prec(precision)
        self._h = None
        self.vel = velocity_set(velset)
        self.ex, self.ey, self.w, self.theta = self.vel
        self.tau = float(tau)
        pb = _problem(nx, ny, p, self.vel, tau, bc, wall_u, x0, y0, lx, ly)
        self._buf = None
        if stream == "torch" or torch_memory:
            import torch  # plumbing only: device memory and streams
            if stream == "torch":
                stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib().dgbgk_create(C.byref(pb), self.precision, C.c_void_p(stream or 0), C.byref(h)))
        self._h = h.value
        K, Np, Nfp, Q = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        self._call("dgbgk_sizes", C.byref(K), C.byref(Np), C.byref(Nfp), C.byref(Q))
        self.K, self.Np, self.Nfp, self.Q = K.value, Np.value, Nfp.value, Q.value
        self.nx, self.ny, self.p = nx, ny, p
        self.lx, self.ly = lx, ly
        if torch_memory:
            import torch
            nbytes = C.c_size_t()
            _check(lib().dgbgk_required_bytes(C.byref(pb), self.precision, C.byref(nbytes)))
            self._buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
            self._call("dgbgk_bind_buffers", C.c_void_p(self._buf.data_ptr()), nbytes.value)

    @classmethod
    def from_spec(cls, spec, **kw):
        tau = spec.tau if spec.tau is not None else tau_from_kn(spec.kn, spec.kn_length,
                                                                spec.kn_convention)
        return cls(spec.nx, spec.ny, spec.p, spec.velset, tau, spec.bc, spec.wall_u,
                   spec.x0, spec.y0, spec.lx, spec.ly, **kw)

    def _call(self, name, *args):
        _check(getattr(lib(), name)(self._h, *args), self._h)

    def close(self):
        if self._h:
            lib().dgbgk_destroy(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.Q, self.K, self.Np)

    @property
    def ndof(self):
        return self.Q * self.K * self.Np

    # -- host-only queries
    def stable_dt(self, cfl):
        dt = C.c_double()
        self._call("dgbgk_stable_dt", cfl, C.byref(dt))
        return dt.value

    def node_coords(self):
        x, y = np.zeros(self.K * self.Np), np.zeros(self.K * self.Np)
        self._call("dgbgk_node_coords", _p(x), _p(y))
        return x.reshape(self.K, self.Np), y.reshape(self.K, self.Np)

    def operator(self, which):
        n1 = self.p + 1
        shapes = {0: (self.Np, self.Np), 1: (self.Np, self.Np), 2: (self.Np, self.Np),
                  3: (self.Np, 4 * self.Nfp), 4: (n1,), 5: (n1, n1), 6: (4,), 7: (n1, n1)}
        out = np.zeros(int(np.prod(shapes[which])))
        self._call("dgbgk_get_operator", which, _p(out))
        return out.reshape(shapes[which])

    def set_tiling(self, mode, velocities_per_tile=0):
        self._call("dgbgk_set_tiling", mode, velocities_per_tile)

    def set_block_elements(self, elems_per_group):
        self._call("dgbgk_set_block_elements", int(elems_per_group))

    def autotune(self, launches=5):
        us = C.c_double()
        self._call("dgbgk_autotune", int(launches), C.byref(us))
        return us.value

    def tiling(self):
        fused, e, qt, lds = C.c_int32(), C.c_int32(), C.c_int32(), C.c_size_t()
        self._call("dgbgk_get_tiling", C.byref(fused), C.byref(e), C.byref(qt), C.byref(lds))
        return {"fused": bool(fused.value), "persistent": fused.value == 2,
                "elems_per_group": e.value, "velocities_per_tile": qt.value,
                "lds_bytes": lds.value}

    # -- device work
    def init_moments(self, rho, ux, uy):
        """f = f^eq(rho, u) node by node; arrays of shape (K, Np) or K*Np."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, ux, uy)]
        self._call("dgbgk_init_moments", _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), arrs[0].size)

    def init_equilibrium(self, rho0=1.0, ux0=0.0, uy0=0.0):
        self._call("dgbgk_init_equilibrium", rho0, ux0, uy0)

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        self._call("dgbgk_set_state", _p(f), f.size)

    def get_state(self):
        f = np.zeros(self.ndof)
        self._call("dgbgk_get_state", _p(f), f.size)
        return f.reshape(self.shape)

    def set_stream(self, stream):
        """Later calls enqueue on stream (a HIP stream handle, or "torch" for
        torch's current stream)."""
        if stream == "torch":
            import torch  # plumbing only: the stream
            stream = torch.cuda.current_stream().cuda_stream
        self._call("dgbgk_set_stream", C.c_void_p(stream or 0))

    def state_device_ptr(self):
        ptr = C.c_void_p()
        self._call("dgbgk_state_device_ptr", C.byref(ptr))
        return ptr.value

    def step(self, nsteps, dt):
        self._call("dgbgk_step", int(nsteps), float(dt))

    def set_graph(self, steps_per_graph):
        """Replay steps_per_graph RK4 steps at a time from a captured hipGraph
        (0: ordinary launches)."""
        self._call("dgbgk_set_graph", int(steps_per_graph))

    def implicit_step(self, nsteps, dt, scheme="backward_euler", max_newton=20, newton_rtol=1e-10,
                      newton_atol=1e-14, restart=30, max_krylov=300, krylov_rtol=1e-6,
                      krylov_fp32=False, noalloc=False):
        """nsteps SDIRK steps (Newton with matrix-free GMRES); returns the report as a dict.
        krylov_fp32: store the Krylov basis in FP32 (needs krylov_rtol >= 1e-5).
        noalloc: the allocation-free entry point (workspace in the library's
        static 64 MiB per-device array)."""
        sc = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        o = ImplicitOptions(int(max_newton), float(newton_rtol), float(newton_atol), int(restart),
                            int(max_krylov), float(krylov_rtol), int(krylov_fp32))
        r = ImplicitReport()
        self._call("dgbgk_implicit_step_noalloc" if noalloc else "dgbgk_implicit_step", sc,
                   int(nsteps), float(dt), C.byref(o), C.byref(r))
        return {name: getattr(r, name) for name, _ in ImplicitReport._fields_}

    def rhs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        k = np.zeros(self.ndof)
        self._call("dgbgk_rhs", _p(f), _p(k), f.size)
        return k.reshape(self.shape)

    def wall_density(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        out = np.zeros(self.K * 4 * self.Nfp)
        self._call("dgbgk_wall_density", _p(f), _p(out), f.size)
        return out.reshape(self.K, 4, self.Nfp)

    def residual(self):
        r = C.c_double()
        self._call("dgbgk_residual", C.byref(r))
        return r.value

    def residual_async(self, device_ptr):
        self._call("dgbgk_residual_async", C.c_void_p(device_ptr))

    def moments(self):
        n = self.K * self.Np
        rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
        self._call("dgbgk_moments", _p(rho), _p(ux), _p(uy))
        return (rho.reshape(self.K, self.Np), ux.reshape(self.K, self.Np),
                uy.reshape(self.K, self.Np))

    def synchronize(self):
        self._call("dgbgk_synchronize")

    def fold(self):
        """Reference forms: move the FP32 correction into the FP64 reference."""
        self._call("dgbgk_fold")

    def steps_taken(self):
        s = C.c_int64()
        self._call("dgbgk_steps_taken", C.byref(s))
        return s.value


class Batch:
    """Several Solvers advanced together by persistent batched kernels (one
    launch per class of precision / order / tile per RK stage), optionally
    replaying each RK4 step from a captured hipGraph.  The solvers must
    outlive the batch."""

    def __init__(self, solvers, stream=None, graph=False):
        self.solvers = list(solvers)
        if stream == "torch":
            import torch  # plumbing only: the stream
            stream = torch.cuda.current_stream().cuda_stream
        arr = (C.c_void_p * len(self.solvers))(*[s._h for s in self.solvers])
        h = C.c_void_p()
        _bcheck(lib().dgbgk_batch_create(arr, len(self.solvers), C.c_void_p(stream or 0),
                                         C.byref(h)))
        self._h = h.value
        if graph:
            self.set_graph(graph)

    def set_graph(self, steps_per_graph):
        """Replay steps_per_graph RK4 steps at a time from a captured hipGraph
        (True: one step; 0 / False: ordinary launches)."""
        _bcheck(lib().dgbgk_batch_set_graph(self._h, int(steps_per_graph)), self._h)

    def step(self, nsteps, dt):
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64),
                                                  (len(self.solvers),)))
        _bcheck(lib().dgbgk_batch_step(self._h, int(nsteps), _p(dt)), self._h)

    def residuals(self):
        r = np.zeros(len(self.solvers))
        _bcheck(lib().dgbgk_batch_residuals(self._h, _p(r)), self._h)
        return r

    def launches_per_step(self):
        n = C.c_int32()
        _bcheck(lib().dgbgk_batch_launches_per_step(self._h, C.byref(n)), self._h)
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().dgbgk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Steady-state solves under continuous batching (dgbgk_server_*): submit
    problems with arrival times, run, then read per-request results and
    latency / throughput statistics."""

    def __init__(self, hbm_budget, max_active=64, precision=FP64, residual_target=1e-6,
                 check_every=50, max_steps=10 ** 6, cfl=0.2, graph=True, stream=None,
                 polish_below=None):
        if stream == "torch":
            import torch  # plumbing only: the stream
            stream = torch.cuda.current_stream().cuda_stream
        if polish_below is None:  # FP32 precisions: finish in FP64 below 15 x the target
            polish_below = (0.0 if _prec(precision) in (FP64, FP32_REF, FP32_BF16MMA_REF)
                            else 15.0 * residual_target)
        opt = ServerOptions(int(hbm_budget), int(max_active), _prec(precision),
                            float(residual_target), int(check_every), int(max_steps), float(cfl),
                            int(bool(graph)), float(polish_below))
        h = C.c_void_p()
        rc = lib().dgbgk_server_create(C.byref(opt), C.c_void_p(stream or 0), C.byref(h))
        if rc != OK:
            raise DgbgkError(rc, "invalid server options")
        self._h = h.value
        self._vel = []  # keeps submitted velocity arrays alive until submit copies them

    def _check(self, rc):
        if rc != OK:
            raise DgbgkError(rc, lib().dgbgk_server_last_error(self._h).decode(errors="replace"))

    def submit(self, spec, arrival_s):
        vel = velocity_set(spec.velset)
        tau = spec.tau if spec.tau is not None else tau_from_kn(spec.kn, spec.kn_length,
                                                                spec.kn_convention)
        pb = _problem(spec.nx, spec.ny, spec.p, vel, tau, spec.bc, spec.wall_u, spec.x0, spec.y0,
                      spec.lx, spec.ly)
        rid = C.c_int64()
        self._check(lib().dgbgk_server_submit(self._h, C.byref(pb), float(arrival_s),
                                              C.byref(rid)))
        return rid.value

    def run(self, time_limit_s=600.0):
        self._check(lib().dgbgk_server_run(self._h, float(time_limit_s)))

    def result(self, rid):
        r = RequestResult()
        self._check(lib().dgbgk_server_result(self._h, int(rid), C.byref(r)))
        return {f: getattr(r, f) for f, _ in RequestResult._fields_}

    def moments(self, rid):
        r = self.result(rid)
        n = r["K"] * r["Np"]
        rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
        self._check(lib().dgbgk_server_moments(self._h, int(rid), _p(rho), _p(ux), _p(uy)))
        return rho, ux, uy

    def stats(self):
        st = ServerStats()
        self._check(lib().dgbgk_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().dgbgk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
