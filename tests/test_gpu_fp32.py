"""GPU parity of the FP32-storage precision path (the state streamed in FP32 as
the deviation from w_q rho_ref; moments, wall densities and residual in FP64)
against the FP64 CPU oracle on the same seeded inputs, and against the GPU
FP64 path at the full precision-workload size; and of its variant with the
volume term's contractions on bf16 matrix cores.  The full-size precision
workload also checks the FP64 path in its velocity-tiled form (bar 1e-12).

Bars: FP32 storage, 1e-5 relative in max-norm on rho and u (normwise over
nodes and components for u, as in the FP64 tests) after the same RK4 steps
and on the right-hand side itself.  bf16 contractions, 2e-3 on rho and u
and on the right-hand side: both factors of the products Dr g, Ds g are
rounded to bf16 (unit roundoff 2^-9 each) after the row mean is subtracted,
so the volume term carries up to about 2 x 2^-9 = 3.9e-3 relative to the
in-element variation of g in the worst case; the rounding errors of the
products' terms are independent and partly cancel, and 2e-3 is the bar the
path is held to."""
import sys

import numpy as np
import pytest

import workloads
from paper_2012_13487_amd import binding

pytestmark = pytest.mark.gpu

TOL64 = 1e-12  # the FP64 path's bar
TOL32 = 1e-5
TOL_BF = 2e-3
TOL_BF_RHS = 2e-3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _moment_errors(mg, mo):
    (rg, uxg, uyg), (ro, uxo, uyo) = mg, mo
    u_g = np.stack([uxg, uyg])
    u_o = np.stack([uxo, uyo])
    return _rel(rg, ro), float(np.max(np.abs(u_g - u_o)) / max(np.max(np.abs(u_o)), 1e-300))


def _pair(oracle_mod, spec, **kw):
    g = binding.Solver.from_spec(spec, precision=binding.FP32, **kw)
    o = oracle_mod.Oracle.from_spec(spec)
    assert g.shape == o.shape
    return g, o


RHS_CASES = [
    ("couette_8x8_p2_gh4", workloads.couette(nx=8, ny=8, p=2)),
    ("cavity_6x5_p3_nc8", workloads.cavity(n=6, ny=5, p=3, m=8, lid=0.1)),
    ("cavity_5x3_p4_nc5_scalar", workloads.cavity(n=5, ny=3, p=4, m=5, lid=0.2)),  # Q Np odd
    ("periodic_7x3_p1_gh3", workloads.periodic_box(nx=7, ny=3, p=1, velset=("gh", 3), kn=0.3)),
    ("cavity_9x7_p3_nc9", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15)),
    ("couette_3x1_p5_gh4", workloads.couette(nx=3, ny=1, p=5)),
    ("cavity_3x2_p6_nc4", workloads.cavity(n=3, ny=2, p=6, m=4)),
    ("cavity_2x3_p7_nc5", workloads.cavity(n=2, ny=3, p=7, m=5, lid=0.2)),
    ("cavity_2x2_p8_nc5_scalar", workloads.cavity(n=2, p=8, m=5)),  # Q Np odd
    ("collisionless_4x4_p3", workloads.periodic_box(nx=4, ny=4, p=3, tau=float("inf"))),
    # strip-ordered blocks: one element per block (20 columns, strips of 16)
    ("cavity_20x3_p2_nc16_strips", workloads.cavity(n=20, ny=3, p=2, m=16, lid=0.1)),
]


@pytest.mark.parametrize("name,spec", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_fp32_rhs_parity(oracle_mod, name, spec):
    _say(f"[gpu] fp32 rhs parity {name}")
    g, o = _pair(oracle_mod, spec)
    assert g.tiling()["fused"]
    f = workloads.perturbed_state(17, o.w, o.K, o.Np, amp=0.2)
    kg = g.rhs(f)
    ko = o.rhs(f)
    assert np.isfinite(kg).all()
    assert _rel(kg, ko) < TOL32, (name, _rel(kg, ko))


@pytest.mark.parametrize("name,spec", RHS_CASES[:3], ids=[c[0] for c in RHS_CASES[:3]])
def test_fp32_wall_density_parity(oracle_mod, name, spec):
    # the wall densities are reduced in FP64 from the FP32 deviation; only the
    # rounding of the stored deviation remains
    _say(f"[gpu] fp32 wall density {name}")
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(5, o.w, o.K, o.Np, amp=0.2)
    wg = g.wall_density(f)
    wo = o.wall_density(f)
    wall = o.operator(7).astype(int) < 0
    if wall.any():
        assert _rel(wg[wall], wo[wall]) < 1e-7
    assert np.all(wg[~wall] == 0.0)


def test_fp32_state_round_trip_and_moments(oracle_mod):
    # set_state / get_state go through the FP32 deviation: exact to the
    # rounding of g; moments are FP64 sums of the stored values
    _say("[gpu] fp32 state round trip")
    spec = workloads.cavity(n=5, p=3, m=8)
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(2, o.w, o.K, o.Np, amp=0.1)
    g.set_state(f)
    dev = f - o.w[:, None, None]
    back = g.get_state() - o.w[:, None, None]
    assert np.max(np.abs(back - dev)) <= 2.0 ** -24 * np.max(np.abs(dev))
    o.set_state(f)
    er, eu = _moment_errors(g.moments(), o.moments())
    assert er < 1e-8 and eu < 1e-6


def test_fp32_init_moments(oracle_mod):
    _say("[gpu] fp32 init_moments")
    spec = workloads.cavity(n=6, p=2, m=8, lid=0.1)
    g, o = _pair(oracle_mod, spec)
    x, y = g.node_coords()
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(np.pi * y)
    ux, uy = 0.1 * np.cos(2 * np.pi * y), -0.08 * np.sin(2 * np.pi * x)
    g.init_moments(rho, ux, uy)
    want = np.empty(o.shape)
    for k in range(o.K):
        for n in range(o.Np):
            want[:, k, n] = o.equilibrium(rho[k, n], ux[k, n], uy[k, n])
    # deviation from w rho_ref stored in FP32: one rounding of a value below |f|
    assert _rel(g.get_state(), want) < 2 ** -23
    o.set_state(want)
    er, eu = _moment_errors(g.moments(), o.moments())
    assert er < TOL32 and eu < TOL32


@pytest.mark.parametrize("p", [5, 7, 8])
def test_fp32_high_order_steps(oracle_mod, p):
    _say(f"[gpu] fp32 steps p={p}")
    spec = workloads.cavity(n=3, ny=2, p=p, m=6, lid=0.1)
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(5, o.w, o.K, o.Np, amp=0.1)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(20, dt)
    o.rk4(20, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"    rho {er:.2e}  u {eu:.2e}")
    assert er < TOL32 and eu < TOL32


def test_fp32_couette_200_steps(oracle_mod):
    _say("[gpu] fp32 couette 8x8 p2 200 steps")
    spec = workloads.COUETTE_8x8_P2_D2Q16
    g, o = _pair(oracle_mod, spec)
    dt = o.stable_dt(spec.cfl)
    g.init_equilibrium()
    o.init_equilibrium()
    g.step(spec.steps, dt)
    o.rk4(spec.steps, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


def test_fp32_cavity_perturbed_steps(oracle_mod):
    _say("[gpu] fp32 cavity 10x7 p3 nc10 perturbed 40 steps")
    spec = workloads.cavity(n=10, ny=7, p=3, m=10, lid=0.1, kn=0.5)
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(23, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(40, dt)
    o.rk4(40, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


def test_fp32_precision_workload_small_mesh(oracle_mod):
    """The precision workload's physics (cavity, Kn = 8, p = 4, NC 24 x 24) on an
    8 x 8 mesh: rho, u after 10 RK4 steps from rest against the oracle."""
    _say("[gpu] fp32 cavity 8x8 p4 nc24 kn8, 10 steps")
    spec = workloads.CAVITY_128x128_P4_NC24_KN8.with_(nx=8, ny=8)
    g, o = _pair(oracle_mod, spec)
    dt = o.stable_dt(spec.cfl)
    g.init_equilibrium()
    o.init_equilibrium()
    g.step(10, dt)
    o.rk4(10, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


def test_fp32_mass_conservation():
    _say("[gpu] fp32 mass conservation")
    spec = workloads.cavity(n=8, p=3, m=10, lid=0.1, kn=0.5)
    g = binding.Solver.from_spec(spec, precision="fp32")
    M = np.kron(g.operator(5), g.operator(5))
    J = (1 / 8) ** 2 / 4
    f = workloads.perturbed_state(8, g.w, g.K, g.Np, amp=0.1)
    g.set_state(f)
    m0 = J * np.einsum("n,kn->", M.sum(axis=0), g.moments()[0])
    g.step(300, g.stable_dt(0.2))
    m1 = J * np.einsum("n,kn->", M.sum(axis=0), g.moments()[0])
    # the deviation form conserves mass up to FP32 rounding of the deviation
    assert abs(m1 - m0) < 1e-7 * m0


def test_fp32_residual_and_determinism(oracle_mod):
    _say("[gpu] fp32 residual / determinism")
    spec = workloads.cavity(n=6, p=2, m=8, lid=0.1)
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(3, o.w, o.K, o.Np, amp=0.1)
    g.set_state(f)
    o.set_state(f)
    rg = g.residual()
    ro, rc = o.residual()
    assert rc == 0 and abs(rg - ro) < TOL32 * ro
    outs = []
    for _ in range(2):
        h = binding.Solver.from_spec(spec, precision=binding.FP32)
        h.init_equilibrium()
        h.step(50, h.stable_dt(0.2))
        outs.append(h.get_state())
    assert np.array_equal(outs[0], outs[1])


BF_CASES = [c for c in RHS_CASES if c[1].p <= 4]


@pytest.mark.parametrize("name,spec", BF_CASES, ids=[c[0] for c in BF_CASES])
def test_bf16_rhs_parity(oracle_mod, name, spec):
    _say(f"[gpu] bf16 rhs parity {name}")
    g = binding.Solver.from_spec(spec, precision=binding.FP32_BF16MMA)
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(17, o.w, o.K, o.Np, amp=0.2)
    e = _rel(g.rhs(f), o.rhs(f))
    _say(f"  err rhs {e:.2e}")
    assert e < TOL_BF_RHS, (name, e)


@pytest.mark.parametrize("spec", [workloads.cavity(n=10, ny=7, p=3, m=10, lid=0.1, kn=0.5),
                                  workloads.COUETTE_8x8_P2_D2Q16],
                         ids=["cavity_10x7_p3_nc10", "couette_8x8_p2"])
def test_bf16_steps(oracle_mod, spec):
    _say(f"[gpu] bf16 {spec.name} 40 steps")
    g = binding.Solver.from_spec(spec, precision="fp32_bf16mma")
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(23, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(40, dt)
    o.rk4(40, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL_BF and eu < TOL_BF, (er, eu)


def test_full_size_precision_workload_all_precisions(oracle_mod):
    """128 x 128 quads, p = 4, NC 24 x 24, Kn = 8 (235.9 M DOF) in the launch
    configuration the benchmark times, for the FP64 path (velocity tiles: one
    element's 576 velocities exceed the fused block's LDS in FP64) and both
    FP32 precisions: the right-hand side of a perturbed state against the
    oracle, and rho, u after 10 RK4 steps from rest against the oracle."""
    _say("[gpu] fp64 / fp32 / bf16 full-size cavity 128x128 p4 nc24 kn8")
    spec = workloads.CAVITY_128x128_P4_NC24_KN8
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(41, o.w, o.K, o.Np, amp=0.05)
    ko = o.rhs(f)
    for prec, tol in ((binding.FP64, TOL64), (binding.FP32, TOL32),
                      (binding.FP32_BF16MMA, TOL_BF_RHS)):
        g = binding.Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
        e = _rel(g.rhs(f), ko)
        _say(f"  rhs prec {prec}: {e:.2e}")
        assert e < tol
        g.close()
    del f, ko
    dt = o.stable_dt(spec.cfl)
    o.init_equilibrium()
    _say("  10 oracle steps")
    o.rk4(10, dt)
    mo = o.moments()
    for prec, tol in ((binding.FP64, TOL64), (binding.FP32, TOL32), (binding.FP32_BF16MMA, TOL_BF)):
        g = binding.Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
        if prec == binding.FP64:
            assert not g.tiling()["fused"]
        g.init_equilibrium()
        g.step(10, dt)
        er, eu = _moment_errors(g.moments(), mo)
        _say(f"  prec {prec}: err rho {er:.2e} u {eu:.2e}")
        assert er < tol and eu < tol, (prec, er, eu)
        g.close()


def test_fp32_against_fp64_gpu_after_2000_steps():
    """The precision workload on the GPU in FP32 and in FP64 from rest, 2000
    RK4 steps each: rho, u agree to the FP32 bar."""
    _say("[gpu] fp32 vs fp64 cavity 128x128 p4 nc24 kn8, 2000 steps")
    spec = workloads.CAVITY_128x128_P4_NC24_KN8
    res = []
    for prec in (binding.FP64, binding.FP32):
        g = binding.Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
        dt = g.stable_dt(spec.cfl)
        g.init_equilibrium()
        for _ in range(4):
            g.step(500, dt)
            g.synchronize()
            _say(f"  prec {prec}: {g.steps_taken()} steps")
        res.append(g.moments())
        g.close()
    er, eu = _moment_errors(res[1], res[0])
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


HANDOFF32_CASES = [
    ("cavity_9x7_p3_nc12", workloads.cavity(n=9, ny=7, p=3, m=12, lid=0.1, kn=0.5)),
    ("couette_6x5_p3_gh4", workloads.couette(nx=6, ny=5, p=3, kn=0.7)),
    ("cavity_7x6_p1_nc10", workloads.cavity(n=7, ny=6, p=1, m=10, lid=0.2, kn=1.5)),
    ("cavity_1x1_p3_nc8", workloads.cavity(n=1, ny=1, p=3, m=8, lid=0.1)),  # four wall faces
]


@pytest.mark.parametrize("prec", [binding.FP32, binding.FP32_REF, binding.FP32_BF16MMA])
@pytest.mark.parametrize("name,spec", HANDOFF32_CASES, ids=[c[0] for c in HANDOFF32_CASES])
def test_fp32_moment_handoff_matches_oracle(oracle_mod, name, spec, prec):
    """One-element blocks of orders 1 and 3 take the FP64 moments of their
    input from the update pass of the stage before (a moment pass over g_n
    first): steps, residuals between them, a state set again, and (reference
    form) a fold, against the oracle."""
    pname = {v: k for k, v in binding.PRECISIONS.items()}[prec]
    _say(f"[gpu] FP32 moment handoff {name} {pname}")
    tol = TOL_BF if prec == binding.FP32_BF16MMA else TOL32
    g = binding.Solver.from_spec(spec, precision=prec)
    o = oracle_mod.Oracle.from_spec(spec)
    g.set_block_elements(1)
    assert g.tiling()["elems_per_group"] == 1
    f = workloads.perturbed_state(67, o.w, o.K, o.Np, amp=0.05)
    dt = o.stable_dt(0.2)
    for s_ in (g, o):
        s_.set_state(f)
    g.step(6, dt)
    o.rk4(6, dt)
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < tol * r
    if prec == binding.FP32_REF:
        g.fold()
    g.step(6, dt)
    o.rk4(6, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    assert er < tol and eu < tol, (er, eu)
    f2 = workloads.perturbed_state(71, o.w, o.K, o.Np, amp=0.05)
    for s_ in (g, o):
        s_.set_state(f2)
    g.step(8, dt)
    o.rk4(8, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < tol and eu < tol, (er, eu)


def test_fp32_moment_handoff_batch_matches_solo():
    """FP32 and reference-form members with one-element blocks form their own
    batch classes (kernels that hand the moments over): states and residuals
    agree bit for bit with the same solvers stepped alone, across a graph
    replay, solo steps of the members in between, and a fold."""
    _say("[gpu] FP32 moment handoff in a batch")
    specs = [(c[1], p) for c in HANDOFF32_CASES[:3]
             for p in (binding.FP32, binding.FP32_REF)]
    def make():
        out = []
        for i, (sp, prec) in enumerate(specs):
            g = binding.Solver.from_spec(sp, precision=prec)
            g.set_block_elements(1)
            g.set_state(workloads.perturbed_state(73 + i, g.w, g.K, g.Np, amp=0.05))
            out.append(g)
        return out
    bm, solo = make(), make()
    dts = np.array([g.stable_dt(0.2) for g in bm])
    b = binding.Batch(bm, graph=3)
    b.step(7, dts)
    for g, dt in zip(solo, dts):
        g.step(7, dt)
    rb = b.residuals()
    for i, (x, y) in enumerate(zip(bm, solo)):
        assert np.array_equal(x.get_state(), y.get_state()), i
        assert rb[i] == y.residual(), i
    for i, (x, y, dt) in enumerate(zip(bm, solo, dts)):
        if specs[i][1] == binding.FP32_REF:
            x.fold()
            y.fold()
        x.step(3, dt)
        y.step(3, dt)
    b.step(4, dts)
    for g, dt in zip(solo, dts):
        g.step(4, dt)
    for i, (x, y) in enumerate(zip(bm, solo)):
        assert np.array_equal(x.get_state(), y.get_state()), i
    b.close()


def test_moment_handoff_streaming_hints_against_fp64_gpu():
    """A cavity large enough (96x96 p=3 NC 16x16, 604 MB per FP32 state set)
    that the FP32 and reference-form stages move their once-read streams with
    non-temporal hints, in the one-element blocks that hand their moments on:
    50 RK4 steps of a perturbed state against the FP64 GPU path (itself held
    to the oracle at 1e-12), at the FP32 bar."""
    _say("[gpu] moment handoff with streaming hints: 96x96 p3 nc16 vs FP64 GPU")
    spec = workloads.cavity(n=96, p=3, m=16, lid=0.1)
    res = {}
    for prec in (binding.FP64, binding.FP32, binding.FP32_REF):
        g = binding.Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
        assert g.tiling()["fused"] and g.tiling()["elems_per_group"] == 1
        g.set_state(workloads.perturbed_state(79, g.w, g.K, g.Np, amp=0.05))
        g.step(50, g.stable_dt(spec.cfl))
        res[prec] = g.moments()
        g.close()
    for prec in (binding.FP32, binding.FP32_REF):
        er, eu = _moment_errors(res[prec], res[binding.FP64])
        _say(f"  precision {prec}: err rho {er:.2e} u {eu:.2e}")
        assert er < TOL32 and eu < TOL32, (prec, er, eu)
