"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  FP64 bar: 1e-12 relative in max-norm (right-hand
side, wall densities, and rho, u after the same RK4 steps)."""
import math
import sys

import numpy as np
import pytest

import workloads
from paper_2012_13487_amd import binding

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _pair(oracle_mod, spec, tiling=None, **kw):
    g = binding.Solver.from_spec(spec, **kw)
    if tiling is not None:
        g.set_tiling(*tiling)
    o = oracle_mod.Oracle.from_spec(spec)
    assert g.shape == o.shape
    return g, o


def _moment_errors(g, o):
    rg, uxg, uyg = g.moments()
    ro, uxo, uyo = o.moments()
    u_g = np.stack([uxg, uyg])
    u_o = np.stack([uxo, uyo])
    return _rel(rg, ro), float(np.max(np.abs(u_g - u_o)) / max(np.max(np.abs(u_o)), 1e-300))


RHS_CASES = [
    ("couette_8x8_p2_gh4", workloads.couette(nx=8, ny=8, p=2), None),
    ("cavity_6x5_p3_nc8", workloads.cavity(n=6, ny=5, p=3, m=8, lid=0.1), None),
    ("cavity_5x3_p4_nc6_tiled", workloads.cavity(n=5, ny=3, p=4, m=6, lid=0.2), (2, 7)),
    ("periodic_7x3_p1_gh3", workloads.periodic_box(nx=7, ny=3, p=1, velset=("gh", 3), kn=0.3), None),
    ("periodic_1x1_p2_gh4", workloads.periodic_box(nx=1, ny=1, p=2, velset=("gh", 4)), None),
    ("couette_3x1_p5_gh4", workloads.couette(nx=3, ny=1, p=5), None),
    ("cavity_2x2_p8_nc4", workloads.cavity(n=2, p=8, m=4), None),
    ("cavity_9x7_p3_nc9_oddQ", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15), None),
    ("cavity_9x7_p3_nc9_tiled", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15), (2, 10)),
    ("cavity_9x7_p3_nc9_persistent", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15), (4, 0)),
    ("couette_8x8_p2_gh4_persistent", workloads.couette(nx=8, ny=8, p=2), (4, 0)),
    ("collisionless_4x4_p3", workloads.periodic_box(nx=4, ny=4, p=3, tau=float("inf")), None),
    # strip-ordered blocks with full strips and a narrower last strip:
    # one element per block (20 columns, strips of 16), two (20 blocks of 2, strips of 8)
    ("cavity_20x3_p2_nc16_strips_E1", workloads.cavity(n=20, ny=3, p=2, m=16, lid=0.1), None),
    ("cavity_40x2_p3_nc10_strips_E2", workloads.cavity(n=40, ny=2, p=3, m=10, lid=0.1), None),
    # the fused forms at higher orders (the tiles of small p = 4 batch and
    # serving members, and orders 6 and 7, which the ABI accepts)
    ("cavity_6x5_p4_nc6_fused", workloads.cavity(n=6, ny=5, p=4, m=6, lid=0.1), None),
    ("cavity_5x4_p4_nc12_fused", workloads.cavity(n=5, ny=4, p=4, m=12, lid=0.15, kn=0.4), None),
    ("cavity_4x3_p6_nc5_fused", workloads.cavity(n=4, ny=3, p=6, m=5, lid=0.1), None),
    ("couette_3x2_p7_gh4_fused", workloads.couette(nx=3, ny=2, p=7), None),
    # the largest velocity set the ABI takes (4096 = NC 64 x 64): velocity tiles with
    # a moments pass before every stage (more tiles than partials are kept for)
    ("cavity_2x2_p2_nc64_maxQ", workloads.cavity(n=2, p=2, m=64, lid=0.1), None),
]


@pytest.mark.parametrize("name,spec,tiling", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_rhs_parity(oracle_mod, name, spec, tiling):
    _say(f"[gpu] rhs parity {name}")
    g, o = _pair(oracle_mod, spec, tiling)
    f = workloads.perturbed_state(17, o.w, o.K, o.Np, amp=0.2)
    kg = g.rhs(f)
    ko = o.rhs(f)
    assert np.isfinite(kg).all()
    assert _rel(kg, ko) < TOL, (name, _rel(kg, ko))


@pytest.mark.parametrize("name,spec,tiling", RHS_CASES[:4] + RHS_CASES[7:9],
                         ids=[c[0] for c in RHS_CASES[:4] + RHS_CASES[7:9]])
def test_wall_density_parity(oracle_mod, name, spec, tiling):
    _say(f"[gpu] wall density parity {name}")
    g, o = _pair(oracle_mod, spec, tiling)
    f = workloads.perturbed_state(5, o.w, o.K, o.Np, amp=0.2)
    wg = g.wall_density(f)
    wo = o.wall_density(f)
    wall = o.operator(7).astype(int) < 0
    if wall.any():
        assert _rel(wg[wall], wo[wall]) < TOL
    assert np.all(wg[~wall] == 0.0)


def test_couette_200_steps_matches_oracle(oracle_mod):
    """Couette 8x8, p=2, D2Q16, Kn=1 (tau = Kn/sqrt(pi/2)), CFL 0.2, 200 steps."""
    _say("[gpu] couette 8x8 p2 200 steps")
    spec = workloads.COUETTE_8x8_P2_D2Q16
    g, o = _pair(oracle_mod, spec)
    dt = o.stable_dt(spec.cfl)
    assert g.stable_dt(spec.cfl) == pytest.approx(dt, rel=1e-15)
    g.init_equilibrium()
    o.init_equilibrium()
    g.step(spec.steps, dt)
    o.rk4(spec.steps, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)
    rho, ux, uy = g.moments()
    assert np.max(np.abs(rho - 1)) < 1e-13 and np.max(np.abs(uy)) < 1e-14
    assert g.steps_taken() == spec.steps


STRIP_CASES = [c for c in RHS_CASES if "_strips_" in c[0]]


@pytest.mark.parametrize("name,spec,tiling", STRIP_CASES, ids=[c[0] for c in STRIP_CASES])
def test_strip_ordered_blocks_steps_match_oracle(oracle_mod, name, spec, tiling):
    _say(f"[gpu] strip-ordered blocks, 20 steps: {name}")
    g, o = _pair(oracle_mod, spec, tiling)
    assert g.tiling()["elems_per_group"] == (1 if "E1" in name else 2)
    f = workloads.perturbed_state(29, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(20, dt)
    o.rk4(20, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)
    assert _rel(g.get_state(), o.get_state()) < TOL


FUSED_HIGH_ORDER = [c for c in RHS_CASES if c[0].endswith("_fused")]


def test_largest_velocity_set_steps_match_oracle(oracle_mod):
    """Q = 4096 (NC 64 x 64) on a 2x2 p = 2 cavity: 10 RK4 steps in the
    automatic (velocity-tiled) form against the oracle."""
    _say("[gpu] largest velocity set, 10 steps")
    spec = workloads.cavity(n=2, p=2, m=64, lid=0.1)
    g, o = _pair(oracle_mod, spec)
    assert g.Q == 4096 and g.tiling()["fused"] == 0
    f = workloads.perturbed_state(47, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(10, dt)
    o.rk4(10, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)


@pytest.mark.parametrize("name,spec,tiling", FUSED_HIGH_ORDER, ids=[c[0] for c in FUSED_HIGH_ORDER])
def test_fused_high_order_steps_match_oracle(oracle_mod, name, spec, tiling):
    """20 RK4 steps of a perturbed state in the automatic (fused) form at
    p = 4, 6 and 7 against the oracle."""
    _say(f"[gpu] fused high order, 20 steps: {name}")
    g, o = _pair(oracle_mod, spec, tiling)
    assert g.tiling()["fused"] == 1
    f = workloads.perturbed_state(37, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(20, dt)
    o.rk4(20, dt)
    er, eu = _moment_errors(g, o)
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL and eu < TOL, (er, eu)
    assert _rel(g.get_state(), o.get_state()) < TOL


@pytest.mark.parametrize("tiling", [None, (2, 13), (4, 0), (2, 50), (2, 34), (2, 25)],
                         ids=["fused", "tiles8", "persistent", "tiles2", "tiles3_ragged", "tiles4"])
def test_cavity_perturbed_steps_match_oracle(oracle_mod, tiling):
    """40 steps in each decomposition; with 2 to 4 velocity tiles the stages
    hand their moment partials on (no moments pass after the first stage),
    and the residual then reads f_n's partials too."""
    _say(f"[gpu] cavity 10x7 p3 nc10 perturbed, tiling={tiling}")
    spec = workloads.cavity(n=10, ny=7, p=3, m=10, lid=0.1, kn=0.5)
    g, o = _pair(oracle_mod, spec, tiling)
    f = workloads.perturbed_state(23, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(15, dt)
    o.rk4(15, dt)
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < TOL * r
    g.step(25, dt)
    o.rk4(25, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)
    assert _rel(g.get_state(), o.get_state()) < TOL
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < TOL * r


HANDOFF_CASES = [
    ("cavity_9x7_p3_nc12", workloads.cavity(n=9, ny=7, p=3, m=12, lid=0.1, kn=0.5)),
    ("couette_6x5_p3_gh4", workloads.couette(nx=6, ny=5, p=3, kn=0.7)),
    ("cavity_7x6_p1_nc10", workloads.cavity(n=7, ny=6, p=1, m=10, lid=0.2, kn=1.5)),
    ("box_5x4_p3_gh3", workloads.periodic_box(nx=5, ny=4, p=3, velset=("gh", 3), kn=0.5)),
]


@pytest.mark.parametrize("name,spec", HANDOFF_CASES, ids=[c[0] for c in HANDOFF_CASES])
def test_moment_handoff_steps_match_oracle(oracle_mod, name, spec):
    """One-element fused blocks of orders 1 and 3 take their input's moments
    from the update pass of the stage before (the first stage from a moment
    pass over f_n): steps, a residual between them, and a state set again in
    the middle, against the oracle."""
    _say(f"[gpu] moment handoff: {name}")
    g, o = _pair(oracle_mod, spec)
    g.set_block_elements(1)
    assert g.tiling()["fused"] == 1 and g.tiling()["elems_per_group"] == 1
    f = workloads.perturbed_state(53, o.w, o.K, o.Np, amp=0.05)
    dt = o.stable_dt(0.2)
    for s_ in (g, o):
        s_.set_state(f)
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < TOL * r
    g.step(7, dt)
    o.rk4(7, dt)
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < TOL * r
    g.step(5, dt)
    o.rk4(5, dt)
    assert _rel(g.get_state(), o.get_state()) < TOL
    f2 = workloads.perturbed_state(59, o.w, o.K, o.Np, amp=0.05)
    for s_ in (g, o):
        s_.set_state(f2)
    g.step(9, dt)
    o.rk4(9, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)
    assert _rel(g.get_state(), o.get_state()) < TOL
    r, rc = o.residual()
    assert rc == 0 and abs(g.residual() - r) < TOL * r


def test_moment_handoff_batch_matches_solo():
    """Batch members with one-element blocks hand their moments on in the
    class kernel as they do alone: the states and residuals agree bit for bit,
    across batch steps, solo steps of the same solvers and a graph replay."""
    _say("[gpu] moment handoff in a batch")
    specs = [c[1] for c in HANDOFF_CASES]
    def make():
        out = []
        for i, sp in enumerate(specs):
            g = binding.Solver.from_spec(sp)
            g.set_block_elements(1)
            g.set_state(workloads.perturbed_state(61 + i, g.w, g.K, g.Np, amp=0.05))
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
        assert np.array_equal(x.get_state(), y.get_state()), specs[i].name
        assert rb[i] == y.residual(), specs[i].name
    # solo steps of batch members continue from the batch's partials
    for x, y, dt in zip(bm, solo, dts):
        x.step(3, dt)
        y.step(3, dt)
    b.step(4, dts)
    for g, dt in zip(solo, dts):
        g.step(4, dt)
    for i, (x, y) in enumerate(zip(bm, solo)):
        assert np.array_equal(x.get_state(), y.get_state()), specs[i].name
    b.close()


@pytest.mark.parametrize("name,spec,tiling", [
    ("couette_8x8_p2_gh4", workloads.COUETTE_8x8_P2_D2Q16, None),
    ("cavity_5x3_p4_nc6_tiled", workloads.cavity(n=5, ny=3, p=4, m=6, lid=0.2), (2, 7)),
    ("cavity_9x7_p3_nc9_persistent", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15), (4, 0)),
    ("cavity_6x5_p3_nc10_tiles3", workloads.cavity(n=6, ny=5, p=3, m=10, lid=0.1), (2, 34))],
    ids=["couette_8x8_p2_gh4", "cavity_5x3_p4_nc6_tiled", "cavity_9x7_p3_nc9_persistent",
         "cavity_6x5_p3_nc10_tiles3"])
def test_graph_replayed_steps_identical_to_eager(oracle_mod, name, spec, tiling):
    """dgbgk_set_graph: steps replayed from a captured hipGraph, with step counts
    that are not multiples of the graph length, a change of dt (re-capture) and
    a change of block size (re-capture), bit-identical to ordinary launches and
    within the FP64 bar of the oracle."""
    _say(f"[gpu] graph-replayed steps: {name}")
    a, o = _pair(oracle_mod, spec, tiling)
    b = binding.Solver.from_spec(spec)
    if tiling is not None:
        b.set_tiling(*tiling)
    b.set_graph(7)
    f = workloads.perturbed_state(43, o.w, o.K, o.Np, amp=0.05)
    for g in (a, b):
        g.set_state(f)
    o.set_state(f)
    dt0 = o.stable_dt(0.2)
    total = 0
    for n, dt in ((20, dt0), (3, dt0), (15, 0.5 * dt0), (14, 0.5 * dt0)):
        a.step(n, dt)
        b.step(n, dt)
        o.rk4(n, dt)
        total += n
        assert np.array_equal(a.get_state(), b.get_state()), (n, dt)
        assert b.steps_taken() == total
    er, eu = _moment_errors(b, o)
    assert er < TOL and eu < TOL, (er, eu)
    if tiling is None:
        for g in (a, b):
            g.set_block_elements(1)
        a.step(9, dt0)
        b.step(9, dt0)
        assert np.array_equal(a.get_state(), b.get_state())
    b.set_graph(0)
    a.step(2, dt0)
    b.step(2, dt0)
    assert np.array_equal(a.get_state(), b.get_state())


def test_fused_and_tiled_agree():
    _say("[gpu] fused vs tiled")
    spec = workloads.cavity(n=8, p=3, m=12, lid=0.1)
    a = binding.Solver.from_spec(spec)
    b = binding.Solver.from_spec(spec)
    b.set_tiling(2, 40)
    assert a.tiling()["fused"] and not b.tiling()["fused"]
    for s in (a, b):
        s.init_equilibrium()
        s.step(30, s.stable_dt(0.2))
    assert _rel(b.get_state(), a.get_state()) < 1e-13


@pytest.mark.parametrize("n,ny,p,m", [(8, 8, 3, 16), (9, 7, 3, 9), (5, 3, 2, 4), (3, 5, 1, 8)])
def test_persistent_and_per_block_kernels_identical(n, ny, p, m):
    # the persistent kernel runs the same arithmetic in the same order as the
    # one-block-per-work-group kernel, so the states agree bit for bit
    _say(f"[gpu] persistent vs per-block {n}x{ny} p{p} nc{m}")
    spec = workloads.cavity(n=n, ny=ny, p=p, m=m, lid=0.1)
    a = binding.Solver.from_spec(spec)
    b = binding.Solver.from_spec(spec)
    a.set_tiling(4, 0)
    b.set_block_elements(a.tiling()["elems_per_group"])  # the same blocks: same sums
    assert a.tiling()["persistent"] and b.tiling()["fused"] and not b.tiling()["persistent"]
    f = workloads.perturbed_state(5, a.w, a.K, a.Np, amp=0.05)
    assert np.array_equal(a.rhs(f), b.rhs(f))
    for s_ in (a, b):
        s_.set_state(f)
        s_.step(12, s_.stable_dt(0.2))
    if p in (1, 3) and b.tiling()["elems_per_group"] == 1:
        # one-element blocks of these orders take the moments of their input
        # from the update of the stage before (another summation order)
        assert _rel(a.get_state(), b.get_state()) < 1e-13
    else:
        assert np.array_equal(a.get_state(), b.get_state())


def test_residual_and_moments_parity(oracle_mod):
    _say("[gpu] residual parity")
    spec = workloads.cavity(n=6, p=2, m=8, lid=0.1)
    g, o = _pair(oracle_mod, spec)
    f = workloads.perturbed_state(3, o.w, o.K, o.Np, amp=0.1)
    g.set_state(f)
    o.set_state(f)
    rg = g.residual()
    ro, rc = o.residual()
    assert rc == 0 and abs(rg - ro) < 1e-12 * ro
    er, eu = _moment_errors(g, o)
    assert er < 1e-14 and eu < 1e-14
    # at rest with the lid stopped the state is a fixed point
    g2 = binding.Solver.from_spec(spec.with_(wall_u=((0, 0),) * 4))
    g2.init_equilibrium()
    assert g2.residual() < 1e-12


def _moment_field(g, seed):
    """Seeded smooth density and velocity at every node (shape K, Np)."""
    x, y = g.node_coords()
    r = np.random.default_rng(seed).uniform(0.5, 1.5, size=4)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * r[0] * x) * np.cos(2 * np.pi * r[1] * y)
    ux = 0.1 * np.cos(2 * np.pi * r[2] * y)
    uy = -0.08 * np.sin(2 * np.pi * r[3] * x)
    return rho, ux, uy


@pytest.mark.parametrize("name,spec", [
    ("cavity_6x5_p2_nc8", workloads.cavity(n=6, ny=5, p=2, m=8, lid=0.1)),
    ("couette_7x3_p3_gh6", workloads.couette(nx=7, ny=3, p=3, velset=("gh", 6))),
], ids=lambda v: v if isinstance(v, str) else "")
def test_init_moments_matches_oracle_equilibrium(oracle_mod, name, spec):
    _say(f"[gpu] init_moments {name}")
    g, o = _pair(oracle_mod, spec)
    rho, ux, uy = _moment_field(g, 11)
    g.init_moments(rho, ux, uy)
    f = g.get_state()
    want = np.empty_like(f)
    for k in range(o.K):
        for n in range(o.Np):
            want[:, k, n] = o.equilibrium(rho[k, n], ux[k, n], uy[k, n])
    assert _rel(f, want) < 1e-14
    # the steps from that state follow the oracle's
    o.set_state(want)
    dt = g.stable_dt(0.2)
    g.step(20, dt)
    o.rk4(20, dt)
    er, eu = _moment_errors(g, o)
    _say(f"    rho {er:.2e}  u {eu:.2e}")
    assert er < TOL and eu < TOL


def test_init_moments_uniform_equals_init_equilibrium():
    _say("[gpu] init_moments uniform")
    spec = workloads.cavity(n=5, p=3, m=8, lid=0.1)
    a = binding.Solver.from_spec(spec)
    b = binding.Solver.from_spec(spec)
    shape = (a.K, a.Np)
    a.init_moments(np.full(shape, 1.3), np.full(shape, 0.02), np.full(shape, -0.05))
    b.init_equilibrium(1.3, 0.02, -0.05)
    assert np.array_equal(a.get_state(), b.get_state())


def test_stream_switch_and_device_state_view():
    """Work enqueued on a caller's stream after dgbgk_set_stream gives the
    same state as on the null stream; dgbgk_state_device_ptr is the
    element-major device copy of the state."""
    import torch
    _say("[gpu] set_stream / state_device_ptr")
    spec = workloads.cavity(n=5, ny=4, p=3, m=8, lid=0.1)
    a = binding.Solver.from_spec(spec)
    b = binding.Solver.from_spec(spec)
    dt = a.stable_dt(0.2)
    a.init_equilibrium()
    a.step(15, dt)
    side = torch.cuda.Stream()
    b.set_stream(side.cuda_stream)
    b.init_equilibrium()
    b.step(15, dt)
    b.synchronize()
    fa, fb = a.get_state(), b.get_state()
    b.set_stream(None)  # the side stream may go away before b does
    assert np.array_equal(fa, fb)

    # a switch while steps are still in flight on the old stream: the new
    # stream's work is ordered after them (no host synchronisation between)
    big = workloads.cavity(n=32, p=3, m=16, lid=0.1)
    c = binding.Solver.from_spec(big)
    d = binding.Solver.from_spec(big)
    dtb = c.stable_dt(0.2)
    c.init_equilibrium()
    c.step(50, dtb)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    d.set_stream(s1.cuda_stream)
    d.init_equilibrium()
    d.step(40, dtb)
    d.set_stream(s2.cuda_stream)
    d.step(10, dtb)
    fc, fd = c.get_state(), d.get_state()
    d.set_stream(None)
    assert np.array_equal(fc, fd)
    c.close()
    d.close()

    # copy the device state out with the HIP runtime the process has loaded
    import ctypes
    path = next(ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln)
    hip = ctypes.CDLL(path)
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    dev = np.empty((b.K, b.Q, b.Np))
    assert hip.hipMemcpy(dev.ctypes.data, b.state_device_ptr(), dev.nbytes, 2) == 0  # to host
    assert np.array_equal(dev.transpose(1, 0, 2), fb)


def test_residual_async_and_nonfinite():
    _say("[gpu] residual async / nonfinite")
    import torch
    spec = workloads.cavity(n=4, p=2, m=6)
    g = binding.Solver.from_spec(spec, stream="torch", torch_memory=True)
    g.init_equilibrium()
    g.step(5, g.stable_dt(0.2))
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    g.residual_async(out.data_ptr())
    torch.cuda.current_stream().synchronize()
    assert out.item() == pytest.approx(g.residual(), rel=0, abs=0)
    f = g.get_state()
    f[2, 3, 1] = np.nan
    g.set_state(f)
    with pytest.raises(binding.DgbgkError) as ei:
        g.residual()
    assert ei.value.code == binding.ENONFINITE
    with pytest.raises(binding.DgbgkError) as ei:
        g.moments()
    assert ei.value.code == binding.ENONFINITE


def test_mass_conservation_on_gpu():
    _say("[gpu] mass conservation")
    spec = workloads.cavity(n=8, p=3, m=10, lid=0.1, kn=0.5)
    g = binding.Solver.from_spec(spec)
    M = np.kron(g.operator(5), g.operator(5))  # tensor mass matrix (host table)
    J = (1 / 8) ** 2 / 4
    f = workloads.perturbed_state(8, g.w, g.K, g.Np, amp=0.1)
    g.set_state(f)
    m0 = J * np.einsum("n,kn->", M.sum(axis=0), g.moments()[0])
    g.step(300, g.stable_dt(0.2))
    m1 = J * np.einsum("n,kn->", M.sum(axis=0), g.moments()[0])
    assert abs(m1 - m0) < 2e-14 * m0


def test_determinism_and_checkpoint():
    _say("[gpu] determinism / checkpoint")
    spec = workloads.cavity(n=8, p=3, m=8, lid=0.1)
    dt = None
    outs = []
    for _ in range(2):
        g = binding.Solver.from_spec(spec)
        dt = g.stable_dt(0.2)
        g.init_equilibrium()
        g.step(60, dt)
        outs.append(g.get_state())
    assert np.array_equal(outs[0], outs[1])
    g = binding.Solver.from_spec(spec)
    g.init_equilibrium()
    g.step(30, dt)
    mid = g.get_state()
    h = binding.Solver.from_spec(spec)
    h.set_state(mid)
    h.step(30, dt)
    assert np.array_equal(h.get_state(), outs[0])


def test_errors_on_device():
    _say("[gpu] error paths")
    g = binding.Solver.from_spec(workloads.cavity(n=3, p=1, m=4))
    with pytest.raises(binding.DgbgkError) as ei:
        g.step(1, 1e-3)
    assert ei.value.code == binding.ESTATE
    with pytest.raises(binding.DgbgkError) as ei:
        g.set_state(np.zeros(5))
    assert ei.value.code == binding.EINVAL
    g.init_equilibrium()
    with pytest.raises(binding.DgbgkError) as ei:
        g.step(1, -1.0)
    assert ei.value.code == binding.EINVAL
    # an unstable step diverges and is reported as non-finite, not hidden
    g.step(400, 50 * g.stable_dt(1.0))
    with pytest.raises(binding.DgbgkError) as ei:
        g.residual()
    assert ei.value.code == binding.ENONFINITE


def test_full_size_cavity_64x64_p3_nc16_matches_oracle(oracle_mod):
    """The benchmark workload at full size (16.8 M DOF) in the launch
    configuration the benchmark times: RHS of a perturbed state, and rho, u
    after 2 RK4 steps, element by element against the oracle."""
    _say("[gpu] full-size cavity 64x64 p3 nc16")
    spec = workloads.CAVITY_64x64_P3_NC16
    g, o = _pair(oracle_mod, spec, stream="torch", torch_memory=True)
    assert g.tiling()["fused"]
    f = workloads.perturbed_state(31, o.w, o.K, o.Np, amp=0.05)
    _say("  rhs")
    assert _rel(g.rhs(f), o.rhs(f)) < TOL
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(spec.cfl)
    _say("  2 steps")
    g.step(2, dt)
    o.rk4(2, dt)
    er, eu = _moment_errors(g, o)
    assert er < TOL and eu < TOL, (er, eu)
