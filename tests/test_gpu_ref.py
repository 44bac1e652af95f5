"""GPU parity of the reference form (DGBGK_FP32_REF and its bf16 variant): the
state is an FP64 reference plus an FP32 correction, folded into the reference
from time to time.  Against the FP64 CPU oracle on the same seeded inputs:
the right-hand side L(f) evaluated as a correction to a different reference
state, rho and u after RK4 steps with folds between them, and a steady-state
solve to residual 1e-6; against the GPU FP64 path after 2000 steps of the
precision workload.  Bars: 1e-5 relative in max-norm (the FP32 storage bar),
2e-3 for the bf16 contractions; a fold leaves the state bit for bit."""
import sys

import numpy as np
import pytest

import workloads
from paper_2012_13487_amd import binding

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_BF = 2e-3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _moment_errors(mg, mo):
    (rg, uxg, uyg), (ro, uxo, uyo) = mg, mo
    u_o = np.stack([uxo, uyo])
    return _rel(rg, ro), float(np.max(np.abs(np.stack([uxg, uyg]) - u_o)) / max(np.max(np.abs(u_o)), 1e-300))


CASES = [
    ("couette_8x8_p2_gh4", workloads.couette(nx=8, ny=8, p=2)),
    ("cavity_6x5_p3_nc8", workloads.cavity(n=6, ny=5, p=3, m=8, lid=0.1)),
    ("cavity_5x3_p4_nc5_scalar", workloads.cavity(n=5, ny=3, p=4, m=5, lid=0.2)),  # Q Np odd
    ("periodic_7x3_p1_gh3", workloads.periodic_box(nx=7, ny=3, p=1, velset=("gh", 3), kn=0.3)),
    ("cavity_9x7_p3_nc9", workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15)),
    ("cavity_4x4_p4_nc12", workloads.cavity(n=4, p=4, m=12, lid=0.1, kn=0.5)),
]


@pytest.mark.parametrize("prec,tol", [("fp32_ref", TOL32), ("fp32_bf16mma_ref", TOL_BF)])
@pytest.mark.parametrize("name,spec", CASES, ids=[c[0] for c in CASES])
def test_ref_rhs_parity(oracle_mod, name, spec, prec, tol):
    """L(f_b) evaluated as the correction f_b - f_a to the reference f_a: FP32,
    an independent state f_a (a correction as large as the state's own
    deviation from rest); bf16, f_a within 1% of f_b, as after a fold (the
    bf16 rounding is relative to the correction's variation inside an
    element, which the plain bf16 path meets at the state's full deviation)."""
    _say(f"[gpu] reference-form rhs parity {name} {prec}")
    g = binding.Solver.from_spec(spec, precision=prec)
    o = oracle_mod.Oracle.from_spec(spec)
    fb = workloads.perturbed_state(17, o.w, o.K, o.Np, amp=0.2)
    if prec == "fp32_ref":
        fa = workloads.perturbed_state(3, o.w, o.K, o.Np, amp=0.1)
    else:
        fa = fb * (1.0 + workloads.uniform_noise(3, fb.shape, -0.01, 0.01))
    g.set_state(fa)
    e = _rel(g.rhs(fb), o.rhs(fb))
    _say(f"  err rhs {e:.2e}")
    assert e < tol, (name, e)
    # with the reference equal to the state: g = 0 and L(f) = L(f_r) in FP64, rounded once
    g.set_state(fb)
    e0 = _rel(g.rhs(fb), o.rhs(fb))
    assert e0 < 1e-7, e0


@pytest.mark.parametrize("name,spec", CASES[:2] + CASES[4:], ids=[c[0] for c in CASES[:2] + CASES[4:]])
def test_ref_steps_with_folds_match_oracle(oracle_mod, name, spec):
    _say(f"[gpu] reference-form steps with folds {name}")
    g = binding.Solver.from_spec(spec, precision="fp32_ref")
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(23, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    o.set_state(f)
    dt = o.stable_dt(0.2)
    for n in (10, 15, 15):
        g.step(n, dt)
        before = g.get_state()
        g.fold()
        assert np.array_equal(g.get_state(), before)  # a fold moves g into f_r exactly
    o.rk4(40, dt)
    er, eu = _moment_errors(g.moments(), o.moments())
    es = _rel(g.get_state(), o.get_state())
    _say(f"  err rho {er:.2e} u {eu:.2e} state {es:.2e}")
    assert er < TOL32 and eu < TOL32 and es < TOL32, (er, eu, es)
    assert g.steps_taken() == 40


def test_ref_steady_state_solve_matches_oracle(oracle_mod):
    """A small cavity from rest to residual 1e-6, folding after every check of
    50 steps (as the server does): the reference form reaches the target, and
    its steady state matches the oracle stepped the same number of steps."""
    _say("[gpu] reference-form steady-state solve")
    spec = workloads.cavity(n=6, p=2, m=8, lid=0.1, kn=2.7)
    g = binding.Solver.from_spec(spec, precision="fp32_ref")
    g.init_equilibrium()
    dt = g.stable_dt(0.2)
    steps = 0
    r = g.residual()
    while r >= 1e-6 and steps < 200_000:
        g.step(50, dt)
        steps += 50
        r = g.residual()
        g.fold()
    _say(f"  {steps} steps, residual {r:.3e}")
    assert r < 1e-6
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium()
    o.rk4(steps, dt)
    ro, rc = o.residual()
    assert rc == 0 and ro < 1.5e-6, ro
    er, eu = _moment_errors(g.moments(), o.moments())
    _say(f"  err rho {er:.2e} u {eu:.2e}; oracle residual {ro:.3e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


def test_ref_against_fp64_gpu_after_2000_steps():
    """The precision workload (128x128 quads, p = 4, NC 24x24, Kn = 8) from rest,
    2000 RK4 steps in the reference form (folded every 50 steps) and in FP64:
    rho, u agree to the FP32 bar."""
    _say("[gpu] reference form vs fp64, cavity 128x128 p4 nc24 kn8, 2000 steps")
    spec = workloads.CAVITY_128x128_P4_NC24_KN8
    out = {}
    for prec in ("fp64", "fp32_ref"):
        g = binding.Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
        dt = g.stable_dt(spec.cfl)
        g.init_equilibrium()
        for _ in range(40):
            g.step(50, dt)
            if prec == "fp32_ref":
                g.fold()
        out[prec] = g.moments()
        g.close()
    er, eu = _moment_errors(out["fp32_ref"], out["fp64"])
    _say(f"  err rho {er:.2e} u {eu:.2e}")
    assert er < TOL32 and eu < TOL32, (er, eu)


def test_ref_errors():
    _say("[gpu] reference-form errors")
    spec = workloads.cavity(n=3, p=2, m=6)
    g = binding.Solver.from_spec(spec, precision="fp32_ref")
    f = workloads.perturbed_state(1, g.w, g.K, g.Np)
    with pytest.raises(binding.DgbgkError) as ei:
        g.rhs(f)  # no reference yet
    assert ei.value.code == binding.ESTATE
    with pytest.raises(binding.DgbgkError) as ei:
        g.fold()
    assert ei.value.code == binding.ESTATE
    g.set_state(f)
    with pytest.raises(binding.DgbgkError) as ei:
        g.wall_density(f)
    assert ei.value.code == binding.ENOTSUP
    h = binding.Solver.from_spec(spec, precision="fp32")
    h.set_state(f)
    with pytest.raises(binding.DgbgkError) as ei:
        h.fold()
    assert ei.value.code == binding.ENOTSUP
    with pytest.raises(binding.DgbgkError) as ei:
        binding.Solver.from_spec(workloads.cavity(n=2, p=5, m=4), precision="fp32_ref")
    assert ei.value.code == binding.ENOTSUP
