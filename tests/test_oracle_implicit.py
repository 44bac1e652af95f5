"""Pins of the oracle's implicit SDIRK steps (Sec. II.B, "Time marching")
against what the mathematics fixes: the Runge-Kutta order conditions and
stability of each tableau, the closed-form solution of a spatially uniform
BGK relaxation (backward Euler exactly, every scheme at its order of
convergence, and the L-stable limit dt/tau -> infinity), conservation of
mass, fixed points, and agreement with the explicit RK4 oracle to the local
truncation order on a non-uniform state."""
import math

import numpy as np
import pytest

import workloads
from oracle import implicit

ORDER = {"backward_euler": 1, "sdirk2": 2, "sdirk4": 4}

# order conditions (rooted trees up to order 4) as functions of (A, b, c)
CONDITIONS = {
    1: [(lambda A, b, c: b.sum(), 1.0)],
    2: [(lambda A, b, c: b @ c, 1 / 2)],
    3: [(lambda A, b, c: b @ c ** 2, 1 / 3), (lambda A, b, c: b @ A @ c, 1 / 6)],
    4: [(lambda A, b, c: b @ c ** 3, 1 / 4), (lambda A, b, c: (b * c) @ A @ c, 1 / 8),
        (lambda A, b, c: b @ A @ c ** 2, 1 / 12), (lambda A, b, c: b @ A @ A @ c, 1 / 24)],
}


@pytest.mark.parametrize("scheme", list(ORDER))
def test_tableau_order_conditions(scheme):
    A, b, c = implicit.tableau(scheme)
    p = ORDER[scheme]
    for q in range(1, p + 1):
        for f, want in CONDITIONS[q]:
            assert f(A, b, c) == pytest.approx(want, abs=1e-14), (scheme, q)
    # not of higher order than claimed (first condition of order p + 1)
    if p < 4:
        assert not all(abs(f(A, b, c) - want) < 1e-12 for f, want in CONDITIONS[p + 1])
    # singly diagonally implicit, stiffly accurate
    assert np.allclose(np.diag(A), A[0, 0]) and np.allclose(np.triu(A, 1), 0.0)
    assert np.array_equal(A[-1], b)


def test_sdirk4_nodes_match_the_published_abscissae():
    # the abscissae are printed alongside the coefficients (Hairer and Wanner,
    # Sec. IV.6); they must be the row sums of the typed A
    _, _, c = implicit.tableau("sdirk4")
    assert np.allclose(c, [1 / 4, 3 / 4, 11 / 20, 1 / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("scheme", list(ORDER))
def test_stability_function(scheme):
    A, b, _ = implicit.tableau(scheme)
    p = ORDER[scheme]
    # L-stable: R(z) -> 0 as z -> -infinity
    assert abs(implicit.stability_function(A, b, -1e9)) < 1e-8
    # A-stable on the imaginary axis
    for y in np.linspace(-50, 50, 201):
        assert abs(implicit.stability_function(A, b, 1j * y)) <= 1 + 1e-12
    # R(z) = e^z + O(z^(p+1))
    e1 = abs(implicit.stability_function(A, b, -0.01) - math.exp(-0.01))
    e2 = abs(implicit.stability_function(A, b, -0.005) - math.exp(-0.005))
    assert math.log2(e1 / e2) == pytest.approx(p + 1, abs=0.2)


def _uniform_relaxation(oracle_mod, seed=3):
    """Periodic box with a spatially uniform, non-equilibrium state: the
    transport term vanishes and BGK relaxes f to the fixed f^eq of its
    conserved moments, df/dt = (f^eq - f) / tau."""
    spec = workloads.periodic_box(nx=2, ny=2, p=1, velset=("gh", 4), kn=0.5)
    o = oracle_mod.Oracle.from_spec(spec)
    rng = np.random.default_rng(seed)
    fq = o.w * (1.0 + 0.2 * rng.uniform(-1, 1, size=o.Q))
    f0 = np.broadcast_to(fq[:, None, None], o.shape).copy()
    rho = fq.sum()
    ux, uy = (fq * o.ex).sum() / rho, (fq * o.ey).sum() / rho
    feq = o.equilibrium(rho, ux, uy)
    return o, f0, np.broadcast_to(feq[:, None, None], o.shape)


def test_backward_euler_uniform_relaxation_closed_form(oracle_mod):
    o, f0, feq = _uniform_relaxation(oracle_mod)
    for ratio in (0.3, 4.0, 250.0):
        dt = ratio * o.tau
        f1 = implicit.implicit_step(o, "backward_euler", 1, dt, f0)
        want = feq + (f0 - feq) / (1.0 + ratio)
        # the rounding noise of the transport of a constant state (~1e-16)
        # enters the stage equation multiplied by dt
        assert np.max(np.abs(f1 - want)) < 1e-15 * (1.0 + ratio), ratio


@pytest.mark.parametrize("scheme", list(ORDER))
def test_uniform_relaxation_converges_at_scheme_order(oracle_mod, scheme):
    o, f0, feq = _uniform_relaxation(oracle_mod, seed=4)
    T = o.tau
    exact = feq + math.exp(-T / o.tau) * (f0 - feq)
    errs = []
    for n in (4, 8):
        f = implicit.implicit_step(o, scheme, n, T / n, f0)
        errs.append(np.max(np.abs(f - exact)))
    rate = math.log2(errs[0] / errs[1])
    assert ORDER[scheme] - 0.3 < rate < ORDER[scheme] + 0.6, (errs, rate)


@pytest.mark.parametrize("scheme", list(ORDER))
def test_uniform_relaxation_follows_the_stability_function(oracle_mod, scheme):
    # a linear ODE y' = lambda y is advanced by R(lambda dt); with the tableau
    # L-stable, a step of dt / tau = 1e4 lands within R(-1e4) = O(1e-4) of f^eq
    o, f0, feq = _uniform_relaxation(oracle_mod, seed=5)
    A, b, _ = implicit.tableau(scheme)
    for ratio in (0.5, 20.0, 1e4):
        f1 = implicit.implicit_step(o, scheme, 1, ratio * o.tau, f0)
        R = implicit.stability_function(A, b, -ratio)
        assert np.max(np.abs(f1 - (feq + R * (f0 - feq)))) < 2e-15 * (1.0 + ratio), ratio
    assert np.max(np.abs(f1 - feq)) < 1e-3 * np.max(np.abs(f0 - feq))


def test_equilibrium_at_rest_is_a_fixed_point(oracle_mod):
    o = oracle_mod.Oracle.from_spec(workloads.cavity(n=2, p=1, m=4, lid=0.0))
    o.init_equilibrium(1.0, 0.0, 0.0)
    f0 = o.get_state()
    f1 = implicit.implicit_step(o, "sdirk2", 1, 50 * o.stable_dt(0.2))
    assert np.max(np.abs(f1 - f0)) < 1e-15


@pytest.mark.parametrize("spec", [
    workloads.cavity(n=2, p=1, m=4, lid=0.2, kn=0.5),
    workloads.couette(nx=2, ny=2, p=2, kn=2.0, velset=("gh", 3)),
])
def test_implicit_steps_conserve_mass(oracle_mod, spec):
    o = oracle_mod.Oracle.from_spec(spec)
    o.set_state(workloads.perturbed_state(7, o.w, o.K, o.Np, amp=0.1))
    m0 = o.total_mass()
    implicit.implicit_step(o, "sdirk2", 2, 20 * o.stable_dt(0.2))
    assert abs(o.total_mass() - m0) < 1e-13 * m0


def test_newton_stage_residual_vanishes(oracle_mod):
    o = oracle_mod.Oracle.from_spec(workloads.cavity(n=2, p=1, m=4, lid=0.2, kn=0.5))
    f = workloads.perturbed_state(8, o.w, o.K, o.Np, amp=0.1).reshape(-1)
    h = 30 * o.stable_dt(0.2)
    y, iters, res = implicit.solve_stage(o, f, h, f)
    assert iters >= 2 and res < 1e-15
    assert np.max(np.abs(y - f - h * o.rhs(y).reshape(-1))) < 1e-15


@pytest.mark.parametrize("scheme", list(ORDER))
def test_agrees_with_explicit_rk4_to_local_order(oracle_mod, scheme):
    """One step from a non-uniform state with walls: the implicit and the
    explicit RK4 steps differ by the implicit scheme's local error
    O(dt^(p+1)), so halving dt divides the difference by about 2^(p+1)."""
    spec = workloads.cavity(n=2, p=1, m=4, lid=0.2, kn=0.5)
    o = oracle_mod.Oracle.from_spec(spec)
    f0 = workloads.perturbed_state(9, o.w, o.K, o.Np, amp=0.1)
    dt0 = 0.5 * o.stable_dt(0.2)
    diffs = []
    for dt in (dt0, dt0 / 2):
        fi = implicit.implicit_step(o, scheme, 1, dt, f0)
        o.set_state(f0)
        o.rk4(1, dt)
        diffs.append(np.max(np.abs(fi - o.get_state())))
    rate = math.log2(diffs[0] / diffs[1])
    assert ORDER[scheme] + 1 - 0.4 < rate < ORDER[scheme] + 1 + 0.8, (diffs, rate)
