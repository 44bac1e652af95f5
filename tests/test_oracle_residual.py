"""Pins of the oracle's steady-state residual and total mass against what fixes
them independently of the oracle's own code.

The residual (the reading of "residual 1e-6" used here for steadiness; the
paper judges steadiness by state differences, Sec. III.A and III.B) is the
largest rate of change of the conserved moments rho, rho u_x, rho u_y over the
nodes, made dimensionless by L_ref / (rho_ref U_ref) with rho_ref = 1,
L_ref = min(lx, ly) and U_ref the largest wall speed (1 when every wall rests).
The moment rates are taken here from the right-hand side L(f) (itself pinned
against an independent quadrature assembly of eq. (10)); the scale is pinned by
cases where a wrong length or speed would change the value: a domain whose
shorter side is not lx, several walls moving at different speeds, linearity
of Couette flow in the wall speed, and invariance under a change of length
unit.  Total mass is pinned by exact integrals of polynomial densities."""
import math

import numpy as np
import pytest

import workloads

PERIODIC, WALL = workloads.PERIODIC, workloads.DIFFUSE_WALL


def _moment_rates_max(o, f):
    """max over nodes of max(|sum_q L_q|, |sum_q e_qx L_q|, |sum_q e_qy L_q|),
    from the oracle's right-hand side."""
    k = o.rhs(f)
    a = np.abs(k.sum(axis=0))
    bx = np.abs(np.einsum("q,qkn->kn", o.ex, k))
    by = np.abs(np.einsum("q,qkn->kn", o.ey, k))
    return float(max(a.max(), bx.max(), by.max()))


def _residual(o, f):
    o.set_state(f)
    r, rc = o.residual()
    assert rc == 0
    return r


def test_residual_scale_uses_shorter_side_and_fastest_wall(oracle_mod):
    """[0,2] x [0,0.5] box with four diffuse walls moving at 0.1 (bottom),
    -0.25 (right, along y), 0.3 (top) and 0 (left): L_ref = 0.5 (ly, the
    shorter side, not lx), U_ref = 0.3 (the fastest wall, not the first one)."""
    spec = workloads.ProblemSpec(
        name="box_2x0.5", nx=4, ny=2, p=2, velset=("nc", 6, 4.0), kn=0.7,
        bc=(WALL,) * 4, wall_u=((0.1, 0.0), (0.0, -0.25), (0.3, 0.0), (0.0, 0.0)),
        x0=-0.3, y0=0.2, lx=2.0, ly=0.5)
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(11, o.w, o.K, o.Np, amp=0.03)
    want = _moment_rates_max(o, f) * 0.5 / 0.3
    got = _residual(o, f)
    assert abs(got - want) <= 1e-14 * want, (got, want)
    # the alternatives a slip would produce differ by far more than rounding
    for wrong in (_moment_rates_max(o, f) * 2.0 / 0.3, _moment_rates_max(o, f) * 0.5 / 0.1):
        assert abs(got - wrong) > 0.5 * want


def test_residual_scale_without_moving_walls_is_one(oracle_mod):
    """Periodic box (no walls): U_ref = 1, so R = L_ref x (max moment rate);
    [0,0.8] x [0,1.6] gives L_ref = 0.8."""
    spec = workloads.periodic_box(nx=2, ny=3, p=2, velset=("gh", 4), kn=0.5,
                                  lx=0.8, ly=1.6)
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(5, o.w, o.K, o.Np, amp=0.05)
    want = _moment_rates_max(o, f) * 0.8
    assert abs(_residual(o, f) - want) <= 1e-14 * want


def test_residual_of_couette_is_independent_of_wall_speed(oracle_mod):
    """Couette flow from rest with D2Q16 is linear in the wall speed U (the x
    momentum responds linearly and rho, rho u_y stay at rest), so its moment
    rates scale with U and the residual, divided by U_ref = U, does not."""
    rs = []
    for u in (0.05, 0.1, 0.2):
        o = oracle_mod.Oracle.from_spec(workloads.couette(nx=2, ny=4, p=2, u_wall=u))
        o.init_equilibrium()
        dt = o.stable_dt(0.2)
        o.rk4(3, dt)
        r, rc = o.residual()
        assert rc == 0
        rs.append(r)
    assert rs[0] > 1e-3
    assert max(rs) - min(rs) <= 1e-12 * rs[1], rs


def test_residual_is_invariant_under_a_change_of_length_unit(oracle_mod):
    """Stretching the domain by s and the relaxation time by s (the same Knudsen
    number) divides every moment rate by s; L_ref grows by s, so R is the same
    for the same nodal state."""
    base = workloads.cavity(n=3, p=2, m=6, lid=0.1, kn=1.0).with_(ny=2, ly=0.6)
    o1 = oracle_mod.Oracle.from_spec(base.with_(tau=0.9))
    f = workloads.perturbed_state(7, o1.w, o1.K, o1.Np, amp=0.04)
    r1 = _residual(o1, f)
    s = 3.0
    o2 = oracle_mod.Oracle.from_spec(base.with_(tau=0.9 * s, lx=s, ly=0.6 * s, x0=1.0, y0=-2.0))
    r2 = _residual(o2, f)
    assert abs(r2 - r1) <= 1e-13 * r1, (r1, r2)


@pytest.mark.parametrize("x0,y0", [(0.0, 0.0), (-0.4, 0.7)])
def test_total_mass_of_uniform_density(oracle_mod, x0, y0):
    """rho = 1.3 everywhere on a 2 x 3 domain: total mass 1.3 x 6 = 7.8."""
    spec = workloads.periodic_box(nx=3, ny=4, p=2, velset=("nc", 6, 4.0), lx=2.0, ly=3.0,
                                  x0=x0, y0=y0)
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium(1.3, 0.0, 0.0)
    assert abs(o.total_mass() - 7.8) < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_total_mass_of_polynomial_density(oracle_mod, p):
    """rho = 1 + 0.2 x + 0.1 x y^2 on [0,2] x [0,3] (degree <= 2 per
    direction, so the element integrals are exact for p >= 2):
    int rho = 6 + 1.2 + 1.8 = 9."""
    spec = workloads.periodic_box(nx=2, ny=3, p=p, velset=("gh", 4), lx=2.0, ly=3.0)
    o = oracle_mod.Oracle.from_spec(spec)
    x, y = o.node_coords()
    rho = 1.0 + 0.2 * x + 0.1 * x * y ** 2
    o.set_state(o.w[:, None, None] * rho[None, :, :])
    assert abs(o.total_mass() - 9.0) < 1e-13
