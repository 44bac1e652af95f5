"""Pins of the oracle's reference element (Sec. II.B: nodal Lagrange basis of
degree p per direction on Gauss-Lobatto-Legendre points) against closed forms
and exact polynomial calculus."""
import math

import numpy as np
import pytest

import workloads

GLL_CLOSED = {
    1: [-1.0, 1.0],
    2: [-1.0, 0.0, 1.0],
    3: [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0],
    4: [-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
}


def _poly_int(k):
    """Integral of r^k over [-1, 1]."""
    return 0.0 if k % 2 else 2.0 / (k + 1)


def _element(oracle_mod, p):
    return oracle_mod.Oracle(1, 1, p, ("gh", 2), 1.0, (0,) * 4, ((0, 0),) * 4)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_forms(oracle_mod, p):
    assert np.allclose(oracle_mod.gll_nodes(p), GLL_CLOSED[p], rtol=0, atol=2e-16)


@pytest.mark.parametrize("p", [5, 6, 8])
def test_gll_are_lobatto_points(oracle_mod, p):
    """Interior nodes are the roots of P_p' (numpy's Legendre algebra)."""
    r = oracle_mod.gll_nodes(p)
    dP = np.polynomial.legendre.Legendre.basis(p).deriv()
    assert np.max(np.abs(dP(r[1:-1]))) < 1e-12 * p * p
    assert r[0] == -1.0 and r[-1] == 1.0 and np.all(np.diff(r) > 0)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_derivative_matrices_exact_on_polynomials(oracle_mod, p):
    o = _element(oracle_mod, p)
    Dr, Ds = o.operator(0), o.operator(1)
    r = o.operator(4)
    R, S = np.meshgrid(r, r, indexing="xy")  # node n = i + (p+1) j -> R.flat[n] = r_i
    R, S = R.reshape(-1), S.reshape(-1)
    for a in range(p + 1):
        for b in range(p + 1):
            u = R ** a * S ** b
            du_r = a * R ** max(a - 1, 0) * S ** b if a else 0 * u
            du_s = b * R ** a * S ** max(b - 1, 0) if b else 0 * u
            assert np.allclose(Dr @ u, du_r, atol=1e-12 * (p + 1) ** 2)
            assert np.allclose(Ds @ u, du_s, atol=1e-12 * (p + 1) ** 2)
    assert np.allclose(Dr @ np.ones_like(R), 0, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_mass_matrix_is_exact_l2(oracle_mod, p):
    """u^T M v = integral of u v over the reference square for all u, v in Q_p
    (exact mass matrix, not the lumped Gauss-Lobatto one)."""
    o = _element(oracle_mod, p)
    M = o.operator(2)
    r = o.operator(4)
    R, S = [a.reshape(-1) for a in np.meshgrid(r, r, indexing="xy")]
    assert abs(np.ones(len(R)) @ M @ np.ones(len(R)) - 4.0) < 1e-13
    for (a, b, c, d) in [(p, p, p, p), (p, 0, 0, p), (1, p, p - 1, 0), (0, 0, p, p)]:
        u = R ** a * S ** b
        v = R ** c * S ** d
        exact = _poly_int(a + c) * _poly_int(b + d)
        assert abs(u @ M @ v - exact) < 1e-13
    M1 = o.operator(5)
    assert abs(np.ones(p + 1) @ M1 @ np.ones(p + 1) - 2.0) < 1e-14
    if p >= 1:
        lumped = np.zeros(p + 1)
        assert not np.allclose(M1, np.diag(np.diag(M1)) + lumped)  # not diagonal


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lift_reproduces_face_integrals(oracle_mod, p):
    """u^T M LIFT g = sum over faces of the face integral of u g (reference face
    length 2), for u in Q_p and face data g of degree <= p; and the face
    columns of 1^T M LIFT are the face quadrature weights (conservation)."""
    o = _element(oracle_mod, p)
    M, LIFT = o.operator(2), o.operator(3)
    r = o.operator(4)
    n1 = p + 1
    R, S = [a.reshape(-1) for a in np.meshgrid(r, r, indexing="xy")]
    # face parametrisation: bottom (t, -1), right (1, t), top (t, 1), left (-1, t)
    face_pts = [(lambda t: (t, -1.0)), (lambda t: (1.0, t)), (lambda t: (t, 1.0)),
                (lambda t: (-1.0, t))]
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    rng = np.random.default_rng(3)
    for _ in range(3):
        cu = rng.normal(size=(n1, n1))      # u = sum cu[a,b] r^a s^b
        u_nodes = sum(cu[a, b] * R ** a * S ** b for a in range(n1) for b in range(n1))
        g = np.zeros(4 * n1)
        exact = 0.0
        for fc in range(4):
            cg = rng.normal(size=n1)        # g(t) = sum cg[m] t^m
            g[fc * n1:(fc + 1) * n1] = [sum(cg[m] * r[i] ** m for m in range(n1)) for i in range(n1)]
            for t, wt in zip(xg, wg):
                rr, ss = face_pts[fc](t)
                uval = sum(cu[a, b] * rr ** a * ss ** b for a in range(n1) for b in range(n1))
                gval = sum(cg[m] * t ** m for m in range(n1))
                exact += wt * uval * gval
        assert abs(u_nodes @ M @ LIFT @ g - exact) < 1e-12 * max(1.0, abs(exact))
    ones_M_lift = np.ones(n1 * n1) @ M @ LIFT
    face_w = [np.sum(wg * np.array([np.prod([(t - r[m]) / (r[i] - r[m]) for m in range(n1) if m != i])
                                    for t in xg])) for i in range(n1)]
    for fc in range(4):
        assert np.allclose(ones_M_lift[fc * n1:(fc + 1) * n1], face_w, atol=1e-14)


def test_mesh_geometry_and_neighbours(oracle_mod):
    spec = workloads.couette(nx=4, ny=3, p=2)
    o = oracle_mod.Oracle.from_spec(spec)
    nb = o.operator(7).astype(int)
    x, y = o.node_coords()
    hx, hy = 1 / 4, 1 / 3
    assert np.allclose(o.operator(6), [2 / hy, 2 / hx, 2 / hy, 2 / hx])
    for k in range(o.K):
        exx, ey = k % 4, k // 4
        assert np.isclose(x[k].min(), exx * hx) and np.isclose(x[k].max(), (exx + 1) * hx)
        assert np.isclose(y[k].min(), ey * hy) and np.isclose(y[k].max(), (ey + 1) * hy)
        assert nb[k, 1] == (exx + 1) % 4 + 4 * ey and nb[k, 3] == (exx - 1) % 4 + 4 * ey
        assert nb[k, 0] == (k - 4 if ey > 0 else -1)
        assert nb[k, 2] == (k + 4 if ey < 2 else -1)


def test_stable_dt_formula(oracle_mod):
    """The explicit step of the workloads: CFL (h/2) min GLL spacing / max(|ex|+|ey|)."""
    o = oracle_mod.Oracle.from_spec(workloads.COUETTE_8x8_P2_D2Q16)
    vmax = 2 * math.sqrt(3 + math.sqrt(6))
    assert abs(o.stable_dt(0.2) - 0.2 * (1 / 16) * 1.0 / vmax) < 1e-17
    assert abs(o.stable_dt(0.2) - 2.6773e-3) < 1e-7
