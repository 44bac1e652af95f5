"""Implicit SDIRK time steps on the CPU oracle's right-hand side.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The paper marches eq. (10) in time with singly diagonally implicit Runge-Kutta
schemes, Newton's method on the nonlinear system of each stage and GMRES for
each linear system (Sec. II.B, "Time marching").  This module restates that
in the plainest form that can be checked by eye: for each stage

    y_i = f_n + dt sum_{j<i} a_ij L(y_j) + dt a_ii L(y_i),

Newton's method on G(y) = y - b_i - dt a_ii L(y), with the Jacobian of L
formed densely, one column per state value, by central differences of the
oracle's own L, and each linear system solved by LU (numpy.linalg.solve) in
place of GMRES.  A dense Jacobian limits this to small problems (a few
thousand unknowns); that is all the tests ask of it.  With a stiffly accurate
tableau f_{n+1} is the last stage value; the general update
f_n + dt sum_i b_i L(y_i) is used otherwise.

The tableaus are typed here from their sources, independently of the GPU
library: backward Euler; Alexander's two-stage L-stable scheme
(gamma = 1 - 1/sqrt(2)); the five-stage fourth-order L-stable scheme of
Hairer and Wanner (Solving ODEs II, Sec. IV.6, gamma = 1/4).  The paper's
fourth-order study names a four-stage scheme without giving its
coefficients; the five-stage one stands in for it.
"""
import math

import numpy as np


def tableau(scheme):
    """(A, b, c) of a scheme as float arrays."""
    if scheme == "backward_euler":
        A = np.array([[1.0]])
    elif scheme == "sdirk2":
        g = 1.0 - 1.0 / math.sqrt(2.0)
        A = np.array([[g, 0.0],
                      [1.0 - g, g]])
    elif scheme == "sdirk4":
        A = np.array([
            [1 / 4, 0, 0, 0, 0],
            [1 / 2, 1 / 4, 0, 0, 0],
            [17 / 50, -1 / 25, 1 / 4, 0, 0],
            [371 / 1360, -137 / 2720, 15 / 544, 1 / 4, 0],
            [25 / 24, -49 / 48, 125 / 16, -85 / 12, 1 / 4],
        ])
    else:
        raise ValueError(f"unknown scheme {scheme!r}")
    b = A[-1].copy()
    c = A.sum(axis=1)
    return A, b, c


def jacobian(orc, y, delta=1e-7):
    """Dense d L / d f at y by central differences, columns in flat state order."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    n = y.size
    J = np.empty((n, n))
    for j in range(n):
        yp = y.copy()
        ym = y.copy()
        yp[j] += delta
        ym[j] -= delta
        J[:, j] = (orc.rhs(yp).reshape(-1) - orc.rhs(ym).reshape(-1)) / (2.0 * delta)
    return J


def solve_stage(orc, rhs_const, h, y0, max_iter=30, tol=1e-15):
    """Newton's method for y - rhs_const - h L(y) = 0 from y0.

    Returns (y, iterations, final residual max-norm).  Stops when the update is
    below tol times max|y| (or after max_iter iterations)."""
    y = np.array(y0, dtype=np.float64).reshape(-1)
    b = np.asarray(rhs_const, dtype=np.float64).reshape(-1)
    n = y.size
    it = 0
    for it in range(1, max_iter + 1):
        G = y - b - h * orc.rhs(y).reshape(-1)
        M = np.eye(n) - h * jacobian(orc, y)
        d = np.linalg.solve(M, -G)
        y = y + d
        if np.max(np.abs(d)) <= tol * max(np.max(np.abs(y)), 1e-300):
            break
    G = y - b - h * orc.rhs(y).reshape(-1)
    return y, it, float(np.max(np.abs(G)))


def implicit_step(orc, scheme, nsteps, dt, f0=None):
    """nsteps steps of the scheme from f0 (default: the oracle's state).

    Returns the new state (shape (Q, K, Np)) and sets it as the oracle's state."""
    A, b, _ = tableau(scheme)
    s = A.shape[0]
    f = (orc.get_state() if f0 is None else np.asarray(f0, dtype=np.float64)).reshape(-1).copy()
    stiffly_accurate = np.array_equal(A[-1], b)
    for _ in range(nsteps):
        k = []
        y = f.copy()
        for i in range(s):
            const = f.copy()
            for j in range(i):
                const += dt * A[i, j] * k[j]
            y, _, _ = solve_stage(orc, const, dt * A[i, i], y)
            k.append(orc.rhs(y).reshape(-1))
        if stiffly_accurate:
            f = y
        else:
            f = f + dt * sum(b[i] * k[i] for i in range(s))
    orc.set_state(f)
    return f.reshape(orc.shape)


def stability_function(A, b, z):
    """R(z) = 1 + z b^T (I - z A)^{-1} 1 of a Runge-Kutta tableau."""
    s = A.shape[0]
    one = np.ones(s)
    return 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * A, one)
