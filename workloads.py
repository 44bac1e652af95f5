"""Synthetic workloads: problem definitions and seeded input generators.

This module is shared by the GPU binding's callers and by the CPU oracle's
callers, so it holds no arithmetic of the method: it names problems (mesh,
polynomial order, velocity-set recipe, Knudsen number, walls) and draws
seeded random numbers.  Each side turns a spec into its own velocity set,
relaxation time and operators.

Workloads follow the shapes of the paper's experiments (Sec. III):
  * micro-Couette flow: plates at y=0 and y=1 moving in opposite directions,
    periodic in x, diffuse walls, D2Q16 Gauss-Hermite velocities;
  * lid-driven micro-cavity: lid at y=1, other walls at rest, diffuse walls,
    Newton-Cotes velocity sets on [-4, 4]^2 (in units of sqrt(RT), RT = 1).
"""
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

PERIODIC = 0
DIFFUSE_WALL = 1


@dataclass(frozen=True)
class ProblemSpec:
    name: str
    nx: int
    ny: int
    p: int
    velset: Tuple            # ("gh", n) | ("nc", m, vmax) | ("custom", ex, ey, w, theta)
    kn: float = 1.0
    kn_convention: int = 1   # 0: tau = Kn L/sqrt3 ; 1: with the sqrt(pi/6) factor
    kn_length: float = 1.0
    tau: Optional[float] = None  # overrides kn when given (e.g. float('inf'))
    bc: Tuple[int, int, int, int] = (DIFFUSE_WALL,) * 4   # bottom, right, top, left
    wall_u: Tuple = ((0.0, 0.0),) * 4
    x0: float = 0.0
    y0: float = 0.0
    lx: float = 1.0
    ly: float = 1.0
    cfl: float = 0.2
    steps: int = 100

    def with_(self, **kw):
        return replace(self, **kw)


def couette(nx=8, ny=8, p=2, u_wall=0.1, kn=1.0, velset=("gh", 4), steps=200, **kw):
    """Couette flow on [0,1]^2: periodic in x, plates y=0 (-u_wall) and y=1 (+u_wall)."""
    return ProblemSpec(
        name=f"couette_{nx}x{ny}_p{p}", nx=nx, ny=ny, p=p, velset=velset, kn=kn,
        bc=(DIFFUSE_WALL, PERIODIC, DIFFUSE_WALL, PERIODIC),
        wall_u=((-u_wall, 0.0), (0.0, 0.0), (u_wall, 0.0), (0.0, 0.0)),
        steps=steps, **kw)


def cavity(n=64, p=3, m=16, vmax=4.0, lid=0.1, kn=1.0, steps=100, ny=None, **kw):
    """Lid-driven cavity on [0,1]^2: lid at y=1 moving at (lid, 0), other walls at rest."""
    return ProblemSpec(
        name=f"cavity_{n}x{ny or n}_p{p}_nc{m}", nx=n, ny=ny or n, p=p,
        velset=("nc", m, vmax), kn=kn,
        bc=(DIFFUSE_WALL,) * 4,
        wall_u=((0.0, 0.0), (0.0, 0.0), (lid, 0.0), (0.0, 0.0)),
        steps=steps, **kw)


def periodic_box(nx=4, ny=4, p=2, velset=("gh", 4), kn=1.0, **kw):
    return ProblemSpec(name=f"periodic_{nx}x{ny}_p{p}", nx=nx, ny=ny, p=p, velset=velset,
                       kn=kn, bc=(PERIODIC,) * 4, **kw)


# The three single-instance workloads of the benchmark plan.
COUETTE_8x8_P2_D2Q16 = couette()                                  # FP64, 200 steps
CAVITY_64x64_P3_NC16 = cavity(n=64, p=3, m=16, kn=1.0)           # FP64
CAVITY_128x128_P4_NC24_KN8 = cavity(n=128, p=4, m=24, kn=8.0)    # precision path


def batch_instances(seed=0, n=64, n_range=(16, 96), p_choices=(2, 3, 4), kn_log10=(-1.0, 1.0),
                    m_range=(8, 24), steps=1000):
    """The mixed batch: n seeded problems, each a Couette or a cavity flow
    (equal odds) on an N x N mesh with N uniform in n_range, p uniform in
    p_choices, Kn log-uniform over 10**kn_log10, and the velocity set D2Q16
    Gauss-Hermite or Newton-Cotes M x M with M uniform in m_range (equal odds).
    Draws come from numpy.random.default_rng(seed) in a fixed order per
    problem (flow, N, p, Kn, set kind, M)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        flow = "couette" if rng.integers(2) == 0 else "cavity"
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(p_choices[rng.integers(len(p_choices))])
        kn = float(10.0 ** rng.uniform(*kn_log10))
        gh = rng.integers(2) == 0
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        velset = ("gh", 4) if gh else ("nc", M, 4.0)
        if flow == "couette":
            spec = couette(nx=N, ny=N, p=p, kn=kn, velset=velset, steps=steps)
        else:
            spec = cavity(n=N, p=p, m=M, kn=kn, steps=steps).with_(velset=velset)
        vs = "gh4" if gh else f"nc{M}"
        out.append(spec.with_(name=f"b{i:02d}_{flow}_{N}x{N}_p{p}_{vs}_kn{kn:.3g}"))
    return out


def poisson_arrivals(seed=1, rate=20.0, n=64):
    """Arrival times (seconds) of a Poisson stream of the given rate: the
    cumulative sums of seeded exponential gaps."""
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))


def uniform_noise(seed, shape, lo=-1.0, hi=1.0):
    """Seeded uniform noise on [lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def perturbed_state(seed, w, K, Np, amp=0.05):
    """f[q][k][n] = w_q (1 + amp * U(-1,1)): a seeded, positive, non-equilibrium
    state around the rest state rho = 1, u = 0 (w: the velocity weights)."""
    w = np.asarray(w, dtype=np.float64)
    noise = uniform_noise(seed, (len(w), K, Np))
    return w[:, None, None] * (1.0 + amp * noise)
