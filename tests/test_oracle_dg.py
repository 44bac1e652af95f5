"""Pins of the oracle's semi-discrete DG operator and RK4 marching against what
the method and the mathematics fix: the weak form eq. (10) assembled
independently by quadrature, conservation, fixed points, the RK4 relaxation
polynomial, symmetries, free streaming and the Couette closed form eq. (11)."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads

INF = float("inf")


def _lagrange(r):
    """1-D Lagrange basis on nodes r as numpy poly1d objects (value, derivative)."""
    basis = []
    for i in range(len(r)):
        others = [r[m] for m in range(len(r)) if m != i]
        denom = np.prod([r[i] - rm for rm in others])
        poly = np.poly1d(others, r=True) / denom
        basis.append((poly, poly.deriv()))
    return basis


def _weak_form_rhs(o, f, rho_w=None):
    """M dfdt assembled from eq. (10) with tau = inf: per element, velocity and
    test function phi_n,
        int F . grad(phi_n) dx  -  oint phi_n (e.n) f^up ds,
    with f^up the upwind trace (interior if e.n >= 0, else exterior), using
    Gauss-Legendre quadrature on the physical element.  Independent of the
    oracle's strong-form operators."""
    p, Np, K, Q = o.p, o.Np, o.K, o.Q
    n1 = p + 1
    r = np.array({1: [-1, 1], 2: [-1, 0, 1], 3: [-1, -5 ** -0.5, 5 ** -0.5, 1]}[p], float)
    L = _lagrange(r)
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    hx, hy = o.lx / o.nx, o.ly / o.ny
    J = hx * hy / 4
    nb = o.operator(7).astype(int)
    # 1-D basis values and derivatives at the Gauss points: l[g, i], dl[g, i]
    l1 = np.array([[L[i][0](t) for i in range(n1)] for t in xg])
    dl1 = np.array([[L[i][1](t) for i in range(n1)] for t in xg])
    # volume points (a, b) -> (r = xg[a], s = xg[b]); node n = i + n1 j
    phi = np.einsum("ai,bj->abji", l1, l1).reshape(len(xg), len(xg), Np)
    dphidx = np.einsum("ai,bj->abji", dl1, l1).reshape(len(xg), len(xg), Np) * (2 / hx)
    dphidy = np.einsum("ai,bj->abji", l1, dl1).reshape(len(xg), len(xg), Np) * (2 / hy)
    wv = np.outer(wg, wg) * J
    # face points: bottom (t,-1), right (1,t), top (t,1), left (-1,t)
    lm1 = np.array([L[i][0](-1.0) for i in range(n1)])
    lp1 = np.array([L[i][0](1.0) for i in range(n1)])
    face_phi = [np.einsum("gi,j->gji", l1, lm1).reshape(len(xg), Np),
                np.einsum("i,gj->gji", lp1, l1).reshape(len(xg), Np),
                np.einsum("gi,j->gji", l1, lp1).reshape(len(xg), Np),
                np.einsum("i,gj->gji", lm1, l1).reshape(len(xg), Np)]
    normals = [(0, -1), (1, 0), (0, 1), (-1, 0)]
    sJ = [hx / 2, hy / 2, hx / 2, hy / 2]
    out = np.zeros_like(f)
    for k in range(K):
        for q in range(Q):
            ex, ey = o.ex[q], o.ey[q]
            fg = phi @ f[q, k]                               # f at volume points
            vol = np.einsum("ab,ab,abn->n", wv, fg, ex * dphidx + ey * dphidy)
            surf = np.zeros(Np)
            for fc in range(4):
                en = ex * normals[fc][0] + ey * normals[fc][1]
                if en >= 0:
                    fup = face_phi[fc] @ f[q, k]
                elif nb[k, fc] >= 0:
                    fup = face_phi[(fc + 2) % 4] @ f[q, nb[k, fc]]   # same physical points
                else:
                    vals = rho_w[k, fc] * o.ghost_feq[fc][q]          # interpolant on the face
                    fup = l1 @ vals
                surf += sJ[fc] * en * np.einsum("g,g,gn->n", wg, fup, face_phi[fc])
            out[q, k] = vol - surf
    return out


def _rho_w_from_eq8(o, f):
    """eq. (8) at wall face nodes, written out independently for the test."""
    n1 = o.p + 1
    fmask = [[m for m in range(n1)], [o.p + n1 * m for m in range(n1)],
             [m + n1 * o.p for m in range(n1)], [n1 * m for m in range(n1)]]
    normals = [(0, -1), (1, 0), (0, 1), (-1, 0)]
    nb = o.operator(7).astype(int)
    rho_w = np.zeros((o.K, 4, n1))
    o.ghost_feq = []
    for fc in range(4):
        ub = o._wall_u[fc]
        cn = (o.ex - ub[0]) * normals[fc][0] + (o.ey - ub[1]) * normals[fc][1]
        fe = o.equilibrium(1.0, ub[0], ub[1])
        o.ghost_feq.append(fe)
        den = np.sum(np.abs(cn[cn < 0]) * fe[cn < 0])
        for k in range(o.K):
            if nb[k, fc] >= 0:
                continue
            for m in range(n1):
                num = np.sum(np.abs(cn[cn > 0]) * f[cn > 0, k, fmask[fc][m]])
                rho_w[k, fc, m] = num / den
    return rho_w


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("walls", [False, True])
def test_strong_form_equals_weak_form(oracle_mod, p, walls):
    if walls:
        spec = workloads.cavity(n=2, p=p, m=4, lid=0.3, ny=3).with_(tau=INF)
        spec = spec.with_(wall_u=((0.0, 0.0), (0.0, 0.2), (0.3, 0.0), (0.0, -0.1)))
    else:
        spec = workloads.periodic_box(nx=3, ny=2, p=p, velset=("gh", 3), tau=INF)
    o = oracle_mod.Oracle.from_spec(spec)
    o._wall_u = spec.wall_u
    rng = np.random.default_rng(11 + p)
    f = o.w[:, None, None] * (1 + 0.3 * rng.uniform(-1, 1, size=o.shape))
    rho_w = _rho_w_from_eq8(o, f)
    if walls:
        assert np.allclose(o.wall_density(f)[rho_w > 0], rho_w[rho_w > 0], rtol=1e-14)
    weak = _weak_form_rhs(o, f, rho_w)
    strong = o.rhs(f)
    hx, hy = spec.lx / spec.nx, spec.ly / spec.ny
    Mphys = (hx * hy / 4) * o.operator(2)
    got = np.einsum("nm,qkm->qkn", Mphys, strong)
    assert np.max(np.abs(got - weak)) < 1e-12 * np.max(np.abs(weak))


@pytest.mark.parametrize("velset", [("gh", 4), ("nc", 8, 4.0), ("gh", 3)])
def test_uniform_equilibrium_is_a_fixed_point(oracle_mod, velset):
    spec = workloads.periodic_box(nx=3, ny=4, p=3, velset=velset)
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium(1.2, 0.08, -0.05)
    k = o.rhs()
    assert np.max(np.abs(k)) < 2e-15 * np.max(o.get_state()) * 40


def test_cavity_at_rest_is_a_fixed_point(oracle_mod):
    spec = workloads.cavity(n=3, p=2, m=8, lid=0.0)
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium(1.0, 0.0, 0.0)
    assert np.allclose(o.wall_density()[o.operator(7).astype(int) < 0], 1.0, rtol=1e-14)
    assert np.max(np.abs(o.rhs())) < 1e-13
    r, rc = o.residual()
    assert rc == 0 and r < 1e-12


@pytest.mark.parametrize("velset", [("gh", 4), ("nc", 12, 4.0)])
def test_collision_conserves_and_vanishes_at_equilibrium(oracle_mod, velset):
    spec = workloads.periodic_box(nx=2, ny=2, p=2, velset=velset, kn=0.3)
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(5, o.w, o.K, o.Np, amp=0.2)
    _, _, C = o.rhs_parts(f)
    scale = np.max(np.abs(C))
    assert scale > 1e-3
    assert np.max(np.abs(C.sum(axis=0))) < 1e-14 * scale * o.Q
    assert np.max(np.abs(np.einsum("q,qkn->kn", o.ex, C))) < 1e-14 * scale * o.Q * 4
    assert np.max(np.abs(np.einsum("q,qkn->kn", o.ey, C))) < 1e-14 * scale * o.Q * 4
    # f = f^eq(rho(x), u(x)) node by node -> C = 0
    rng = np.random.default_rng(9)
    feq = np.zeros(o.shape)
    for k in range(o.K):
        for n in range(o.Np):
            feq[:, k, n] = o.equilibrium(1 + 0.1 * rng.uniform(), 0.1 * rng.uniform(-1, 1),
                                         0.1 * rng.uniform(-1, 1))
    _, _, C0 = o.rhs_parts(feq)
    assert np.max(np.abs(C0)) < 1e-14


@pytest.mark.parametrize("velset,kn", [(("gh", 4), 0.5), (("nc", 10, 4.0), 2.0)])
def test_rk4_relaxation_polynomial(oracle_mod, velset, kn):
    """Spatially uniform non-equilibrium on a periodic box: the transport terms
    vanish, rho and u are conserved, and classical RK4 advances the deviation by
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, z = -dt/tau, per step."""
    spec = workloads.periodic_box(nx=2, ny=3, p=2, velset=velset, kn=kn)
    o = oracle_mod.Oracle.from_spec(spec)
    rng = np.random.default_rng(4)
    f0q = o.w * (1 + 0.3 * rng.uniform(-1, 1, size=o.Q))
    f0 = np.broadcast_to(f0q[:, None, None], o.shape).copy()
    o.set_state(f0)
    rho = f0q.sum()
    feq = o.equilibrium(rho, (o.ex * f0q).sum() / rho, (o.ey * f0q).sum() / rho)
    dt = o.stable_dt(0.3)
    n = int(math.ceil(1.5 * o.tau / dt))
    o.rk4(n, dt)
    z = -dt / o.tau
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    want = feq + (f0q - feq) * R ** n
    got = o.get_state()
    assert abs(R ** n) < 0.5
    assert np.max(np.abs(got - want[:, None, None])) < 1e-15 * n


@pytest.mark.parametrize("spec", [
    workloads.cavity(n=4, p=2, m=8, lid=0.1, kn=0.5),
    workloads.periodic_box(nx=4, ny=3, p=3, velset=("gh", 4), kn=0.2),
    workloads.couette(nx=3, ny=4, p=1, kn=2.0),
])
def test_mass_conservation(oracle_mod, spec):
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(2, o.w, o.K, o.Np, amp=0.1)
    o.set_state(f)
    m0 = o.total_mass()
    o.rk4(300, o.stable_dt(0.2))
    assert abs(o.total_mass() - m0) < 2e-14 * m0
    assert np.isfinite(o.get_state()).all()


def _run_couette(oracle_mod, nx, ny, p, u_wall, steps):
    o = oracle_mod.Oracle.from_spec(workloads.couette(nx=nx, ny=ny, p=p, u_wall=u_wall))
    o.init_equilibrium()
    o.rk4(steps, o.stable_dt(0.2))
    return o


def test_couette_invariants(oracle_mod):
    """D2Q16 Couette from rest: rho = 1 and u_y = 0 at every node and step; u_x
    is linear in the wall speed, antisymmetric about mid-channel and
    independent of x (1 x N and N x N meshes agree)."""
    a = _run_couette(oracle_mod, 6, 6, 2, 0.1, 60)
    rho, ux, uy = a.moments()
    assert np.max(np.abs(rho - 1)) < 2e-15 * 10
    assert np.max(np.abs(uy)) < 1e-15 * 10
    assert np.max(np.abs(ux)) > 1e-3
    b = _run_couette(oracle_mod, 6, 6, 2, 0.2, 60)
    assert np.max(np.abs(b.moments()[1] - 2 * ux)) < 1e-14 * 10
    # mirror y -> 1 - y: element row ey -> ny-1-ey, node row j -> p-j
    nx, ny, n1 = 6, 6, 3
    for k in range(a.K):
        kk = k % nx + nx * (ny - 1 - k // nx)
        for n in range(a.Np):
            nn = n % n1 + n1 * (n1 - 1 - n // n1)
            assert abs(ux[kk, nn] + ux[k, n]) < 1e-15 * 20
    c = _run_couette(oracle_mod, 1, 6, 2, 0.1, 60)
    uxc = c.moments()[1]
    for k in range(a.K):
        for n in range(a.Np):
            assert abs(uxc[k // nx, n] - ux[k, n]) < 1e-15 * 20


def test_cavity_mirror_symmetry(oracle_mod):
    """Reflecting x -> L - x maps the cavity with lid speed U onto the cavity
    with lid speed -U: (rho, u_x, u_y)(x) -> (rho, -u_x, u_y)(L - x)."""
    sa = workloads.cavity(n=4, p=2, m=8, lid=0.1, kn=1.0)
    sb = workloads.cavity(n=4, p=2, m=8, lid=-0.1, kn=1.0)
    oa, ob = oracle_mod.Oracle.from_spec(sa), oracle_mod.Oracle.from_spec(sb)
    for o in (oa, ob):
        o.init_equilibrium()
        o.rk4(80, o.stable_dt(0.2))
    ra, uxa, uya = oa.moments()
    rb, uxb, uyb = ob.moments()
    assert np.max(np.abs(uxa)) > 1e-4
    # mirror x -> 1 - x: element column ex -> nx-1-ex, node column i -> p-i
    nx, n1 = 4, 3
    for k in range(oa.K):
        kk = (nx - 1 - k % nx) + nx * (k // nx)
        for n in range(oa.Np):
            nn = (n1 - 1 - n % n1) + n1 * (n // n1)
            assert abs(rb[kk, nn] - ra[k, n]) < 1e-14
            assert abs(uxb[kk, nn] + uxa[k, n]) < 1e-15 * 10
            assert abs(uyb[kk, nn] - uya[k, n]) < 1e-15 * 10


def _free_streaming_error(oracle_mod, n, p, t_end=0.25):
    ex = [1.0, -0.5, 0.3]
    ey = [0.4, 1.0, -0.8]
    spec = workloads.periodic_box(nx=n, ny=n, p=p,
                                  velset=("custom", ex, ey, [1 / 3] * 3, 1.0), tau=INF)
    o = oracle_mod.Oracle.from_spec(spec)
    x, y = o.node_coords()

    def field(xx, yy):
        return 1 + 0.1 * np.sin(2 * np.pi * xx) * np.sin(2 * np.pi * yy)

    o.set_state(np.stack([field(x, y) for _ in range(3)]))
    dt0 = o.stable_dt(0.1)
    steps = int(math.ceil(t_end / dt0))
    o.rk4(steps, t_end / steps)
    f = o.get_state()
    M = (o.lx / n) * (o.ly / n) / 4 * o.operator(2)
    err2 = 0.0
    for q in range(3):
        e = f[q] - field(x - ex[q] * t_end, y - ey[q] * t_end)
        err2 += np.einsum("kn,nm,km->", e, M, e)
    return math.sqrt(err2)


@pytest.mark.slow
@pytest.mark.parametrize("p", [1, 2, 3])
def test_free_streaming_converges_at_p_plus_1(oracle_mod, p):
    """tau = inf on a periodic box: the DG solution approaches the exact
    translate f_q(x - e_q t, 0) in L2 at rate p+1 under h-refinement."""
    ns = [4, 8, 16]
    errs = [_free_streaming_error(oracle_mod, n, p) for n in ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert rates[-1] > p + 1 - 0.3, (errs, rates)


def _couette_bvp_ux(y, tau, L, u_top, u_bot):
    """Steady D2Q16 Couette solved as a linear two-point boundary-value problem
    with a matrix exponential.  The x-momentum carried by each y-speed class,
    g_a = sum_b e_xb f_ab, obeys c_a g_a' = -(g_a - w_a sum g)/tau (rho = 1,
    u_y = 0), with diffuse walls fixing the incoming classes to w_a U_wall."""
    c = np.array([-math.sqrt(3 + math.sqrt(6)), -math.sqrt(3 - math.sqrt(6)),
                  math.sqrt(3 - math.sqrt(6)), math.sqrt(3 + math.sqrt(6))])
    w = np.array([(3 - math.sqrt(6)) / 12, (3 + math.sqrt(6)) / 12,
                  (3 + math.sqrt(6)) / 12, (3 - math.sqrt(6)) / 12])
    A = -(1 / tau) * np.diag(1 / c) @ (np.eye(4) - np.outer(w, np.ones(4)))
    E = scipy.linalg.expm(A * L)
    inc0 = c > 0         # incoming at the bottom plate
    incL = c < 0         # incoming at the top plate
    g0 = np.zeros(4)
    g0[inc0] = w[inc0] * u_bot
    # unknowns: g0 on the outgoing classes at y=0; conditions: (E g0)[incL] = w U_top
    B = E[np.ix_(incL, ~inc0)]
    rhs = w[incL] * u_top - E[np.ix_(incL, inc0)] @ g0[inc0]
    g0[~inc0] = np.linalg.solve(B, rhs)
    return np.array([np.sum(scipy.linalg.expm(A * yy) @ g0) for yy in np.atleast_1d(y)])


@pytest.mark.parametrize("kn", [0.5, 1.0, 1.381976597885, 1.5])
def test_couette_closed_form_matches_bvp(oracle_mod, kn):
    """eq. (11) (with the missing '+' restored and s measured from mid-channel)
    equals the exact steady solution of the D2Q16 Couette problem."""
    tau = kn / math.sqrt(3)
    ys = np.linspace(0, 1, 11)
    bvp = _couette_bvp_ux(ys, tau, 1.0, 0.1, -0.1)
    cf = np.array([oracle_mod.couette_ux(y, 1.0, kn, 0.1, -0.1) for y in ys])
    assert np.max(np.abs(bvp - cf)) < 1e-12
    bvp2 = _couette_bvp_ux(ys, tau, 1.0, 0.16, 0.02)
    cf2 = np.array([oracle_mod.couette_ux(y, 1.0, kn, 0.16, 0.02) for y in ys])
    assert np.max(np.abs(bvp2 - cf2)) < 1e-12


def _couette_steady_error(oracle_mod, ny, p, tol=1e-13, max_t=60.0):
    spec = workloads.couette(nx=1, ny=ny, p=p, kn=1.0)
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium()
    dt = o.stable_dt(0.3)
    chunk = max(1, int(1.0 / dt))
    prev = o.moments()[1].copy()
    t = 0.0
    while t < max_t:
        o.rk4(chunk, dt)
        t += chunk * dt
        ux = o.moments()[1]
        if np.max(np.abs(ux - prev)) < tol:
            break
        prev = ux.copy()
    kn_eff = oracle_mod.couette_kn_eff(o.tau)
    return o.l2_error_couette(kn_eff, 0.1, -0.1)


@pytest.mark.slow
@pytest.mark.parametrize("p", [1, 2, 3])
def test_couette_h_refinement_rate(oracle_mod, p):
    """Sec. III.A: the steady DG Couette solution converges to eq. (11) in L2 at
    rate p+1 (D2Q16, Kn of the benchmark's Couette workload)."""
    nys = {1: [4, 8, 16], 2: [4, 8, 16], 3: [2, 4, 8]}[p]
    errs = [_couette_steady_error(oracle_mod, ny, p) for ny in nys]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > p + 1 - 0.3, (errs, rates)


def test_residual_flags_nonfinite(oracle_mod):
    o = oracle_mod.Oracle.from_spec(workloads.cavity(n=2, p=1, m=4))
    f = workloads.perturbed_state(1, o.w, o.K, o.Np)
    f[3, 1, 2] = np.nan
    o.set_state(f)
    r, rc = o.residual()
    assert rc == -4 and math.isnan(r)
