"""Serving on the GPU: steady-state solves under continuous batching.  Every
request must end below the residual target, and its result must be the same
alone and in the mix (bit for bit: each request's steps and checks depend only
on its own residual history); the memory budget must bound the requests on
the device; the mixed-precision server (FP32 storage, finished in FP64) must
reach the same target; every served result must match the FP64 oracle run
from rest for the same number of RK4 steps (1e-12 for FP64, 1e-5 for FP32
storage finished in FP64 and for the reference form, which runs in FP32 to the
end, its correction folded into its FP64 reference at every check)."""
import sys

import numpy as np
import pytest

import workloads
from paper_2012_13487_amd import binding

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


REQS = workloads.batch_instances(seed=2, n=5, n_range=(5, 8), p_choices=(2, 3),
                                 kn_log10=(0.0, 1.0), m_range=(6, 8))
ARRIVALS = [0.0, 0.003, 0.006, 0.2, 0.21]


def _serve(reqs, arrivals, **kw):
    sv = binding.Server(hbm_budget=kw.pop("hbm_budget", 4 << 30), check_every=50,
                        max_steps=300000, **kw)
    ids = [sv.submit(r, a) for r, a in zip(reqs, arrivals)]
    sv.run(240.0)
    res = [sv.result(i) for i in ids]
    mom = [sv.moments(i) for i in ids]
    st = sv.stats()
    sv.close()
    return res, mom, st


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_ref"])
def test_served_alone_and_in_mix_identical(precision):
    _say(f"[gpu] serving {precision}: mix of {len(REQS)} vs alone")
    res, mom, st = _serve(REQS, ARRIVALS, precision=precision)
    assert st["completed"] == len(REQS) and st["peak_active"] >= 2
    for r in res:
        assert r["status"] == binding.REQ_CONVERGED and r["residual"] < 1e-6
    if precision == "fp32":
        assert st["precision_switches"] >= 1
    for i, req in enumerate(REQS):
        ra, ma, _ = _serve([req], [0.0], precision=precision)
        _say(f"  {req.name}: steps {res[i]['steps']} (fp64 {res[i]['steps_fp64']})")
        assert ra[0]["steps"] == res[i]["steps"]
        for a, b in zip(ma[0], mom[i]):
            assert np.array_equal(a, b)


def test_mixed_precision_reaches_the_fp64_steady_state():
    # both end below residual 1e-6 in FP64 arithmetic, near the same steady state
    _say("[gpu] serving fp32 + fp64 finish vs fp64")
    r64, m64, _ = _serve(REQS, ARRIVALS, precision="fp64")
    r32, m32, _ = _serve(REQS, ARRIVALS, precision="fp32")
    for i in range(len(REQS)):
        rho64, ux64, uy64 = m64[i]
        rho32, ux32, uy32 = m32[i]
        u64 = np.stack([ux64, uy64])
        du = np.max(np.abs(np.stack([ux32, uy32]) - u64)) / np.max(np.abs(u64))
        drho = np.max(np.abs(rho32 - rho64))
        _say(f"  {REQS[i].name}: |du|/|u| {du:.2e}, |drho| {drho:.2e}")
        assert du < 1e-3 and drho < 1e-4


def test_admission_bounded_by_memory():
    _say("[gpu] serving under a memory budget")
    need = max(binding.required_bytes(r.nx, r.ny, r.p, binding.velocity_set(r.velset), 1.0,
                                      r.bc, r.wall_u) for r in REQS)
    budget = 2 * need + 1  # room for two of the largest request, never for all five
    res, mom, st = _serve(REQS, [0.0] * len(REQS), precision="fp64", hbm_budget=budget)
    assert st["peak_bytes"] <= budget and 2 <= st["peak_active"] < len(REQS)
    assert all(r["status"] == binding.REQ_CONVERGED for r in res)
    ref, mref, _ = _serve(REQS, [0.0] * len(REQS), precision="fp64")
    for a, b in zip(mom, mref):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def _oracle_errors(oracle_mod, spec, steps, moments):
    o = oracle_mod.Oracle.from_spec(spec)
    o.init_equilibrium()
    o.rk4(steps, o.stable_dt(0.2))
    ro, uxo, uyo = o.moments()
    rg, uxg, uyg = (m.reshape(ro.shape) for m in moments)
    er = float(np.max(np.abs(rg - ro)) / np.max(np.abs(ro)))
    u_o = np.stack([uxo, uyo])
    eu = float(np.max(np.abs(np.stack([uxg, uyg]) - u_o)) / np.max(np.abs(u_o)))
    return er, eu


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp32_ref", 1e-5)])
def test_served_results_match_oracle(oracle_mod, precision, tol):
    """Each request of the mix, served to residual 1e-6, against the oracle
    run from rest (f = w) for exactly the request's RK4 steps at the same dt."""
    _say(f"[gpu] served {precision} results vs oracle")
    res, mom, _ = _serve(REQS, ARRIVALS, precision=precision)
    for req, r, m in zip(REQS, res, mom):
        assert r["status"] == binding.REQ_CONVERGED
        er, eu = _oracle_errors(oracle_mod, req, r["steps"], m)
        _say(f"  {req.name}: {r['steps']} steps: err rho {er:.2e} u {eu:.2e}")
        assert er < tol and eu < tol, (req.name, er, eu)
