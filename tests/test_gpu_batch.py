"""Batched execution on the GPU: several problems (mixed meshes, orders,
velocity sets, Kn, walls and precisions) advanced by persistent batched
kernels.  Each member's result must be bit-identical to the same solver
stepped alone (batch invariance), with and without hipGraph replay, and
within its precision's bar of the FP64 oracle (1e-12 FP64, 1e-5 FP32
storage, 2e-3 bf16 contractions); the autotuner must keep results within the
FP64 bar against the oracle."""
import sys

import numpy as np
import pytest

import workloads
from paper_2012_13487_amd import binding

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


MEMBERS = [
    (workloads.couette(nx=6, ny=6, p=2), binding.FP64),
    (workloads.cavity(n=5, ny=4, p=3, m=8, lid=0.1), binding.FP64),
    (workloads.cavity(n=3, ny=3, p=4, m=6, lid=0.2, kn=0.3), binding.FP64),
    (workloads.periodic_box(nx=4, ny=3, p=1, velset=("gh", 3), kn=0.5), binding.FP64),
    (workloads.cavity(n=6, ny=6, p=3, m=10, lid=0.1, kn=2.0), binding.FP32),
    (workloads.couette(nx=5, ny=7, p=2, kn=0.4), binding.FP32),
    (workloads.cavity(n=4, ny=5, p=2, m=5, lid=0.1), binding.FP32),  # Q Np odd: 4-byte accesses
    (workloads.cavity(n=4, ny=4, p=2, m=6, lid=0.1), binding.FP32_BF16MMA),
    # second members of classes: their descriptors sit at index >= 1
    (workloads.cavity(n=3, ny=5, p=3, m=7, lid=0.05, kn=0.7), binding.FP64),
    (workloads.couette(nx=4, ny=4, p=2, kn=2.0), binding.FP64),
    (workloads.cavity(n=5, ny=3, p=3, m=10, lid=0.2), binding.FP32),
    (workloads.cavity(n=3, ny=4, p=4, m=8, lid=0.1, kn=0.6), binding.FP32),
    (workloads.cavity(n=4, ny=3, p=4, m=6, lid=0.15, kn=1.5), binding.FP32_BF16MMA),
    # reference forms (FP64 reference + FP32 correction)
    (workloads.cavity(n=5, ny=4, p=3, m=8, lid=0.1, kn=0.8), binding.FP32_REF),
    (workloads.couette(nx=4, ny=5, p=2, kn=0.6), binding.FP32_BF16MMA_REF),
    (workloads.cavity(n=3, ny=3, p=4, m=6, lid=0.2, kn=0.3), binding.FP32_REF),
]

# bars against the FP64 oracle per precision
TOLS = {binding.FP64: 1e-12, binding.FP32: 1e-5, binding.FP32_BF16MMA: 2e-3,
        binding.FP32_REF: 1e-5, binding.FP32_BF16MMA_REF: 2e-3}


def _make(seed_base=100):
    out = []
    for i, (spec, prec) in enumerate(MEMBERS):
        g = binding.Solver.from_spec(spec, precision=prec)
        g.set_state(workloads.perturbed_state(seed_base + i, g.w, g.K, g.Np, amp=0.05))
        out.append(g)
    return out


def _dts(solvers):
    return np.array([g.stable_dt(0.2) * (1.0 + 0.01 * i) for i, g in enumerate(solvers)])


@pytest.mark.parametrize("graph", [0, 1, 4], ids=["eager", "graph1", "graph4"])
def test_batch_members_match_solo(graph):
    _say(f"[gpu] batch vs solo, graph={graph}")
    members = _make()
    dts = _dts(members)
    b = binding.Batch(members, graph=graph)
    assert b.launches_per_step() >= 4 * 4  # at least FP64 p=1..4 classes
    b.step(15, dts)
    solo = _make()
    for g, dt in zip(solo, dts):
        g.step(15, dt)
    for i, (gb, gs) in enumerate(zip(members, solo)):
        assert gb.steps_taken() == 15
        assert np.array_equal(gb.get_state(), gs.get_state()), MEMBERS[i][0].name
    b.close()


def test_batch_members_match_oracle(oracle_mod):
    """Every member of the mixed batch (FP64, FP32 and bf16 members, fused p = 4
    members among them) after 15 hipGraph-replayed batched RK4 steps, against
    the oracle stepped from the same state with the member's own dt."""
    _say("[gpu] batch vs oracle")
    members = _make()
    dts = _dts(members)
    for (spec, prec), g in zip(MEMBERS, members):
        if spec.p == 4:
            assert g.tiling()["fused"] == 1, spec.name
    b = binding.Batch(members, graph=True)
    b.step(15, dts)
    for i, ((spec, prec), g) in enumerate(zip(MEMBERS, members)):
        o = oracle_mod.Oracle.from_spec(spec)
        o.set_state(workloads.perturbed_state(100 + i, o.w, o.K, o.Np, amp=0.05))
        o.rk4(15, dts[i])
        ro, uxo, uyo = o.moments()
        rg, uxg, uyg = g.moments()
        er = float(np.max(np.abs(rg - ro)) / np.max(np.abs(ro)))
        u_o = np.stack([uxo, uyo])
        eu = float(np.max(np.abs(np.stack([uxg, uyg]) - u_o)) / np.max(np.abs(u_o)))
        _say(f"  {spec.name} prec {prec}: err rho {er:.2e} u {eu:.2e}")
        assert er < TOLS[prec] and eu < TOLS[prec], (spec.name, prec, er, eu)
    b.close()


def test_graph_replays_with_eager_work_between():
    # replays interleaved with residual evaluations, synchronisations and a
    # change of dt (the descriptor tables are rewritten, the graph is kept)
    _say("[gpu] graph replays")
    ref = _make()
    dts = _dts(ref)
    be = binding.Batch(ref, graph=False)
    gr = _make()
    bg = binding.Batch(gr, graph=3)  # chunks of 3, 4, 2 and 5 steps: full graphs and remainders
    for chunk, scale in ((3, 1.0), (4, 1.0), (2, 0.5), (5, 0.5)):
        be.step(chunk, dts * scale)
        bg.step(chunk, dts * scale)
        re = be.residuals()
        rg = bg.residuals()
        assert np.array_equal(re, rg)
        for a, c in zip(ref, gr):
            assert np.array_equal(a.get_state(), c.get_state())
    be.close()
    bg.close()


def test_batch_residuals_match_solvers():
    _say("[gpu] batch residuals")
    members = _make()
    b = binding.Batch(members)
    b.step(3, _dts(members))
    r = b.residuals()
    for g, rb in zip(members, r):
        assert rb == g.residual()
    b.close()


def test_batch_rejects_unfit_member_and_needs_state():
    _say("[gpu] batch errors")
    big = binding.Solver.from_spec(workloads.cavity(n=2, p=8, m=24))  # fused tile > 160 KB
    with pytest.raises(binding.DgbgkError) as ei:
        binding.Batch([big])
    assert ei.value.code == binding.ENOTSUP
    g = binding.Solver.from_spec(workloads.cavity(n=3, p=2, m=4))
    b = binding.Batch([g])
    with pytest.raises(binding.DgbgkError) as ei:
        b.step(1, [1e-3])
    assert ei.value.code == binding.ESTATE
    g.init_equilibrium()
    with pytest.raises(binding.DgbgkError) as ei:
        b.step(1, [-1.0])
    assert ei.value.code == binding.EINVAL
    b.step(2, [g.stable_dt(0.2)])
    assert g.steps_taken() == 2
    # re-tiling a member after the batch was built is refused
    e0 = g.tiling()["elems_per_group"]
    g.set_block_elements(1 if e0 != 1 else 2)
    with pytest.raises(binding.DgbgkError) as ei:
        b.step(1, [g.stable_dt(0.2)])
    assert ei.value.code == binding.ESTATE
    assert g.steps_taken() == 2
    b.close()


def test_autotune_keeps_parity(oracle_mod):
    _say("[gpu] autotune")
    spec = workloads.cavity(n=9, ny=7, p=3, m=9, lid=0.15)
    g = binding.Solver.from_spec(spec)
    o = oracle_mod.Oracle.from_spec(spec)
    f = workloads.perturbed_state(7, o.w, o.K, o.Np, amp=0.05)
    g.set_state(f)
    us = g.autotune(3)
    assert us > 0.0
    t = g.tiling()
    assert t["lds_bytes"] <= 160 * 1024 and t["elems_per_group"] >= 1
    assert np.array_equal(g.get_state(), f)  # timing leaves the state alone
    o.set_state(f)
    dt = o.stable_dt(0.2)
    g.step(20, dt)
    o.rk4(20, dt)
    rg, ro = g.moments()[0], o.moments()[0]
    assert np.max(np.abs(rg - ro)) / np.max(np.abs(ro)) < 1e-12
    # an explicit block size
    g.set_block_elements(1)
    assert g.tiling()["elems_per_group"] == 1
    with pytest.raises(binding.DgbgkError):
        g.set_block_elements(3)  # not a power of two


def test_full_mixed_batch_sampled_members(oracle_mod):
    """The 64-problem mixed batch (seed 0) at full size in FP64, stepped twice
    as the benchmark times it (four lanes, graph replay); three sampled members
    against solo runs (bit for bit) and against the oracle (1e-12)."""
    _say("[gpu] full mixed batch, 64 problems")
    specs = workloads.batch_instances(seed=0, n=64)
    members = [binding.Solver.from_spec(s, stream="torch") for s in specs]
    for g in members:
        g.init_equilibrium()
    dts = np.array([g.stable_dt(s.cfl) for g, s in zip(members, specs)])
    b = binding.Batch(members, stream="torch", graph=True)
    b.step(2, dts)
    for i in (0, 21, 63):
        _say(f"  member {i}: {specs[i].name}")
        g = binding.Solver.from_spec(specs[i], stream="torch")
        g.set_tiling(1)  # batch members run the fused per-block form
        assert g.tiling()["elems_per_group"] == members[i].tiling()["elems_per_group"]
        g.init_equilibrium()
        g.step(2, dts[i])
        assert np.array_equal(g.get_state(), members[i].get_state())
        g.close()
        o = oracle_mod.Oracle.from_spec(specs[i])
        o.init_equilibrium()
        o.rk4(2, dts[i])
        ro, uxo, uyo = o.moments()
        rg, uxg, uyg = members[i].moments()
        er = float(np.max(np.abs(rg - ro)) / np.max(np.abs(ro)))
        u_o = np.stack([uxo, uyo])
        eu = float(np.max(np.abs(np.stack([uxg, uyg]) - u_o)) / np.max(np.abs(u_o)))
        _say(f"    vs oracle: err rho {er:.2e} u {eu:.2e}")
        assert er < 1e-12 and eu < 1e-12, (er, eu)
        del o
    b.close()
    for g in members:
        g.close()
