"""Benchmark: DG-BGK DOF-updates/s on one MI355X.

Workload: lid-driven cavity on [0,1]^2, 64 x 64 quadrilaterals, p = 3 (16 GLL
nodes per element), Newton-Cotes 16 x 16 velocities on [-4,4]^2, Kn = 1,
lid speed 0.1, diffuse walls, FP64, explicit RK4 at CFL 0.2 -- 16.8 M
degrees of freedom (nodes x velocities).  One step = one RK4 step (four
fused stage kernels); the steady-state residual is evaluated on the device
inside the timed region after every 50 steps (--resid-every), so a run of
fewer steps evaluates none.  Before the W warm-up steps the solver steps for
--settle-s seconds untimed: the GPU's clocks ramp for about 40 steps after an
idle period (stage launches run at 115-122 us instead of 104 us), and the
timed region should see the steady device, as a solve of 1e5 steps does.

Prints one JSON line with the metric, a roofline object for the stage kernel
(its average duration measured with HIP events on the stream it runs on), the
CPU oracle timed on a bounded sample of the same workload, and the precision
path (FP32 storage) measured on the same GPU: on this workload and on the
precision workload (cavity 128x128 quads, p=4, NC 24x24, Kn=8) beside FP64;
batched and served mixes of problems (served in plain FP64 and in the
reference form: an FP32 correction to an FP64 reference); and the implicit
(backward Euler, Newton-Krylov) steps beside explicit RK4.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ALG_BYTES_PER_DOF_STAGE = 32.0  # FP64 RK4, 3 registers: 24/40/40/24 B per stage -> 32 mean
# what the FP64 kernels move (the accumulator written once per step): 16/32/24/32 -> 26 mean
ALG_BYTES_PER_DOF_STAGE_KERNEL = 26.0
# FP32 increment-form RK4: 12/20/20/16 B per stage -> 17 mean (what the
# kernels move); the method's own FP32 figure (3 registers) is 16 B
ALG_BYTES_PER_DOF_STAGE_FP32 = 17.0
ALG_BYTES_PER_DOF_STAGE_FP32_METHOD = 16.0
# reference form: the FP32 increment form plus the FP32 L(f_r) read once per stage
ALG_BYTES_PER_DOF_STAGE_REF = 21.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_cavity64x64_p3_nc16_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2012_13487_amd", "csrc", "kernels.hip")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic():
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken from a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(spec, budget_s):
    """The FP64 oracle on the host's cores, on a bounded number of RK4 steps;
    then on one thread, on a smaller bounded sample of the same workload."""
    import oracle

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o = oracle.Oracle.from_spec(spec)
    dt = o.stable_dt(spec.cfl)
    dof = o.Q * o.K * o.Np

    def rate(nthreads, budget, cap):
        oracle.set_threads(nthreads)
        o.init_equilibrium()
        t0 = time.perf_counter()
        o.rk4(1, dt)
        one = time.perf_counter() - t0
        n = max(1, min(cap, int(budget / max(one, 1e-9)) - 1))
        t0 = time.perf_counter()
        o.rk4(n, dt)
        return dof * 4 * n / (time.perf_counter() - t0), n, oracle.num_threads()

    v, n, used = rate(threads, budget_s, 50)
    v1, n1, _ = rate(1, budget_s / 3, 10)
    return {"value": v, "unit": "DOF-updates/s", "cores": used, "kind": "oracle",
            "sample": f"{n} RK4 steps ({4 * n} stages) of the same {dof}-DOF cavity workload, "
                      f"FP64 C oracle, OpenMP over elements",
            "single_thread": {"value": v1, "unit": "DOF-updates/s", "cores": 1,
                              "sample": f"{n1} RK4 steps of the same workload on one thread"},
            "cpu_model": cpu_model(), "host_cpus_visible": len(os.sched_getaffinity(0))}


def time_steps(solver, steps, dt):
    """Wall time of `steps` RK4 steps on the solver's stream (HIP events)."""
    import torch
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    solver.step(steps, dt)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def precision_path(steps_small, steps_big):
    """DOF-updates/s of the FP32-storage path next to FP64, on the benchmark
    workload and on the precision workload (all inputs resident in HBM)."""
    import workloads
    from paper_2012_13487_amd import Solver
    out = {}
    for key, spec, steps, precs in (
            ("cavity64x64_p3_nc16", workloads.CAVITY_64x64_P3_NC16, steps_small,
             ("fp32", "fp32_bf16mma", "fp32_ref")),
            ("cavity128x128_p4_nc24_kn8", workloads.CAVITY_128x128_P4_NC24_KN8, steps_big,
             ("fp32", "fp32_bf16mma", "fp32_ref", "fp64"))):
        entry = {}
        for prec in precs:
            g = Solver.from_spec(spec, precision=prec, stream="torch", torch_memory=True)
            dt = g.stable_dt(spec.cfl)
            g.init_equilibrium()
            time_steps(g, 2, dt)
            ms = time_steps(g, steps, dt)
            stage_us = 1000.0 * ms / (4 * steps)
            bpd = (ALG_BYTES_PER_DOF_STAGE if prec == "fp64" else
                   ALG_BYTES_PER_DOF_STAGE_REF if prec == "fp32_ref" else ALG_BYTES_PER_DOF_STAGE_FP32)
            ach = bpd * g.ndof / (stage_us * 1e-6) / 1e9
            entry["dof"] = g.ndof
            entry[prec] = {"value": g.ndof * 4 * steps / (ms / 1000.0), "unit": "DOF-updates/s",
                           "avg_launch_us": stage_us, "alg_bytes_per_dof_stage": bpd,
                           "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS, "steps": steps,
                           "tiling": g.tiling()}
            if prec in ("fp32", "fp32_bf16mma"):
                # the method's 3-register FP32 figure, beside the increment form's
                m = ALG_BYTES_PER_DOF_STAGE_FP32_METHOD * g.ndof / (stage_us * 1e-6) / 1e9
                entry[prec]["frac_at_16B_per_dof_stage"] = m / HBM_PEAK_GBS
            g.close()
        out[key] = entry
    big = out["cavity128x128_p4_nc24_kn8"]
    out["fp32_over_fp64_precision_workload"] = big["fp32"]["value"] / big["fp64"]["value"]
    out["bf16_over_fp64_precision_workload"] = big["fp32_bf16mma"]["value"] / big["fp64"]["value"]
    out["ref_over_fp64_precision_workload"] = big["fp32_ref"]["value"] / big["fp64"]["value"]
    out["note"] = ("fp32 = state stored as the FP32 deviation from w_q; moments, wall densities and "
                   "residual in FP64 (error vs the FP64 oracle <= 1e-5 in the GPU tests); "
                   "fp32_bf16mma = the same with the volume contractions on bf16 matrix cores "
                   "(<= 2e-3); fp32_ref = FP32 correction to an FP64 reference state, L(f_r) "
                   "streamed in FP32 (<= 1e-5, reaches FP64's steady-state residuals)")
    return out


def batching(steps):
    """The 64-problem mixed batch (seed 0): aggregate DOF-updates/s of the
    problems stepped one after another by the single-problem path (FP64, each
    in its default decomposition), and of the persistent batched kernels with
    hipGraph-replayed RK4 steps in FP64 and in FP32 storage."""
    import numpy as np
    import workloads
    from paper_2012_13487_amd import Batch, Solver

    specs = workloads.batch_instances(seed=0, n=64)
    out = {"workload": "64 mixed problems, seed 0: Couette or cavity, N x N quads with N in "
                       "16..96, p in 2..4, Kn log-uniform in [0.1, 10], D2Q16 GH or NC MxM, "
                       "M in 8..24",
           "steps": steps}

    def run(prec, batched):
        solvers = [Solver.from_spec(sp, precision=prec, stream="torch", torch_memory=True)
                   for sp in specs]
        for g in solvers:
            g.init_equilibrium()
        tuned = {}
        if batched:
            # the autotuner on every member (fused blocks of each admissible
            # size and, in FP64, velocity tiles); the batch keeps the choice of
            # members large enough to run their own kernels and gives the
            # others the fused form
            for g in solvers:
                g.autotune(3)
                tuned[(g.p, g.Q)] = g.tiling()["elems_per_group"]
        dts = np.array([g.stable_dt(sp.cfl) for g, sp in zip(solvers, specs)])
        dof = sum(g.ndof for g in solvers)
        if batched:
            b = Batch(solvers, stream="torch", graph=True)
            b.step(1, dts)  # builds the graph
            ms = _timed(lambda: b.step(steps, dts))
            launches = b.launches_per_step()
            b.close()
        else:
            for g, dt in zip(solvers, dts):
                g.step(1, dt)
            ms = _timed(lambda: [g.step(steps, dt) for g, dt in zip(solvers, dts)])
            launches = 4 * len(solvers)
        for g in solvers:
            g.close()
        res = {"value": dof * 4 * steps / (ms / 1000.0), "unit": "DOF-updates/s",
               "ms_per_step": ms / steps, "launches_per_step": launches}
        if tuned:
            res["autotuned_classes"] = len(tuned)
        return res, dof

    out["sequential_fp64"], out["dof"] = run("fp64", False)
    out["batched_fp64_graph"], _ = run("fp64", True)
    out["batched_fp32_graph"], _ = run("fp32", True)
    out["batched_fp64_over_sequential"] = (out["batched_fp64_graph"]["value"]
                                           / out["sequential_fp64"]["value"])
    out["batched_fp32_over_sequential_fp64"] = (out["batched_fp32_graph"]["value"]
                                                / out["sequential_fp64"]["value"])
    return out


# The served workload of the default run: the config-4 mix of problems scaled
# down (N x N quads with N in 16..28, p in 2..3, Kn log-uniform in
# [10^-0.5, 10], NC M x M with M in 6..12) so that 32 steady-state solves finish
# in about half a minute per precision; the full mix is served by --serving-full.
SERVE_REDUCED = dict(n_range=(16, 28), p_choices=(2, 3), kn_log10=(-0.5, 1.0), m_range=(6, 12))
SERVE_FULL = dict(n_range=(16, 96), p_choices=(2, 3, 4), kn_log10=(-1.0, 1.0), m_range=(8, 24))


def serving(n_requests, dist, time_limit_s, label, precisions=("fp64", "fp32_ref"), max_active=16):
    """Steady-state serving (continuous batching) of a seeded Poisson stream
    (rate 20/s, seed 1) of requests drawn from the mixed-problem distribution
    `dist` (seed 2), each run from rest to residual 1e-6: served DOF-updates/s
    and p50/p99 latency (arrival to residual 1e-6) for plain FP64 and for the
    reference form (FP32 correction streamed, FP64 reference folded at every
    residual check).  At most max_active requests run at once (the others wait
    for a slot); requests still running at the time limit count in
    `dof_updates_all_per_s` and not in `value`."""
    import workloads
    from paper_2012_13487_amd import Server

    reqs = workloads.batch_instances(seed=2, n=n_requests, **dist)
    arrivals = workloads.poisson_arrivals(seed=1, rate=20.0, n=n_requests)
    out = {"workload": f"{n_requests} requests, Poisson arrivals at 20/s (seed 1), {label} (seed 2): "
                       f"N x N quads with N in {dist['n_range'][0]}..{dist['n_range'][1]}, "
                       f"p in {dist['p_choices']}, Kn log-uniform in "
                       f"[{10 ** dist['kn_log10'][0]:.3g}, {10 ** dist['kn_log10'][1]:.3g}], "
                       f"D2Q16 GH or NC MxM with M in {dist['m_range'][0]}..{dist['m_range'][1]}",
           "residual_target": 1e-6, "check_every": 50, "time_limit_s": time_limit_s,
           "max_active": max_active, "hbm_budget_bytes": 64 << 30,
           "offered_requests_per_s": 20.0}
    for prec in precisions:
        sv = Server(hbm_budget=64 << 30, max_active=max_active, precision=prec,
                    residual_target=1e-6, check_every=50, max_steps=5_000_000, graph=True)
        ids = [sv.submit(r, a) for r, a in zip(reqs, arrivals)]
        # in slices of at most a minute (the server resumes where it stopped),
        # reporting progress between them
        t0 = time.perf_counter()
        while True:
            left = time_limit_s - (time.perf_counter() - t0)
            try:
                sv.run(max(1.0, min(60.0, left)))
                break  # every request completed
            except Exception as e:  # a time limit: report what was served
                if "time limit" not in str(e):
                    raise
            st = sv.stats()
            print(f"serving {label} {prec}: {st['completed']}/{n_requests} completed after "
                  f"{st['wall_s']:.0f} s", file=sys.stderr, flush=True)
            if time.perf_counter() - t0 >= time_limit_s:
                break
        st = sv.stats()
        res = [sv.result(i) for i in ids]
        conv = sum(r["status"] == 2 for r in res)
        sv.close()
        done = [r for r in res if r["status"] == 2]
        out[prec] = {
            "value": st["dof_updates"] / st["wall_s"], "unit": "DOF-updates/s",
            "dof_updates_all_per_s": st["dof_updates_all"] / st["wall_s"],
            "latency_p50_s": st["latency_p50_s"], "latency_p99_s": st["latency_p99_s"],
            "wall_s": st["wall_s"], "converged": conv, "admitted": st["admitted"],
            "served_requests_per_s": conv / st["wall_s"],
            "peak_active": st["peak_active"], "batch_rebuilds": st["batch_rebuilds"],
            "steps_median": float(sorted(r["steps"] for r in done)[len(done) // 2]) if done else None,
            "steps_max": max((r["steps"] for r in done), default=None)}
        print(f"serving {label} {prec}: {json.dumps(out[prec])}", file=sys.stderr, flush=True)
    if "fp32_ref" in out and "fp64" in out:
        out["mixed_over_fp64"] = out["fp32_ref"]["value"] / out["fp64"]["value"]
        out["mixed_note"] = ("mixed = the reference form: FP32 correction streamed by the stages, FP64 "
                             "reference, moments and residual; error vs the FP64 oracle <= 1e-5 in the "
                             "GPU tests (1e-10 observed on served results)")
    return out


def implicit_path(steps=2, mult=10.0, race_target=1e-6):
    """Implicit backward-Euler steps (Newton with matrix-free GMRES, the
    paper's time marching) on the benchmark cavity at 10 explicit step sizes,
    against explicit RK4 covering the same simulated time; and a race to the
    steady state (residual below race_target times its initial value) on a
    small cavity (8x8 quads, p=2, NC 8x8, Kn=1): backward Euler at 5000
    explicit step sizes against explicit RK4 at CFL 0.2."""
    import torch

    import workloads
    from paper_2012_13487_amd import Solver

    spec = workloads.CAVITY_64x64_P3_NC16
    g = Solver.from_spec(spec)
    g.init_equilibrium()
    dt = g.stable_dt(spec.cfl)
    g.implicit_step(1, mult * dt, "backward_euler")  # workspace allocation, warm-up
    t0 = time.perf_counter()
    rep = g.implicit_step(steps, mult * dt, "backward_euler")
    imp_s = (time.perf_counter() - t0) / steps
    g.synchronize()
    t0 = time.perf_counter()
    g.step(int(mult) * steps, dt)
    g.synchronize()
    exp_s = (time.perf_counter() - t0) / (int(mult) * steps)
    out = {"workload": "cavity 64x64 p=3 NC16, backward Euler at dt = "
                       f"{mult:g} x the explicit CFL-0.2 step, from rest",
           "ms_per_step": imp_s * 1e3,
           "newton_per_step": rep["newton_iterations"] / steps,
           "krylov_per_step": rep["krylov_iterations"] / steps,
           "rhs_evaluations_per_step": rep["rhs_evaluations"] / steps,
           "simulated_time_per_s": mult * dt / imp_s,
           "explicit_rk4_simulated_time_per_s": dt / exp_s}
    out["implicit_over_explicit"] = out["simulated_time_per_s"] / out["explicit_rk4_simulated_time_per_s"]
    # the Krylov basis in FP32 against FP64 at the loosest tolerance it allows
    basis = {"krylov_rtol": 1e-5}
    for name, fp32 in (("fp64_basis", False), ("fp32_basis", True)):
        g.init_equilibrium()
        g.implicit_step(1, mult * dt, "backward_euler", krylov_rtol=1e-5, krylov_fp32=fp32)
        t0 = time.perf_counter()
        rep = g.implicit_step(steps, mult * dt, "backward_euler", krylov_rtol=1e-5, krylov_fp32=fp32)
        basis[name] = {"ms_per_step": (time.perf_counter() - t0) / steps * 1e3,
                       "krylov_per_step": rep["krylov_iterations"] / steps}
    basis["fp32_over_fp64_speed"] = basis["fp64_basis"]["ms_per_step"] / basis["fp32_basis"]["ms_per_step"]
    out["krylov_basis"] = basis
    del g

    small = workloads.cavity(n=8, p=2, m=8, lid=0.1, kn=1.0)
    race = {"workload": small.name, "target": f"residual < {race_target:g} x initial"}
    g = Solver.from_spec(small)
    g.init_equilibrium()
    r0 = g.residual()
    dts = g.stable_dt(small.cfl)
    t0 = time.perf_counter()
    n = 0
    while g.residual() > race_target * r0 and n < 50:
        g.implicit_step(1, 5000 * dts, "backward_euler", max_krylov=1000)
        n += 1
    race["backward_euler_s"] = time.perf_counter() - t0
    race["backward_euler_steps"] = n
    g.init_equilibrium()
    t0 = time.perf_counter()
    n = 0
    while g.residual() > race_target * r0 and n < 400_000:
        g.step(500, dts)
        n += 500
    race["explicit_rk4_s"] = time.perf_counter() - t0
    race["explicit_rk4_steps"] = n
    out["steady_state_race"] = race
    torch.cuda.synchronize()
    return out


def couette_config1(repeats=5):
    """The plain-method Couette workload (8x8 quads, p=2, D2Q16, Kn=1, 200 RK4
    steps from rest, 9,216 DOF): latency-bound, so timed with the autotuned
    block size, with ordinary launches and with the steps replayed from a
    captured hipGraph (50 steps per graph), each the median of `repeats`
    200-step solves."""
    import workloads
    from paper_2012_13487_amd import Solver

    spec = workloads.COUETTE_8x8_P2_D2Q16
    out = {"workload": "Couette [0,1]^2, walls +-0.1, 8x8 quads p=2, D2Q16 Gauss-Hermite, Kn=1 "
                       "(tau = Kn/sqrt(pi/2)), FP64 RK4 CFL 0.2, 200 steps from rest",
           "steps": spec.steps}
    for name, k in (("eager", 0), ("graph", 50)):
        g = Solver.from_spec(spec, stream="torch", torch_memory=True)
        g.set_graph(k)
        dt = g.stable_dt(spec.cfl)
        g.init_equilibrium()
        # the autotuner's block size: alone, this 64-element problem runs fastest with
        # one element per work-group (the automatic choice, 16, suits batches of it)
        g.autotune(200)  # (launches of a few us: fewer than ~100 let noise pick the block size)
        g.step(spec.steps, dt)  # warm-up (and the graph capture)
        times = []
        for _ in range(repeats):
            g.init_equilibrium()
            times.append(_timed(lambda: g.step(spec.steps, dt)))
        ms = sorted(times)[len(times) // 2]
        out[name] = {"value": g.ndof * 4 * spec.steps / (ms / 1000.0), "unit": "DOF-updates/s",
                     "ms_per_solve": ms, "us_per_stage": 1000.0 * ms / (4 * spec.steps),
                     "steps_per_graph": k, "tiling": g.tiling()}
        out["dof"] = g.ndof
        g.close()
    out["graph_over_eager"] = out["graph"]["value"] / out["eager"]["value"]
    return out


def converge(resid_every, max_steps, max_s, target=1e-6, precision="fp64"):
    """The benchmark cavity (64x64 quads, p=3, NC 16x16, Kn=1) from rest to
    residual `target`: RK4 steps and device time, the residual evaluated on
    the device every `resid_every` steps (its launches are in the time); in a
    reference form the correction is folded after every evaluation."""
    import torch

    import workloads
    from paper_2012_13487_amd import Solver

    spec = workloads.CAVITY_64x64_P3_NC16
    g = Solver.from_spec(spec, precision=precision, stream="torch", torch_memory=True)
    dt = g.stable_dt(spec.cfl)
    g.init_equilibrium()
    fold = precision.endswith("_ref")
    resid = torch.zeros(1, dtype=torch.float64, device="cuda")
    history = []
    steps = 0
    t0 = time.perf_counter()
    r = g.residual()
    history.append((0, r))
    while r >= target and steps < max_steps and time.perf_counter() - t0 < max_s:
        g.step(resid_every, dt)
        steps += resid_every
        g.residual_async(resid.data_ptr())
        if fold:
            g.fold()
        r = float(resid.item())
        if steps % (50 * resid_every) == 0 or r < target:
            history.append((steps, r))
            print(f"converge: step {steps} residual {r:.3e} "
                  f"elapsed {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    return {"workload": "lid-driven cavity 64x64 quads p=3, NC 16x16 velocities on [-4,4]^2, Kn=1, "
                        "lid 0.1, diffuse walls, RK4 CFL 0.2, from rest", "precision": precision,
            "target": target, "converged": r < target, "steps": steps, "residual": r,
            "dt": dt, "simulated_time": steps * dt, "wall_s": wall,
            "dof_updates_per_s": g.ndof * 4 * steps / wall, "residual_every": resid_every,
            "history": history}


def _timed(fn):
    """Milliseconds of the device work `fn` enqueues on torch's current stream."""
    import torch
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--resid-every", type=int, default=50)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up (clock ramp)")
    ap.add_argument("--converge", action="store_true",
                    help="only run the benchmark cavity from rest to residual 1e-6 and "
                         "report steps and time")
    ap.add_argument("--converge-max-s", type=float, default=1000.0)
    ap.add_argument("--converge-precision", default="fp64",
                    help="precision of the --converge run (fp64, fp32_ref, ...)")
    ap.add_argument("--no-couette", action="store_true")
    ap.add_argument("--precision-steps", default="100,20", metavar="S,B",
                    help="RK4 steps timed on the 64x64 and on the 128x128 precision workloads")
    ap.add_argument("--serving-full", type=int, default=0, metavar="N",
                    help="only serve N requests of the full-size mixed distribution (both "
                         "precisions, each under --serving-time-limit seconds)")
    ap.add_argument("--serving-time-limit", type=float, default=480.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-path", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-implicit", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB (5 times), to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters of the stage kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the workload runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2012_13487_amd import Solver

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": x.numel() * 8,
                          "bytes_written": x.numel() * 8, "launches": 5}), flush=True)
        return
    if args.converge:
        print(json.dumps({"converge": converge(1000, 3_000_000, args.converge_max_s,
                                                precision=args.converge_precision)}), flush=True)
        return
    if args.serving_full:
        print(json.dumps({"serving_full": serving(
            args.serving_full, SERVE_FULL, args.serving_time_limit,
            "the config-4 mixed-problem distribution at full size, request count capped",
            max_active=64)}),
            flush=True)
        return
    spec = workloads.CAVITY_64x64_P3_NC16
    g = Solver.from_spec(spec, stream="torch", torch_memory=True)
    dt = g.stable_dt(spec.cfl)
    dof = g.ndof
    g.init_equilibrium()
    resid = torch.zeros(max(1, args.steps // max(1, args.resid_every)) + 1,
                        dtype=torch.float64, device="cuda")
    settle_steps = 0
    if args.settle_s > 0:
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.settle_s:
            g.step(20, dt)
            settle_steps += 20
            torch.cuda.synchronize()
        g.init_equilibrium()  # the timed steps start from rest, as without settling
    if args.warmup:
        g.step(args.warmup, dt)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    chunk = max(1, args.resid_every)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    pairs = []
    t_start.record(stream)
    done, nres = 0, 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        g.step(n, dt)
        b.record(stream)
        pairs.append((a, b, n))
        done += n
        if done % chunk == 0:
            g.residual_async(resid[nres].data_ptr())
            nres += 1
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    step_ms = sum(a.elapsed_time(b) for a, b, _ in pairs)
    stage_launches = 4 * sum(n for _, _, n in pairs)
    stage_us = 1000.0 * step_ms / stage_launches
    value = dof * 4 * args.steps / (total_ms / 1000.0)
    achieved = ALG_BYTES_PER_DOF_STAGE * dof / (stage_us * 1e-6) / 1e9
    traffic = measured_traffic()
    res = resid[:nres].cpu().tolist()

    out = {
        "metric": "DG-BGK DOF-updates/s (nodes x velocities x RK stages)",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "lid-driven cavity 64x64 quads p=3, NC 16x16 velocities on [-4,4]^2, "
                        "Kn=1, lid 0.1, diffuse walls, FP64 RK4 CFL 0.2",
            "dof": dof, "elements": g.K, "nodes_per_element": g.Np, "velocities": g.Q,
            "dt": dt, "residual_every": args.resid_every,
            "residual_last": res[-1] if res else None,
            "device_settle_steps": settle_steps,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "stage_kernel<3>",
            "avg_launch_us": stage_us,
            "alg_bytes_per_launch": ALG_BYTES_PER_DOF_STAGE * dof,
            "kernel_alg_bytes_per_launch": ALG_BYTES_PER_DOF_STAGE_KERNEL * dof,
            "frac_at_kernel_bytes": ALG_BYTES_PER_DOF_STAGE_KERNEL * dof / (stage_us * 1e-6) / 1e9
                                    / HBM_PEAK_GBS,
        },
        "cpu_baseline": None,
    }
    del g
    if not args.no_couette:
        out["couette_config1"] = couette_config1()
    if not args.no_precision_path:
        ps, pb = (int(x) for x in args.precision_steps.split(","))
        out["precision_path"] = precision_path(ps, pb)
    if not args.no_batching:
        out["batching"] = batching(10)
    if not args.no_serving:
        out["serving"] = serving(32, SERVE_REDUCED, 300.0,
                                 "the mixed-problem distribution scaled down (not config 5's sizes)")
    if not args.no_implicit:
        out["implicit"] = implicit_path()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
