"""The C ABI from a plain C99 program: include/dgbgk.h compiles with
gcc -std=c99 -pedantic -Werror, the program links against libdgbgk.so, and its
results equal the Python binding's on the same problem (the binding is a thin
marshalling layer over the same calls)."""
import os
import shutil
import subprocess

import pytest

import workloads
from paper_2012_13487_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_client.c")
PKG = os.path.dirname(binding.LIB_PATH)
SPEC = workloads.cavity(n=6, ny=5, p=2, m=8, vmax=4.0, lid=0.1, kn=1.0)


def _build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "abi_client")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), SRC, "-L", PKG, "-ldgbgk",
                    f"-Wl,-rpath,{PKG}", "-lm", "-o", exe], check=True)
    return exe


def _run(exe, mode):
    r = subprocess.run([exe, mode], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    assert "ok" in lines
    head = lines[0].split()
    out = {head[i]: head[i + 1] for i in range(0, len(head), 2)}
    for ln in lines[1:]:
        if len(ln.split()) == 2:
            out[ln.split()[0]] = ln.split()[1]
    return out


def test_c_client_host_calls(tmp_path):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present: the device calls would succeed")
    except ImportError:
        pass
    out = _run(_build(tmp_path), "cpu")
    g = binding.Solver.from_spec(SPEC)
    assert (int(out["K"]), int(out["Np"]), int(out["Nfp"]), int(out["Q"])) == \
        (g.K, g.Np, g.Nfp, g.Q)
    assert float(out["dt"]) == g.stable_dt(0.2)
    assert int(out["bytes"]) == binding.required_bytes(
        SPEC.nx, SPEC.ny, SPEC.p, g.vel, g.tau, SPEC.bc, SPEC.wall_u)


@pytest.mark.gpu
def test_c_client_matches_binding_on_gpu(tmp_path):
    print("[gpu] C client: cavity 6x5 p2 nc8, 50 steps", flush=True)
    out = _run(_build(tmp_path), "gpu")
    g = binding.Solver.from_spec(SPEC)
    g.init_equilibrium()
    dt = g.stable_dt(0.2)
    assert float(out["dt"]) == dt
    g.step(50, dt)
    rho, ux, uy = g.moments()
    assert float(out["residual"]) == g.residual()
    assert float(out["umax"]) == float(abs(ux).max())
