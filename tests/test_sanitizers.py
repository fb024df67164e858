"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

A child process loads an instrumented copy of the oracle's C library and runs
every entry point on small 2D and 3D meshes (a power-of-two mesh and one of
25 * 2^k elements in 2D, whose coarse grid takes the other coarse-solve branch),
plus the iteration-limit and invalid-argument paths.  Any out-of-bounds
access, use after free, misaligned load or undefined arithmetic aborts the
child, and the test fails with the sanitizer's report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle.okref as R
R._LIBPATH = %r
from paper_1603_04570_amd.inputs import noise_state

def run(dim, n, theta):
    o = R.Oracle(dim, n, eps=0.05, sigma=30.0, m=0.1, dt=1e-3, theta=theta)
    u, w = noise_state(dim, n, 0.1, 7)
    for which in (R.MAT_M, R.MAT_K, R.MAT_A):
        o.matrix(which)
    o.matrix(R.MAT_ME, u=u)
    for lev in range(o.levels):
        o.matrix(R.MAT_A, level=lev)
        o.cheb_interval(lev)
        if lev < o.levels - 1:  # prolongation from level lev + 1
            o.matrix(R.MAT_P, level=lev)
    o.cheb_interval(0, mass=True)
    o.nonlinear(u)
    w0 = o.initial_w(u)
    o.residual(u, w0, u, w0)
    x = np.linspace(-1, 1, 2 * o.nodes)
    o.jacobian_apply(u, x)
    o.cheb_mass(x[:o.nodes])
    o.mg(x[:o.nodes], cycles=2)
    o.schur_apply(u, x[:o.nodes])
    o.precond_apply(u, x)
    o.fgmres(u, x)
    o.newton_step(u.copy(), w0.copy(), u, w0)
    o.timestep(u.copy(), w0.copy(), 2)
    nodes = np.arange(0, o.nodes, 3)
    R.local_residual(o.params, u, w0, u, w0, nodes)
    R.local_jacobian(o.params, u, x, nodes)
    o.close()

for dim, n, theta in [(2, 16, 1.0), (2, 50, 0.5), (3, 8, 1.0), (3, 16, 0.5)]:
    run(dim, n, theta)
# iteration limits and bad arguments take their error paths
o = R.Oracle(2, 16, eps=0.05, sigma=30.0, m=0.1, dt=1e-3, gmres_restart=1,
             gmres_max_restarts=0, gmres_rtol=1e-15)
u, w = noise_state(2, 16, 0.1, 8)
o.fgmres(u, np.ones(2 * o.nodes))
o.close()
try:
    R.Oracle(2, 1, eps=0.05, sigma=30.0, m=0.1, dt=1e-3)
except Exception:
    pass
print("sanitized oracle ok")
"""


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if not asan:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = str(tmp_path / "libokref_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    os.path.join(ROOT, "oracle", "okref.c"), "-o", lib, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD % lib], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    assert "sanitized oracle ok" in r.stdout
