"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import json
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ok.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ok_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1603_04570_amd import ok
    if not os.path.exists(ok.LIBPATH):
        from paper_1603_04570_amd.build import build
        build()
    return ok.load()


def test_exports_every_declared_symbol(lib):
    from paper_1603_04570_amd import ok
    syms = declared_symbols()
    assert len(syms) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", ok.LIBPATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ok_\w+)", out))
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    for s in syms:
        assert hasattr(lib, s)


def test_default_params_and_workspace(lib):
    from paper_1603_04570_amd import ok
    p = ok.default_params()
    assert (p.dim, p.n, p.gmres_restart, p.cheb_A_its, p.mg_pre, p.mg_post) == (3, 128, 30, 10, 2, 2)
    assert p.eps == 0.01 and p.sigma == 1000.0 and p.dt == 2e-5 and p.theta == 1.0
    b = ok.workspace_bytes(p)
    n = 129 ** 3
    # V (31 x 2n) and Z (30 x 2n) dominate: 61*2n doubles
    assert 61 * 2 * n * 8 <= b <= 61 * 2 * n * 8 + 40 * n * 8
    pm = ok.default_params(precision=ok.OK_MIXED)
    assert ok.workspace_bytes(pm) < b


def test_non_power_of_two_meshes_accepted(lib):
    """N = 25 * 2^k coarsens to 25 elements per direction (26^d coarse nodes)."""
    from paper_1603_04570_amd import ok
    for dim, n in [(2, 100), (3, 50), (3, 100), (2, 400)]:
        p = ok.default_params(dim=dim, n=n)
        b = C.c_size_t()
        assert lib.ok_workspace_bytes(C.byref(p), C.byref(b)) == 0 and b.value > 0


@pytest.mark.parametrize("field,value", [("dim", 4), ("n", 1), ("eps", 0.0), ("dt", -1.0),
                                         ("theta", 0.0), ("theta", 1.5), ("m", 1.0),
                                         ("precision", 7), ("gmres_restart", 0),
                                         ("gmres_restart", 65), ("cheb_A_its", 0),
                                         ("mg_pre", 0), ("mg_levels", 9),
                                         ("linear_solver", 2), ("linear_solver", -1),
                                         # 130 -> 65 elements: 66 coarse nodes per direction
                                         ("n", 130)])
def test_invalid_params_rejected(lib, field, value):
    from paper_1603_04570_amd import ok
    p = ok.default_params(**{field: value})
    b = C.c_size_t()
    assert lib.ok_workspace_bytes(C.byref(p), C.byref(b)) == -1
    ctx = C.c_void_p()
    assert lib.ok_assemble_mesh(C.byref(p), C.c_void_p(256), C.c_size_t(1 << 40), None,
                                C.byref(ctx)) == -1
    assert not ctx.value


def test_minres_params(lib):
    """MINRES is an FP64 path; its class keeps at least nine work vectors."""
    from paper_1603_04570_amd import ok
    b = C.c_size_t()
    pm = ok.default_params(linear_solver=ok.OK_SOLVER_MINRES, precision=ok.OK_MIXED)
    assert lib.ok_workspace_bytes(C.byref(pm), C.byref(b)) == -1
    p = ok.default_params(dim=2, n=64, linear_solver=ok.OK_SOLVER_MINRES)
    assert ok.workspace_bytes(p) > 0
    # gmres_restart below 8: the MINRES class still holds its nine vectors
    f4 = ok.workspace_bytes(ok.default_params(dim=2, n=64, gmres_restart=4))
    m4 = ok.workspace_bytes(ok.default_params(dim=2, n=64, gmres_restart=4,
                                              linear_solver=ok.OK_SOLVER_MINRES))
    assert m4 - f4 >= 4 * 2 * 65 * 65 * 8 - 256  # four more vectors of 2n, up to alignment
    assert lib.ok_sym_apply(None, None, None, None, None) == -1
    assert lib.ok_minres(None, None, None, None, None, None) == -1


def test_workspace_errors(lib):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=2, n=64)
    need = ok.workspace_bytes(p)
    ctx = C.c_void_p()
    # null, misaligned, and one byte too small: rejected without any device access
    assert lib.ok_assemble_mesh(C.byref(p), None, C.c_size_t(need), None, C.byref(ctx)) == -2
    assert lib.ok_assemble_mesh(C.byref(p), C.c_void_p(4096 + 8), C.c_size_t(need), None,
                                C.byref(ctx)) == -2
    assert lib.ok_assemble_mesh(C.byref(p), C.c_void_p(4096), C.c_size_t(need - 1), None,
                                C.byref(ctx)) == -2


def test_error_strings(lib):
    from paper_1603_04570_amd import ok
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert ok.error_string(s)
    assert ok.error_string(-99) == "unknown status"


def test_null_context_calls(lib):
    assert lib.ok_destroy(None) == -1
    assert lib.ok_jacobian_apply(None, None, None, None, None) == -1
    assert lib.ok_timestep(None, None, None, 1, None, None) == -1


def test_launch_shape_arguments(lib):
    """ok_set_launch_shape only edits the host-side shape table: argument
    checks run without a GPU."""
    E = -1  # OK_E_INVALID
    f = lib.ok_set_launch_shape  # (dim, n, kernel, precision, items, threads, zchunks)
    assert f(3, 64, 1, 0, 4, 256, 5) == 0
    assert f(3, 64, 1, 0, 4, 512, 5) == 0      # 512 threads of 4 nodes
    assert f(3, 64, 1, 0, 0, 0, 0) == 0        # clear
    assert f(3, 64, 3, 1, 2, 512, 65) == 0     # 512-thread fused pair
    assert f(3, 64, 3, 1, 0, 0, 0) == 0
    assert f(4, 64, 1, 0, 4, 256, 5) == E      # dim
    assert f(3, 0, 1, 0, 4, 256, 5) == E       # n
    assert f(3, 64, 12, 0, 4, 256, 5) == E     # kernel
    assert f(3, 64, 0, 0, 2, 256, 5) == E
    # strips (9, 10, 11): 3D, window configuration 1..5, 256 threads
    assert f(3, 64, 9, 0, 1, 256, 5) == 0 and f(3, 64, 10, 1, 2, 256, 9) == 0
    assert f(3, 64, 11, 0, 3, 256, 65) == 0
    assert f(3, 64, 9, 0, 4, 256, 5) == 0 and f(3, 64, 10, 0, 5, 256, 5) == 0
    assert f(3, 64, 9, 0, 0, 0, 0) == 0 and f(3, 64, 10, 0, 0, 0, 0) == 0
    assert f(3, 64, 9, 0, 0, 0, 0) == 0 and f(3, 64, 10, 1, 0, 0, 0) == 0
    assert f(3, 64, 11, 0, 0, 0, 0) == 0
    assert f(2, 64, 9, 0, 1, 256, 5) == E      # strips: 3D only
    assert f(3, 64, 9, 0, 6, 256, 5) == E      # configurations 1..5
    assert f(3, 64, 10, 0, 1, 512, 5) == E     # 256 threads
    assert f(3, 64, 6, 0, 2, 512, 5) == 0      # fused pair on in-plane tiles
    assert f(3, 64, 7, 0, 1, 256, 9) == 0 and f(3, 64, 8, 1, 2, 512, 3) == 0  # smoothers
    assert f(3, 64, 7, 0, 0, 0, 0) == 0 and f(3, 64, 8, 1, 0, 0, 0) == 0
    assert f(2, 64, 7, 0, 1, 256, 9) == E and f(3, 64, 8, 0, 3, 256, 9) == E
    assert f(3, 256, 6, 1, 1, 256, 257) == 0
    assert f(3, 64, 6, 0, 0, 0, 0) == 0 and f(3, 256, 6, 1, 0, 0, 0) == 0
    assert f(2, 64, 6, 0, 2, 256, 5) == E      # tiles: 3D only
    assert f(3, 64, 6, 0, 4, 256, 5) == E      # 1 or 2 nodes per thread
    assert f(3, 64, 6, 0, 2, 128, 5) == E
    assert f(3, 64, 1, 2, 4, 256, 5) == E      # precision
    assert f(3, 64, 1, 0, 3, 256, 5) == E      # items
    assert f(3, 64, 1, 0, 8, 512, 5) == E      # 512 threads: at most 4 nodes
    assert f(2, 64, 1, 0, 2, 512, 5) == E      # 512 threads: 3D only
    assert f(3, 64, 1, 0, 4, 128, 5) == E      # threads
    assert f(3, 64, 2, 0, 8, 256, 5) == E      # two fields: at most 4 nodes
    assert f(3, 64, 3, 0, 4, 256, 5) == E      # fused pair: 1 or 2 nodes
    assert f(2, 64, 3, 0, 2, 512, 5) == E      # fused 512-thread pair: 3D only
    assert f(3, 64, 4, 0, 2, 512, 9) == 0      # fused multigrid smoothers
    assert f(3, 64, 5, 1, 1, 256, 9) == 0
    assert f(3, 64, 4, 0, 0, 0, 0) == 0 and f(3, 64, 5, 1, 0, 0, 0) == 0
    assert f(3, 64, 5, 0, 4, 256, 9) == E
    assert f(3, 64, 1, 0, 4, 256, 0) == E      # zchunks
    assert f(3, 64, 1, 0, 4, 256, 66) == E


def test_set_option(lib):
    """ok_set_option edits process-wide host flags: every declared option is
    accepted (and restored to its default here), unknown ones are rejected."""
    from paper_1603_04570_amd import ok
    defaults = {ok.OK_OPT_FUSE_CHEB: 1, ok.OK_OPT_FUSE_MG: 1, ok.OK_OPT_ISSUE_AHEAD: 0,
                ok.OK_OPT_TRACE_RANGES: 0, ok.OK_OPT_GRAM_SCHMIDT: 0, ok.OK_OPT_FUSE_PROLONG: 1}
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    declared = {int(v) for v in re.findall(r"\bOK_OPT_[A-Z_]+\s*=\s*(\d+)", text)}
    assert declared == set(defaults)
    for opt, dflt in defaults.items():
        assert lib.ok_set_option(opt, 1 - dflt) == 0
        assert lib.ok_set_option(opt, dflt) == 0
    for bad in (0, 7, -1, 1000):
        assert lib.ok_set_option(bad, 1) == -1


def test_get_launch_shape_round_trip(lib):
    """ok_get_launch_shape reads back what ok_set_launch_shape wrote (host
    table only), and reports 0s for a grid with no entry."""
    from paper_1603_04570_amd import ok
    cases = [(3, 64, ok.OK_SHAPE_MG_POST_STRIP, ok.OK_FP64, 4, 256, 9),
             (3, 96, ok.OK_SHAPE_CHEB2_TILE, ok.OK_MIXED, 2, 512, 97),
             (2, 64, ok.OK_SHAPE_STENCIL, ok.OK_FP64, 8, 256, 5)]
    try:
        for dim, n, kern, prec, items, threads, zch in cases:
            assert ok.get_launch_shape(dim, n, kern, prec) == (0, 0, 0)
            ok.set_launch_shape(dim, n, kern, prec, items, threads, zch)
            assert ok.get_launch_shape(dim, n, kern, prec) == (items, threads, zch)
            other = ok.OK_MIXED if prec == ok.OK_FP64 else ok.OK_FP64
            assert ok.get_launch_shape(dim, n, kern, other) == (0, 0, 0)
    finally:
        for dim, n, kern, prec, *_ in cases:
            ok.set_launch_shape(dim, n, kern, prec, 0)
    for dim, n, kern, prec, *_ in cases:
        assert ok.get_launch_shape(dim, n, kern, prec) == (0, 0, 0)
    i = C.c_int32()
    E = -1
    assert lib.ok_get_launch_shape(4, 64, 1, 0, C.byref(i), C.byref(i), C.byref(i)) == E
    assert lib.ok_get_launch_shape(3, 64, 12, 0, C.byref(i), C.byref(i), C.byref(i)) == E
    assert lib.ok_get_launch_shape(3, 64, 1, 2, C.byref(i), C.byref(i), C.byref(i)) == E
    assert lib.ok_get_launch_shape(3, 64, 1, 0, None, C.byref(i), C.byref(i)) == E


def test_bench_launch_shapes_save_and_load(lib, tmp_path):
    """bench.py --save-shapes writes the table entries of the configuration's
    grids (every level of the hierarchy, both precisions) and --load-shapes
    pins them instead of autotuning (host-side table only)."""
    import argparse
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_1603_04570_amd import ok
    path = str(tmp_path / "shapes.json")
    pins = [(64, ok.OK_SHAPE_MG_POST_STRIP, ok.OK_FP64, 4, 256, 9),
            (32, ok.OK_SHAPE_CHEB2_TILE, ok.OK_MIXED, 2, 512, 5),
            (16, ok.OK_SHAPE_STENCIL, ok.OK_FP64, 2, 256, 3)]

    class FakeProblem:
        def autotune(self):
            for n, kern, prec, items, threads, zch in pins:
                ok.set_launch_shape(3, n, kern, prec, items, threads, zch)
            return len(pins)

    cfg = {"dim": 3, "n": 64}
    try:
        args = argparse.Namespace(load_shapes=None, save_shapes=path, no_autotune=False)
        assert bench._tune(args, ok, FakeProblem(), cfg) == len(pins)
        saved = json.load(open(path))
        assert {(e["n"], e["kernel"], e["precision"], e["items"], e["threads"], e["zchunks"])
                for e in saved} == set(pins)
        for n, kern, prec, *_ in pins:
            ok.set_launch_shape(3, n, kern, prec, 0)
        args = argparse.Namespace(load_shapes=path, save_shapes=None, no_autotune=False)
        assert bench._tune(args, ok, None, cfg) == len(pins)
        for n, kern, prec, items, threads, zch in pins:
            assert ok.get_launch_shape(3, n, kern, prec) == (items, threads, zch)
    finally:
        for n, kern, prec, *_ in pins:
            ok.set_launch_shape(3, n, kern, prec, 0)
