"""ctypes binding of libok.so (argument marshalling only).

Every operation runs in the library's HIP kernels; PyTorch is used only to
allocate device memory and to supply the current HIP stream.  The binding
raises if the library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "libok.so")

OK_FP64, OK_MIXED = 0, 1
OK_SOLVER_FGMRES, OK_SOLVER_MINRES = 0, 1
OK_K_NONE, OK_K_CHEB_MASS, OK_K_MG_SMOOTH, OK_K_ELEMENT, OK_K_KRYLOV = 0, 1, 2, 3, 5
HIST = 256

STATUS = {0: "OK_SUCCESS", -1: "OK_E_INVALID", -2: "OK_E_WORKSPACE", -3: "OK_E_HIP",
          -4: "OK_E_GMRES_MAXIT", -5: "OK_E_NEWTON_MAXIT", -6: "OK_E_NONFINITE",
          -7: "OK_E_REJECTED"}
OK_E_WORKSPACE, OK_E_REJECTED = -2, -7


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32),
                ("eps", C.c_double), ("sigma", C.c_double), ("m", C.c_double),
                ("dt", C.c_double), ("theta", C.c_double),
                ("precision", C.c_int32),
                ("gmres_restart", C.c_int32), ("gmres_max_restarts", C.c_int32),
                ("gmres_rtol", C.c_double), ("newton_atol", C.c_double),
                ("newton_max_it", C.c_int32), ("cheb_A_its", C.c_int32),
                ("schur_richardson", C.c_int32), ("mg_levels", C.c_int32),
                ("mg_pre", C.c_int32), ("mg_post", C.c_int32), ("mg_cycles", C.c_int32),
                ("linear_solver", C.c_int32)]


class NewtonInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("fgmres_its", C.c_int32), ("restarts", C.c_int32),
                ("fnorm", C.c_double), ("lin_res", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps_done", C.c_int32), ("newton_its", C.c_int32),
                ("fgmres_its_total", C.c_int32), ("newton_per_step", C.c_int32 * HIST),
                ("fgmres_its", C.c_int32 * HIST), ("fnorm", C.c_double * HIST),
                ("fnorm_count", C.c_int32), ("step_ms", C.c_double * HIST)]

    def its(self):
        return [self.fgmres_its[i] for i in range(min(self.newton_its, HIST))]

    def per_step(self):
        return [self.newton_per_step[i] for i in range(min(self.steps_done, HIST))]

    def fnorms(self):
        return [self.fnorm[i] for i in range(min(self.fnorm_count, HIST))]

    def ms(self):
        return [self.step_ms[i] for i in range(min(self.steps_done, HIST))]


class ServerConfig(C.Structure):
    _fields_ = [("max_queue", C.c_int32), ("max_slots_per_pool", C.c_int32),
                ("graphs", C.c_int32), ("reserved", C.c_int32), ("pool_bytes", C.c_double)]


class RequestResult(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("sim", C.c_int32), ("nsteps", C.c_int32),
                ("status", C.c_int32), ("steps_done", C.c_int32), ("newton_its", C.c_int32),
                ("fgmres_its", C.c_int32), ("t_arrival", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "submitted", "admitted", "completed", "failed", "rejected", "deferred", "ticks",
        "pools_created", "pools_freed", "pools_live", "max_active", "max_queue_seen",
        "peak_bytes", "bytes_in_use")] + [("dof_steps", C.c_double), ("busy_s", C.c_double),
                                          ("now", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OkError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libok.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise OSError(f"{LIBPATH} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(LIBPATH)
    vp, i32, d = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    lib.ok_default_params.argtypes = [P(Params)]
    lib.ok_workspace_bytes.argtypes = [P(Params), P(C.c_size_t)]
    lib.ok_assemble_mesh.argtypes = [P(Params), vp, C.c_size_t, vp, P(vp)]
    lib.ok_residual.argtypes = [vp, vp, vp, vp, vp, vp, P(d), vp]
    lib.ok_residual_noalloc.argtypes = [P(Params), vp, vp, vp, vp, vp, P(d), vp]
    lib.ok_jacobian_apply.argtypes = [vp, vp, vp, vp, vp]
    lib.ok_precond_apply.argtypes = [vp, vp, vp, vp, vp]
    lib.ok_sym_apply.argtypes = [vp, vp, vp, vp, vp]
    lib.ok_minres.argtypes = [vp, vp, vp, vp, P(i32), vp]
    lib.ok_cheb_mass.argtypes = [vp, vp, vp, vp]
    lib.ok_mg_apply.argtypes = [vp, vp, vp, i32, vp]
    lib.ok_fgmres.argtypes = [vp, vp, vp, vp, P(i32), vp]
    lib.ok_newton_step.argtypes = [vp, vp, vp, vp, vp, P(NewtonInfo), vp]
    lib.ok_timestep.argtypes = [vp, vp, vp, i32, P(Stats), vp]
    lib.ok_autotune.argtypes = [vp, vp, P(i32)]
    lib.ok_profile_enable.argtypes = [vp, i32]
    lib.ok_profile_read.argtypes = [vp, i32, P(C.c_int64), P(d), P(d)]
    lib.ok_destroy.argtypes = [vp]
    lib.ok_batch_workspace_bytes.argtypes = [P(Params), i32, P(C.c_size_t)]
    lib.ok_batch_create.argtypes = [P(Params), i32, vp, C.c_size_t, vp, P(vp)]
    lib.ok_batch_set_state.argtypes = [vp, i32, vp, vp, vp]
    lib.ok_batch_get_state.argtypes = [vp, i32, vp, vp, vp]
    lib.ok_batch_timestep.argtypes = [vp, i32, P(Stats), vp]
    lib.ok_batch_autotune.argtypes = [vp, vp, P(i32)]
    lib.ok_batch_classes.argtypes = [vp]
    lib.ok_batch_destroy.argtypes = [vp]
    lib.ok_batch_last_error.argtypes = [vp]
    lib.ok_batch_last_error.restype = C.c_char_p
    lib.ok_use_graphs.argtypes = [vp, i32]
    lib.ok_set_option.argtypes = [i32, i32]
    lib.ok_set_launch_shape.argtypes = [i32] * 7
    lib.ok_get_launch_shape.argtypes = [i32] * 4 + [C.POINTER(i32)] * 3
    lib.ok_initial_w.argtypes = [vp, vp, vp, vp]
    lib.ok_batch_use_graphs.argtypes = [vp, i32]
    lib.ok_server_default_config.argtypes = [P(ServerConfig)]
    lib.ok_server_state_bytes.argtypes = [P(Params), i32, P(C.c_size_t)]
    lib.ok_server_create.argtypes = [P(Params), i32, P(ServerConfig), vp, C.c_size_t, vp, P(vp)]
    lib.ok_server_set_state.argtypes = [vp, i32, vp, vp, vp]
    lib.ok_server_get_state.argtypes = [vp, i32, vp, vp, vp]
    lib.ok_server_start.argtypes = [vp]
    lib.ok_server_now.argtypes = [vp]
    lib.ok_server_now.restype = d
    lib.ok_server_submit.argtypes = [vp, i32, i32, d, P(C.c_int64)]
    lib.ok_server_poll.argtypes = [vp, P(RequestResult), i32, P(i32), d]
    lib.ok_server_stop.argtypes = [vp, i32]
    lib.ok_server_get_stats.argtypes = [vp, P(ServerStats)]
    lib.ok_server_reset_stats.argtypes = [vp]
    lib.ok_server_destroy.argtypes = [vp]
    lib.ok_server_last_error.argtypes = [vp]
    lib.ok_server_last_error.restype = C.c_char_p
    lib.ok_error_string.argtypes = [C.c_int]
    lib.ok_error_string.restype = C.c_char_p
    lib.ok_last_error.argtypes = [vp]
    lib.ok_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def default_params(**kw) -> Params:
    p = Params()
    load().ok_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def workspace_bytes(p: Params) -> int:
    b = C.c_size_t()
    st = load().ok_workspace_bytes(C.byref(p), C.byref(b))
    if st:
        raise OkError(st, "ok_workspace_bytes")
    return b.value


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "need a contiguous cuda float64 tensor"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def residual_noalloc(p: Params, u, w, un, wn=None, F=None, stream=None) -> float:
    """ok_residual_noalloc: F (written into F when given) and ||F||_2 with no
    context and no workspace (the library's static device scratch)."""
    nrm = C.c_double()
    st = load().ok_residual_noalloc(C.byref(p), _ptr(u), _ptr(w), _ptr(un), _ptr(wn), _ptr(F),
                                    C.byref(nrm), _stream(stream))
    if st:
        raise OkError(st, "ok_residual_noalloc")
    return nrm.value


class Problem:
    """One assembled problem (ok_assemble_mesh) with its torch-owned workspace."""

    def __init__(self, params: Params, device="cuda", stream=None):
        import torch
        self.lib = load()
        self.params = params
        self.device = torch.device(device)
        self.stream = stream
        self.ws_bytes = workspace_bytes(params)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.ctx = C.c_void_p()
        st = self.lib.ok_assemble_mesh(C.byref(params), C.c_void_p(base + off),
                                       C.c_size_t(self.ws_bytes), _stream(stream),
                                       C.byref(self.ctx))
        if st:
            raise OkError(st, "ok_assemble_mesh")
        self.nodes = (params.n + 1) ** params.dim

    # -- helpers -------------------------------------------------------------
    def _check(self, st, what):
        if st:
            msg = self.lib.ok_last_error(self.ctx).decode()
            raise OkError(st, f"{what}: {msg}")

    def field(self, k=1):
        import torch
        return torch.zeros(k * self.nodes, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ok_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls -----------------------------------------------------------
    def residual(self, u, w, un, wn=None, F=None):
        nrm = C.c_double()
        st = self.lib.ok_residual(self.ctx, _ptr(u), _ptr(w), _ptr(un), _ptr(wn), _ptr(F),
                                  C.byref(nrm), _stream(self.stream))
        self._check(st, "ok_residual")
        return nrm.value

    def jacobian_apply(self, u, x, y=None):
        y = self.field(2) if y is None else y
        self._check(self.lib.ok_jacobian_apply(self.ctx, _ptr(u), _ptr(x), _ptr(y),
                                               _stream(self.stream)), "ok_jacobian_apply")
        return y

    def precond_apply(self, u, r, z=None):
        z = self.field(2) if z is None else z
        self._check(self.lib.ok_precond_apply(self.ctx, _ptr(u), _ptr(r), _ptr(z),
                                              _stream(self.stream)), "ok_precond_apply")
        return z

    def cheb_mass(self, r, x=None):
        x = self.field(1) if x is None else x
        self._check(self.lib.ok_cheb_mass(self.ctx, _ptr(r), _ptr(x), _stream(self.stream)),
                    "ok_cheb_mass")
        return x

    def mg_apply(self, b, x=None, cycles=1):
        x = self.field(1) if x is None else x
        self._check(self.lib.ok_mg_apply(self.ctx, _ptr(b), _ptr(x), cycles,
                                         _stream(self.stream)), "ok_mg_apply")
        return x

    def sym_apply(self, u, x, y=None):
        """ok_sym_apply: the symmetric rearranged operator on x = [dw; du]."""
        y = self.field(2) if y is None else y
        self._check(self.lib.ok_sym_apply(self.ctx, _ptr(u), _ptr(x), _ptr(y),
                                          _stream(self.stream)), "ok_sym_apply")
        return y

    def minres(self, u, b, x=None):
        """ok_minres: preconditioned MINRES on the symmetric rearranged system."""
        x = self.field(2) if x is None else x
        its = C.c_int32()
        st = self.lib.ok_minres(self.ctx, _ptr(u), _ptr(b), _ptr(x), C.byref(its),
                                _stream(self.stream))
        return x, its.value, st

    def fgmres(self, u, b, x=None):
        x = self.field(2) if x is None else x
        its = C.c_int32()
        st = self.lib.ok_fgmres(self.ctx, _ptr(u), _ptr(b), _ptr(x), C.byref(its),
                                _stream(self.stream))
        return x, its.value, st

    def newton_step(self, u, w, un, wn=None):
        info = NewtonInfo()
        st = self.lib.ok_newton_step(self.ctx, _ptr(u), _ptr(w), _ptr(un), _ptr(wn),
                                     C.byref(info), _stream(self.stream))
        return info, st

    def timestep(self, u, w, nsteps=1, check=True):
        stats = Stats()
        st = self.lib.ok_timestep(self.ctx, _ptr(u), _ptr(w), nsteps, C.byref(stats),
                                  _stream(self.stream))
        if check:
            self._check(st, "ok_timestep")
        return stats

    def autotune(self):
        n = C.c_int32()
        self._check(self.lib.ok_autotune(self.ctx, _stream(self.stream), C.byref(n)), "ok_autotune")
        return n.value

    def use_graphs(self, enable=True):
        self._check(self.lib.ok_use_graphs(self.ctx, int(bool(enable))), "ok_use_graphs")

    def initial_w(self, u, w=None):
        """w from u by (okb): M w = eps^2 K u + N(u)."""
        w = self.field(1) if w is None else w
        self._check(self.lib.ok_initial_w(self.ctx, _ptr(u), _ptr(w), _stream(self.stream)),
                    "ok_initial_w")
        return w

    def profile_enable(self, *kernel_classes):
        mask = 0
        for k in kernel_classes:
            mask |= 1 << k
        self._check(self.lib.ok_profile_enable(self.ctx, mask), "ok_profile_enable")

    def profile_read(self, kernel_class):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self._check(self.lib.ok_profile_read(self.ctx, kernel_class, C.byref(n), C.byref(ms),
                                             C.byref(by)), "ok_profile_read")
        return n.value, ms.value, by.value


def batch_workspace_bytes(params_list) -> int:
    """ok_batch_workspace_bytes: device bytes of a batch (also one server pool
    when every entry shares a class)."""
    arr = (Params * len(params_list))(*params_list)
    b = C.c_size_t()
    st = load().ok_batch_workspace_bytes(arr, len(params_list), C.byref(b))
    if st:
        raise OkError(st, "ok_batch_workspace_bytes")
    return b.value


class Batch:
    """Many independent problems (ok_batch_*) sharing one torch-owned workspace."""

    def __init__(self, params_list, device="cuda", stream=None):
        import torch
        self.lib = load()
        self.count = len(params_list)
        self.params = (Params * self.count)(*params_list)
        self.device = torch.device(device)
        self.stream = stream
        b = C.c_size_t()
        st = self.lib.ok_batch_workspace_bytes(self.params, self.count, C.byref(b))
        if st:
            raise OkError(st, "ok_batch_workspace_bytes")
        self.ws_bytes = b.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.ctx = C.c_void_p()
        st = self.lib.ok_batch_create(self.params, self.count, C.c_void_p(base + off),
                                      C.c_size_t(self.ws_bytes), _stream(stream),
                                      C.byref(self.ctx))
        if st:
            raise OkError(st, "ok_batch_create")
        self.nodes = [(p.n + 1) ** p.dim for p in params_list]

    def _check(self, st, what):
        if st:
            raise OkError(st, f"{what}: {self.lib.ok_batch_last_error(self.ctx).decode()}")

    def classes(self):
        return self.lib.ok_batch_classes(self.ctx)

    def set_state(self, i, u, w):
        self._check(self.lib.ok_batch_set_state(self.ctx, i, _ptr(u), _ptr(w),
                                                _stream(self.stream)), "ok_batch_set_state")

    def get_state(self, i, u=None, w=None):
        import torch
        if u is None:
            u = torch.empty(self.nodes[i], dtype=torch.float64, device=self.device)
        if w is None:
            w = torch.empty(self.nodes[i], dtype=torch.float64, device=self.device)
        self._check(self.lib.ok_batch_get_state(self.ctx, i, _ptr(u), _ptr(w),
                                                _stream(self.stream)), "ok_batch_get_state")
        return u, w

    def timestep(self, nsteps=1, check=True):
        stats = (Stats * self.count)()
        st = self.lib.ok_batch_timestep(self.ctx, nsteps, stats, _stream(self.stream))
        if check:
            self._check(st, "ok_batch_timestep")
        return list(stats)

    def autotune(self):
        n = C.c_int32()
        self._check(self.lib.ok_batch_autotune(self.ctx, _stream(self.stream), C.byref(n)),
                    "ok_batch_autotune")
        return n.value

    def use_graphs(self, enable=True):
        self._check(self.lib.ok_batch_use_graphs(self.ctx, int(bool(enable))),
                    "ok_batch_use_graphs")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ok_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


OK_OPT_FUSE_CHEB = 1
OK_OPT_FUSE_MG = 2
OK_OPT_ISSUE_AHEAD = 3
OK_OPT_TRACE_RANGES = 4
OK_OPT_GRAM_SCHMIDT = 5
OK_OPT_FUSE_PROLONG = 6


def set_option(option: int, value: int):
    """ok_set_option: process-wide tuning switches (results unchanged)."""
    st = load().ok_set_option(option, value)
    if st:
        raise OkError(st, "ok_set_option")


OK_SHAPE_STENCIL, OK_SHAPE_STENCIL2, OK_SHAPE_CHEB2, OK_SHAPE_MG_PRE, OK_SHAPE_MG_POST = 1, 2, 3, 4, 5
OK_SHAPE_CHEB2_TILE = 6
OK_SHAPE_MG_PRE_TILE, OK_SHAPE_MG_POST_TILE = 7, 8
OK_SHAPE_CHEB2_STRIP, OK_SHAPE_MG_PRE_STRIP, OK_SHAPE_MG_POST_STRIP = 9, 10, 11


def set_launch_shape(dim: int, n: int, kernel: int, precision: int, items: int,
                     threads: int = 256, zchunks: int = 1):
    """ok_set_launch_shape: pin (items > 0) or clear (items = 0) the launch
    shape of one stencil kernel class on one grid."""
    st = load().ok_set_launch_shape(dim, n, kernel, precision, items, threads, zchunks)
    if st:
        raise OkError(st, "ok_set_launch_shape")


def get_launch_shape(dim: int, n: int, kernel: int, precision: int):
    """ok_get_launch_shape: (items, threads, zchunks) of the table entry, all 0
    when the grid uses the built-in default."""
    it, th, zc = C.c_int32(), C.c_int32(), C.c_int32()
    st = load().ok_get_launch_shape(dim, n, kernel, precision, C.byref(it), C.byref(th),
                                    C.byref(zc))
    if st:
        raise OkError(st, "ok_get_launch_shape")
    return it.value, th.value, zc.value


def server_config(**kw) -> ServerConfig:
    c = ServerConfig()
    load().ok_server_default_config(C.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Server:
    """Serving loop (ok_server_*): resident simulations, timestep requests,
    admission by HBM budget, continuous batching on a native worker thread.
    `budget_bytes` is the device memory for slot pools (the resident states
    come on top of it)."""

    def __init__(self, params_list, budget_bytes, config=None, device="cuda"):
        import torch
        self.lib = load()
        self.count = len(params_list)
        self.params = (Params * self.count)(*params_list)
        self.device = torch.device(device)
        b = C.c_size_t()
        st = self.lib.ok_server_state_bytes(self.params, self.count, C.byref(b))
        if st:
            raise OkError(st, "ok_server_state_bytes")
        self.state_bytes = b.value
        self.ws_bytes = self.state_bytes + int(budget_bytes)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.config = config if config is not None else server_config()
        self.ctx = C.c_void_p()
        st = self.lib.ok_server_create(self.params, self.count, C.byref(self.config),
                                       C.c_void_p(base + off), C.c_size_t(self.ws_bytes),
                                       None, C.byref(self.ctx))
        if st:
            raise OkError(st, "ok_server_create")
        self.nodes = [(p.n + 1) ** p.dim for p in params_list]

    def _check(self, st, what):
        if st:
            raise OkError(st, f"{what}: {self.lib.ok_server_last_error(self.ctx).decode()}")

    def set_state(self, i, u, w):
        self._check(self.lib.ok_server_set_state(self.ctx, i, _ptr(u), _ptr(w), _stream(None)),
                    "ok_server_set_state")

    def get_state(self, i):
        import torch
        u = torch.empty(self.nodes[i], dtype=torch.float64, device=self.device)
        w = torch.empty(self.nodes[i], dtype=torch.float64, device=self.device)
        self._check(self.lib.ok_server_get_state(self.ctx, i, _ptr(u), _ptr(w), _stream(None)),
                    "ok_server_get_state")
        return u, w

    def start(self):
        self._check(self.lib.ok_server_start(self.ctx), "ok_server_start")

    def now(self):
        return self.lib.ok_server_now(self.ctx)

    def submit(self, sim, nsteps=1, t_arrival=-1.0):
        t = C.c_int64()
        self._check(self.lib.ok_server_submit(self.ctx, sim, nsteps, float(t_arrival),
                                              C.byref(t)), "ok_server_submit")
        return t.value

    def poll(self, max_results=4096, wait_s=0.0):
        buf = (RequestResult * max_results)()
        n = C.c_int32()
        self._check(self.lib.ok_server_poll(self.ctx, buf, max_results, C.byref(n),
                                            float(wait_s)), "ok_server_poll")
        return [buf[i].as_dict() for i in range(n.value)]

    def stop(self, drain=True):
        self._check(self.lib.ok_server_stop(self.ctx, int(bool(drain))), "ok_server_stop")

    def stats(self):
        s = ServerStats()
        self._check(self.lib.ok_server_get_stats(self.ctx, C.byref(s)), "ok_server_get_stats")
        return s.as_dict()

    def reset_stats(self):
        self._check(self.lib.ok_server_reset_stats(self.ctx), "ok_server_reset_stats")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ok_server_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_string(status: int) -> str:
    return load().ok_error_string(status).decode()
