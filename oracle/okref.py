"""ctypes wrapper over oracle/libokref.so (the plain FP64 CSR oracle).

TEST INFRASTRUCTURE ONLY.  Arrays are float64 numpy vectors in the node order
i + (N+1)*(j + (N+1)*k); two-field vectors are [u-block; w-block].
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libokref.so")
_lib = None

HIST = 256
MAT_M, MAT_K, MAT_ME, MAT_A, MAT_P = 0, 1, 2, 3, 4


class OracleParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32),
                ("eps", C.c_double), ("sigma", C.c_double), ("m", C.c_double),
                ("dt", C.c_double), ("theta", C.c_double),
                ("gmres_restart", C.c_int32), ("gmres_max_restarts", C.c_int32),
                ("gmres_rtol", C.c_double), ("newton_atol", C.c_double),
                ("newton_max_it", C.c_int32), ("cheb_A_its", C.c_int32),
                ("schur_richardson", C.c_int32), ("mg_levels", C.c_int32),
                ("mg_pre", C.c_int32), ("mg_post", C.c_int32), ("mg_cycles", C.c_int32),
                ("linear_solver", C.c_int32)]


class OracleInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_its", C.c_int32),
                ("fgmres_its_total", C.c_int32), ("fgmres_its", C.c_int32 * HIST),
                ("fnorm", C.c_double * (HIST + 1))]

    def its(self):
        return [self.fgmres_its[i] for i in range(min(self.newton_its, HIST))]

    def fnorms(self):
        return [self.fnorm[i] for i in range(min(self.newton_its + 1, HIST + 1))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from .build import build
        build()
    lib = C.CDLL(_LIBPATH)
    P = C.POINTER
    d = P(C.c_double)
    lib.okref_create.argtypes = [P(OracleParams), P(C.c_void_p)]
    lib.okref_destroy.argtypes = [C.c_void_p]
    lib.okref_nodes.argtypes = [C.c_void_p, C.c_int]
    lib.okref_nodes.restype = C.c_int64
    lib.okref_levels.argtypes = [C.c_void_p]
    lib.okref_matrix.argtypes = [C.c_void_p, C.c_int, C.c_int, d, P(C.c_int64), P(C.c_int64),
                                 P(C.c_int64), P(C.c_int64), P(C.c_int32), d]
    lib.okref_nonlinear.argtypes = [C.c_void_p, d, d]
    lib.okref_initial_w.argtypes = [C.c_void_p, d, d]
    lib.okref_cheb_interval.argtypes = [C.c_void_p, C.c_int, C.c_int, d, d]
    lib.okref_residual.argtypes = [C.c_void_p, d, d, d, d, d]
    lib.okref_residual.restype = C.c_double
    lib.okref_jacobian_apply.argtypes = [C.c_void_p, d, d, d]
    lib.okref_cheb_mass.argtypes = [C.c_void_p, d, d]
    lib.okref_mg.argtypes = [C.c_void_p, d, d, C.c_int]
    lib.okref_schur_apply.argtypes = [C.c_void_p, d, d, d]
    lib.okref_precond_apply.argtypes = [C.c_void_p, d, d, d]
    lib.okref_fgmres.argtypes = [C.c_void_p, d, d, d, P(C.c_int32)]
    lib.okref_newton_step.argtypes = [C.c_void_p, d, d, d, d, d, P(C.c_int32)]
    lib.okref_newton_solve.argtypes = [C.c_void_p, d, d, d, d, P(OracleInfo)]
    lib.okref_timestep.argtypes = [C.c_void_p, d, d, C.c_int32, P(OracleInfo)]
    lib.okref_sym_apply.argtypes = [C.c_void_p, d, d, d]
    lib.okref_sym_precond.argtypes = [C.c_void_p, d, d]
    lib.okref_minres.argtypes = [C.c_void_p, d, d, d, P(C.c_int32)]
    lib.okref_local_residual.argtypes = [P(OracleParams), d, d, d, d, P(C.c_int64), C.c_int64, d]
    lib.okref_local_jacobian.argtypes = [P(OracleParams), d, d, P(C.c_int64), C.c_int64, d]
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(dim, n, eps, sigma, m, dt, theta=1.0, gmres_restart=30, gmres_max_restarts=10,
                gmres_rtol=1e-8, newton_atol=1e-10, newton_max_it=25, cheb_A_its=10,
                schur_richardson=1, mg_levels=0, mg_pre=2, mg_post=2, mg_cycles=1,
                linear_solver=0):
    return OracleParams(dim, n, eps, sigma, m, dt, theta, gmres_restart, gmres_max_restarts,
                        gmres_rtol, newton_atol, newton_max_it, cheb_A_its, schur_richardson,
                        mg_levels, mg_pre, mg_post, mg_cycles, linear_solver)


class Oracle:
    """One assembled problem: M, K, the multigrid hierarchy and the coarse factor."""

    def __init__(self, dim, n, eps, sigma, m, dt, theta=1.0, **kw):
        self.lib = _load()
        self.params = make_params(dim, n, eps, sigma, m, dt, theta, **kw)
        self.h = C.c_void_p()
        st = self.lib.okref_create(C.byref(self.params), C.byref(self.h))
        if st != 0:
            raise ValueError(f"okref_create failed: {st}")
        self.dim, self.n = dim, n
        self.nodes = int(self.lib.okref_nodes(self.h, 0))
        self.levels = int(self.lib.okref_levels(self.h))

    def close(self):
        if self.h:
            self.lib.okref_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_nodes(self, level):
        return int(self.lib.okref_nodes(self.h, level))

    def matrix(self, which, level=0, u=None):
        """Return (rowptr, colidx, values, shape) of an assembled operator."""
        nr, nc, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        st = self.lib.okref_matrix(self.h, which, level, _dp(u), C.byref(nr), C.byref(nc),
                                   C.byref(nnz), None, None, None)
        if st:
            raise ValueError(st)
        rp = np.zeros(nr.value + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        v = np.zeros(nnz.value, np.float64)
        self.lib.okref_matrix(self.h, which, level, _dp(u), C.byref(nr), C.byref(nc), C.byref(nnz),
                              rp.ctypes.data_as(C.POINTER(C.c_int64)),
                              ci.ctypes.data_as(C.POINTER(C.c_int32)), _dp(v))
        return rp, ci, v, (nr.value, nc.value)

    def dense(self, which, level=0, u=None):
        rp, ci, v, shape = self.matrix(which, level, u)
        A = np.zeros(shape)
        for r in range(shape[0]):
            A[r, ci[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
        return A

    def scipy(self, which, level=0, u=None):
        import scipy.sparse as sp
        rp, ci, v, shape = self.matrix(which, level, u)
        return sp.csr_matrix((v, ci, rp), shape=shape)

    def nonlinear(self, u):
        out = np.zeros(self.nodes)
        self.lib.okref_nonlinear(self.h, _dp(u), _dp(out))
        return out

    def initial_w(self, u):
        """w from u by (okb): M w = eps^2 K u + N(u) (CG to round-off)."""
        out = np.zeros(self.nodes)
        st = self.lib.okref_initial_w(self.h, _dp(u), _dp(out))
        if st:
            raise RuntimeError(f"okref_initial_w failed: {st}")
        return out

    def cheb_interval(self, level=0, mass=False):
        lo, hi = C.c_double(), C.c_double()
        self.lib.okref_cheb_interval(self.h, level, int(mass), C.byref(lo), C.byref(hi))
        return lo.value, hi.value

    def residual(self, u, w, un, wn=None):
        F = np.zeros(2 * self.nodes)
        nrm = self.lib.okref_residual(self.h, _dp(u), _dp(w), _dp(un), _dp(wn), _dp(F))
        return F, nrm

    def jacobian_apply(self, u, x):
        y = np.zeros(2 * self.nodes)
        self.lib.okref_jacobian_apply(self.h, _dp(u), _dp(x), _dp(y))
        return y

    def cheb_mass(self, r):
        x = np.zeros(self.nodes)
        self.lib.okref_cheb_mass(self.h, _dp(r), _dp(x))
        return x

    def mg(self, b, cycles=1):
        x = np.zeros(self.nodes)
        self.lib.okref_mg(self.h, _dp(b), _dp(x), cycles)
        return x

    def schur_apply(self, u, x):
        y = np.zeros(self.nodes)
        self.lib.okref_schur_apply(self.h, _dp(u), _dp(x), _dp(y))
        return y

    def precond_apply(self, u, r):
        z = np.zeros(2 * self.nodes)
        self.lib.okref_precond_apply(self.h, _dp(u), _dp(r), _dp(z))
        return z

    def fgmres(self, u, b):
        x = np.zeros(2 * self.nodes)
        its = C.c_int32()
        st = self.lib.okref_fgmres(self.h, _dp(u), _dp(b), _dp(x), C.byref(its))
        return x, its.value, st

    def sym_apply(self, u, x):
        """The symmetric rearranged operator on x = [dw; du]."""
        y = np.zeros(2 * self.nodes)
        self.lib.okref_sym_apply(self.h, _dp(u), _dp(x), _dp(y))
        return y

    def sym_precond(self, r):
        z = np.zeros(2 * self.nodes)
        self.lib.okref_sym_precond(self.h, _dp(r), _dp(z))
        return z

    def minres(self, u, b):
        x = np.zeros(2 * self.nodes)
        its = C.c_int32()
        st = self.lib.okref_minres(self.h, _dp(u), _dp(b), _dp(x), C.byref(its))
        return x, its.value, st

    def newton_step(self, u, w, un, wn=None):
        """One Newton iteration in place on copies; returns (u, w, ||F|| before, its, status)."""
        u = np.array(u, np.float64)
        w = np.array(w, np.float64)
        fn = C.c_double()
        its = C.c_int32()
        st = self.lib.okref_newton_step(self.h, _dp(u), _dp(w), _dp(un), _dp(wn), C.byref(fn),
                                        C.byref(its))
        return u, w, fn.value, its.value, st

    def timestep(self, u, w, nsteps=1):
        u = np.array(u, np.float64)
        w = np.array(w, np.float64)
        info = OracleInfo()
        st = self.lib.okref_timestep(self.h, _dp(u), _dp(w), nsteps, C.byref(info))
        return u, w, info, st


def _nodes_arg(nodes):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    return nodes, nodes.ctypes.data_as(C.POINTER(C.c_int64))


def local_residual(params, u, w, un, wn, nodes):
    lib = _load()
    nodes, np_ = _nodes_arg(nodes)
    out = np.zeros(2 * len(nodes))
    st = lib.okref_local_residual(C.byref(params), _dp(u), _dp(w), _dp(un), _dp(wn), np_,
                                  len(nodes), _dp(out))
    if st:
        raise ValueError(st)
    return out[:len(nodes)], out[len(nodes):]


def local_jacobian(params, u, x, nodes):
    lib = _load()
    nodes, np_ = _nodes_arg(nodes)
    out = np.zeros(2 * len(nodes))
    st = lib.okref_local_jacobian(C.byref(params), _dp(u), _dp(x), np_, len(nodes), _dp(out))
    if st:
        raise ValueError(st)
    return out[:len(nodes)], out[len(nodes):]
