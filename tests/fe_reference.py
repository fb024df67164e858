"""Independent closed forms and brute-force evaluations used to pin the oracle.

Nothing here is shared with the oracle or the GPU library: the matrices come
from Kronecker products of the 1D Q1 matrices, the nonlinear integrals from a
5-point Gauss rule on each element (more points than the 3 the oracle uses),
and the exact shifted-Laplacian solve from the DCT-I eigenbasis.
"""
import numpy as np


def m1(n):
    """1D Q1 mass on n elements of [0,1]: (h/6) tridiag(1,4,1), ends 2."""
    h = 1.0 / n
    A = np.zeros((n + 1, n + 1))
    for e in range(n):
        A[e:e + 2, e:e + 2] += (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    return A


def k1(n):
    """1D Q1 stiffness: (1/h) tridiag(-1,2,-1), ends 1."""
    h = 1.0 / n
    A = np.zeros((n + 1, n + 1))
    for e in range(n):
        A[e:e + 2, e:e + 2] += (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return A


def kron_list(mats):
    """mats ordered slowest (z) to fastest (x) index."""
    out = mats[0]
    for a in mats[1:]:
        out = np.kron(out, a)
    return out


def mass(dim, n):
    return kron_list([m1(n)] * dim)


def stiffness(dim, n):
    out = 0
    for d in range(dim):
        out = out + kron_list([k1(n) if e == d else m1(n) for e in range(dim)])
    return out


def prolongation_1d(nc):
    n = 2 * nc
    P = np.zeros((n + 1, nc + 1))
    for i in range(n + 1):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, (i - 1) // 2] = 0.5
            P[i, (i + 1) // 2] = 0.5
    return P


def coords(dim, n):
    """Node coordinates (nodes x dim), x fastest."""
    t = np.linspace(0.0, 1.0, n + 1)
    grids = np.meshgrid(*([t] * dim), indexing="ij")   # axis 0 slowest
    # grids[0] varies along axis 0 (slowest == last coordinate)
    cols = [g.ravel() for g in grids]
    return np.stack(cols[::-1], axis=1)   # column 0 = x (fastest)


def brute_element_integrals(dim, n, u, npts=5):
    """M_E(u) (dense) and N(u) by npts-point Gauss-Legendre per direction on
    every element, with u the Q1 interpolant of the nodal values."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    h = 1.0 / n
    nn = n + 1
    nodes = nn ** dim
    ME = np.zeros((nodes, nodes))
    NV = np.zeros(nodes)
    nloc = 2 ** dim
    # quadrature points of the reference element
    pts = np.array(np.meshgrid(*([np.arange(npts)] * dim), indexing="ij")).reshape(dim, -1).T
    phis = np.zeros((len(pts), nloc))
    wts = np.zeros(len(pts))
    for q, idx in enumerate(pts):
        xi = xg[idx]
        wts[q] = np.prod(wg[idx]) * h ** dim
        for a in range(nloc):
            bits = [(a >> d) & 1 for d in range(dim)]
            phis[q, a] = np.prod([xi[d] if bits[d] else 1.0 - xi[d] for d in range(dim)])
    ranges = [range(n)] * dim
    for e in np.ndindex(*([n] * dim)):
        corner = e[::-1]  # (ei, ej[, ek])
        gidx = []
        for a in range(nloc):
            c = [corner[d] + ((a >> d) & 1) for d in range(dim)]
            g = c[0] + nn * c[1] + (nn * nn * c[2] if dim == 3 else 0)
            gidx.append(g)
        gidx = np.array(gidx)
        uq = phis @ u[gidx]
        coef = wts * (3.0 * uq ** 2 - 1.0)
        ME[np.ix_(gidx, gidx)] += (phis * coef[:, None]).T @ phis
        NV[gidx] += phis.T @ (wts * (uq ** 3 - uq))
    del ranges
    return ME, NV


def dct_matrix(n):
    j = np.arange(n + 1)
    return np.cos(np.pi * np.outer(j, j) / n)   # V[j, k] = cos(k pi j / n)


def dct_mode(dim, n, ks):
    """prod_d cos(k_d pi j_d / n), x fastest; ks = (kx, ky[, kz])."""
    V = dct_matrix(n)
    vecs = [V[:, k] for k in ks]
    return kron_list(vecs[::-1])


def gen_eig_1d(n, k):
    """Generalised (K1, M1) eigenvalue of the DCT-I mode k."""
    h = 1.0 / n
    c = np.cos(np.pi * k / n)
    return (6.0 / h ** 2) * (1.0 - c) / (2.0 + c)


def fast_diag_solve(dim, n, alpha, b):
    """Exact (M + alpha K)^-1 b via the DCT-I eigenbasis:
    x = V (Lambda Gamma)^-1 V^T b with V the tensor cosine matrix."""
    h = 1.0 / n
    V = dct_matrix(n)
    c = np.cos(np.pi * np.arange(n + 1) / n)
    mu = (h / 3.0) * (2.0 + c)
    kap = (2.0 / h) * (1.0 - c)
    gam = np.full(n + 1, n / 2.0)
    gam[0] = gam[-1] = n
    nn = n + 1
    X = b.reshape((nn,) * dim)
    # apply V^T along every axis
    for ax in range(dim):
        X = np.moveaxis(np.tensordot(V.T, X, axes=([1], [ax])), 0, ax)
    grids = np.meshgrid(*([np.arange(nn)] * dim), indexing="ij")
    lam = np.ones((nn,) * dim)
    for g in grids:
        lam = lam * mu[g]
    st = np.zeros((nn,) * dim)
    for d, gd in enumerate(grids):
        t = kap[gd]
        for e, ge in enumerate(grids):
            if e != d:
                t = t * mu[ge]
        st = st + t
    gm = np.ones((nn,) * dim)
    for g in grids:
        gm = gm * gam[g]
    X = X / ((lam + alpha * st) * gm)
    for ax in range(dim):
        X = np.moveaxis(np.tensordot(V, X, axes=([1], [ax])), 0, ax)
    return X.ravel()


def cheb_T(k, x):
    """Chebyshev polynomial of the first kind (scalar x, any real)."""
    if abs(x) <= 1.0:
        return np.cos(k * np.arccos(x))
    return np.sign(x) ** k * np.cosh(k * np.arccosh(abs(x)))
