"""GPU parity of the symmetric rearranged Newton system and its MINRES solver
(Sec. 2, after eq. (schurapprox)) against the FP64 CPU oracle.

Bars: the symmetric operator elementwise within 1e-13 of the largest entry
(a few FP64 roundings); MINRES solves and timesteps with identical iteration
counts and the fields within 1e-10 relative in the 2-norm, as for FGMRES.
"""
import numpy as np
import pytest

from oracle.okref import Oracle
from paper_1603_04570_amd.inputs import noise_state, uniform01

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CFG1 = dict(eps=0.02, sigma=100.0, m=0.0, dt=1e-4)
CFG2 = dict(eps=0.01, sigma=1000.0, m=0.1, dt=2e-5)
MINRES = 1


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def relnorm(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def make(dim, n, cfg, **kw):
    from paper_1603_04570_amd import ok
    o = Oracle(dim, n, **cfg, linear_solver=MINRES, **kw)
    p = ok.default_params(dim=dim, n=n, **cfg, linear_solver=MINRES, **kw)
    return o, ok.Problem(p)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 64), (2, 128), (3, 8), (3, 16), (3, 32)])
def test_sym_apply(dim, n):
    say("sym_apply", dim, n)
    o, P = make(dim, n, CFG2)
    u, _ = noise_state(dim, n, 0.1, 2)
    x = uniform01(33, 2 * o.nodes) - 0.5
    y = host(P.sym_apply(dev(u), dev(x)))
    assert relmax(y, o.sym_apply(u, x)) < 1e-13


@pytest.mark.parametrize("dim,n,cfg", [(2, 64, CFG1), (2, 32, CFG2), (3, 16, CFG2),
                                       (3, 32, CFG2)])
def test_minres(dim, n, cfg):
    say("minres", dim, n)
    o, P = make(dim, n, cfg)
    u, _ = noise_state(dim, n, cfg["m"], 1)
    b = uniform01(73, 2 * o.nodes) - 0.5
    x_o, its_o, st_o = o.minres(u, b)
    x, its, st = P.minres(dev(u), dev(b))
    say("  its", its, its_o)
    assert st == 0 and st_o == 0 and its == its_o
    assert relnorm(host(x), x_o) < 1e-10


@pytest.mark.parametrize("restart,restarts", [(4, 1), (3, 2), (1, 0)])
def test_minres_iteration_limit(restart, restarts):
    """A limit below the iterations needed: status OK_E_GMRES_MAXIT after
    exactly gmres_restart * (gmres_max_restarts + 1) iterations, and the
    iterate equals the oracle's at that point (an even and two odd limits:
    the device adds the directions to x two iterations at a time, and in an
    odd-numbered last iteration alone)."""
    dim, n = 2, 32
    limit = restart * (restarts + 1)
    o, P = make(dim, n, CFG2, gmres_restart=restart, gmres_max_restarts=restarts)
    u, _ = noise_state(dim, n, 0.1, 1)
    b = uniform01(74, 2 * o.nodes) - 0.5
    x_o, its_o, st_o = o.minres(u, b)
    x, its, st = P.minres(dev(u), dev(b))
    assert st == st_o == -4 and its == its_o == limit
    assert relnorm(host(x), x_o) < 1e-10


def test_minres_zero_rhs():
    dim, n = 2, 16
    o, P = make(dim, n, CFG1)
    u, _ = noise_state(dim, n, 0.0, 1)
    x, its, st = P.minres(dev(u), dev(np.zeros(2 * o.nodes)))
    assert st == 0 and its == 0 and not host(x).any()


@pytest.mark.parametrize("dim,n,cfg,seed", [(2, 64, CFG1, 1), (2, 32, CFG2, 3), (3, 16, CFG2, 2),
                                            (3, 32, CFG2, 2)])
def test_minres_timestep(dim, n, cfg, seed):
    say("minres timestep", dim, n)
    o, P = make(dim, n, cfg)
    u0, w0 = noise_state(dim, n, cfg["m"], seed)
    u_o, w_o, info, st_o = o.timestep(u0, w0, 2)
    u, w = dev(u0), dev(w0)
    stats = P.timestep(u, w, 2)
    say("  its", stats.its(), info.its())
    assert st_o == 0 and stats.status == 0
    assert stats.its() == info.its()
    assert relnorm(host(u), u_o) < 1e-10
    assert relnorm(host(w), w_o) < 1e-10


def test_minres_and_fgmres_classes_in_one_batch():
    """A batch holding FGMRES and MINRES instances of one grid: two classes,
    each instance equal to its own oracle run."""
    from paper_1603_04570_amd import ok
    dim, n = 2, 32
    specs = [(0, CFG1, 1), (MINRES, CFG1, 1), (MINRES, CFG2, 3), (0, CFG2, 3)]
    plist = [ok.default_params(dim=dim, n=n, **cfg, linear_solver=ls) for ls, cfg, _ in specs]
    B = ok.Batch(plist)
    assert B.classes() == 2
    init = []
    for i, (ls, cfg, seed) in enumerate(specs):
        u0, w0 = noise_state(dim, n, cfg["m"], seed)
        init.append((u0, w0))
        B.set_state(i, dev(u0), dev(w0))
    bst = B.timestep(1)
    for i, (ls, cfg, seed) in enumerate(specs):
        o = Oracle(dim, n, **cfg, linear_solver=ls)
        u_o, w_o, info, st_o = o.timestep(*init[i], 1)
        ub, wb = B.get_state(i)
        assert st_o == 0 and bst[i].status == 0
        assert bst[i].its() == info.its(), (i, bst[i].its(), info.its())
        assert relnorm(host(ub), u_o) < 1e-10 and relnorm(host(wb), w_o) < 1e-10


def test_minres_rejects_fgmres_context():
    from paper_1603_04570_amd import ok
    P = ok.Problem(ok.default_params(dim=2, n=16))
    u = dev(np.zeros(17 * 17))
    _, _, st = P.minres(u, dev(np.ones(2 * 17 * 17)))
    assert st == -1


def test_sym_apply_rows_at_full_size():
    """3D 256^3: rows of A_sym at sampled nodes (and the grid's corners) equal
    the oracle's matrix-free Jacobian rows of eq. (newton) rearranged: row 1
    of A_sym [a; b] is row 1 of J [b; a] divided by 1 + dt th sigma, row 2 is
    row 2 of J [b; a]."""
    from oracle.okref import local_jacobian, make_params
    from paper_1603_04570_amd import ok
    from paper_1603_04570_amd.inputs import CONFIGS, sample_nodes
    cfg = CONFIGS["3d256"]
    dim, n = cfg["dim"], cfg["n"]
    say("full-size A_sym rows", dim, n)
    P = ok.Problem(ok.default_params(dim=dim, n=n, eps=cfg["eps"], sigma=cfg["sigma"],
                                     m=cfg["m"], dt=cfg["dt"], theta=cfg["theta"],
                                     linear_solver=MINRES))
    nodes = (n + 1) ** dim
    u0, _ = noise_state(dim, n, cfg["m"], cfg["seed"])
    x = uniform01(92, 2 * nodes) - 0.5
    y = host(P.sym_apply(dev(u0), dev(x)))
    idx = sample_nodes(nodes, 4096, seed=80)
    idx = np.unique(np.concatenate([idx, [0, n, nodes - 1, (n + 1) ** 2 - 1]]))
    prm = make_params(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"])
    j1, j2 = local_jacobian(prm, u0, np.concatenate([x[nodes:], x[:nodes]]), idx)
    sA = 1.0 + cfg["dt"] * cfg["theta"] * cfg["sigma"]
    ref = np.concatenate([j1 / sA, j2])
    got = np.concatenate([y[idx], y[nodes + idx]])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_minres_timestep_at_full_size():
    """3D 256^3, one timestep with MINRES: the oracle's residual rows at
    sampled nodes of the new state are below the Newton tolerance, and it
    agrees with the FGMRES timestep to the Newton tolerance's reach."""
    from oracle.okref import local_residual, make_params
    from paper_1603_04570_amd import ok
    from paper_1603_04570_amd.inputs import CONFIGS, sample_nodes
    cfg = CONFIGS["3d256"]
    dim, n = cfg["dim"], cfg["n"]
    say("full-size MINRES timestep", dim, n)
    kw = dict(dim=dim, n=n, eps=cfg["eps"], sigma=cfg["sigma"], m=cfg["m"], dt=cfg["dt"],
              theta=cfg["theta"])
    u0, w0 = noise_state(dim, n, cfg["m"], cfg["seed"])
    Pm = ok.Problem(ok.default_params(**kw, linear_solver=MINRES))
    u, w = dev(u0), dev(w0)
    st = Pm.timestep(u, w, 1)
    assert st.status == 0
    say("  its", st.its())
    uh, wh = host(u), host(w)
    del Pm
    idx = sample_nodes(uh.size, 4096, seed=81)
    prm = make_params(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"])
    f1, f2 = local_residual(prm, uh, wh, u0, None, idx)
    assert max(np.abs(f1).max(), np.abs(f2).max()) <= 1e-10
    Pf = ok.Problem(ok.default_params(**kw))
    uf, wf = dev(u0), dev(w0)
    assert Pf.timestep(uf, wf, 1).status == 0
    assert relnorm(uh, host(uf)) < 1e-8 and relnorm(wh, host(wf)) < 1e-8
