"""The paper's own workload on Q1 (Sec. 4): theta = 1/2, m = 0.4, eps = 0.02,
sigma = 100, dt = eps^2, cosine initial condition, w0 from (okb), and the
paper's solver preset (two Richardson iterations of S~^-1, five V-cycles per
S^^-1), on meshes N = 25 * 2^k whose multigrid coarsens to 25 elements per
direction (a 26^3 coarse grid, solved axis by axis on the GPU and by CG in the
oracle).  Against the oracle: w0 to 1e-12, the V-cycle to 1e-12, one
timestep to 1e-10 with identical iteration counts, also with the autotuner's
launch shapes and fused-kernel choices on the 3D N = 50 hierarchy."""
import numpy as np
import pytest

from oracle.okref import Oracle
from paper_1603_04570_amd.inputs import cosine_state, uniform01

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PAPER = dict(eps=0.02, sigma=100.0, m=0.4, dt=4e-4, theta=0.5)
PRESET = dict(schur_richardson=2, mg_cycles=5)


def problem(dim, n, **kw):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=dim, n=n, **PAPER, **kw)
    return ok.Problem(p), Oracle(dim, n, PAPER["eps"], PAPER["sigma"], PAPER["m"], PAPER["dt"],
                                 PAPER["theta"], **kw)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dim,n", [(2, 64), (2, 100), (3, 16), (3, 50)])
def test_initial_w_matches_oracle(dim, n):
    print("initial w", dim, n, flush=True)
    P, o = problem(dim, n)
    u0, _ = cosine_state(dim, n, PAPER["m"])
    w = P.initial_w(torch.from_numpy(u0).cuda()).cpu().numpy()
    assert rel(w, o.initial_w(u0)) < 1e-12


@pytest.mark.parametrize("dim,n", [(2, 100), (3, 50)])
def test_multigrid_large_coarse_grid(dim, n):
    print("mg coarse 26^d", dim, n, flush=True)
    P, o = problem(dim, n)
    b = uniform01(23, o.nodes) - 0.5
    for cycles in (1, 2):
        x = P.mg_apply(torch.from_numpy(b).cuda(), cycles=cycles).cpu().numpy()
        assert np.abs(x - o.mg(b, cycles)).max() / np.abs(x).max() < 1e-12


@pytest.mark.parametrize("dim,n,tuned", [(2, 100, False), (3, 50, False), (3, 50, True)])
def test_paper_timestep_matches_oracle(dim, n, tuned):
    print("paper timestep", dim, n, "autotuned" if tuned else "", flush=True)
    P, o = problem(dim, n, **PRESET)
    if tuned:  # the launch shapes and fused kernels bench --config paper runs
        P.autotune()
    u0, _ = cosine_state(dim, n, PAPER["m"])
    ud = torch.from_numpy(u0).cuda()
    wd = P.initial_w(ud)
    w0 = o.initial_w(u0)
    st = P.timestep(ud, wd, 1)
    uo, wo, info, sto = o.timestep(u0, w0, 1)
    assert st.status == 0 and sto == 0
    assert st.its() == info.its()
    assert rel(ud.cpu().numpy(), uo) < 1e-10
    assert rel(wd.cpu().numpy(), wo) < 1e-10
