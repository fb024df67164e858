"""The fused two-iteration Chebyshev kernel (OK_OPT_FUSE_CHEB) against the
one-iteration kernels: bitwise equal results (it rounds every intermediate
to the storage type where the unfused kernels store it), on grids of every
halo class the fused kernel supports, in FP64 and mixed precision."""
import numpy as np
import pytest

from paper_1603_04570_amd.inputs import noise_state, uniform01

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run_both(fn):
    from paper_1603_04570_amd import ok
    out = []
    for fuse in (0, 1):
        ok.set_option(ok.OK_OPT_FUSE_CHEB, fuse)
        try:
            out.append(fn())
        finally:
            ok.set_option(ok.OK_OPT_FUSE_CHEB, 1)
    return out


# (dim, n): 2D rows; 3D halo classes of nn = 17, 65, 129, 257
CASES = [(2, 64), (2, 1024), (3, 16), (3, 64), (3, 128), (3, 256)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("dim,n", CASES)
def test_fused_cheb_mass_bitwise(dim, n, precision):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=dim, n=n, precision=precision)
    P = ok.Problem(p)
    nodes = (n + 1) ** dim
    r = torch.from_numpy(uniform01(11 + n, nodes) - 0.5).cuda()
    print("fused cheb", dim, n, precision, flush=True)

    def once():
        x = torch.empty(nodes, dtype=torch.float64, device="cuda")
        P.cheb_mass(r, x)
        torch.cuda.synchronize()
        return x.cpu().numpy()

    a, b = run_both(once)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dim,n,precision", [(2, 64, 0), (3, 32, 1), (3, 64, 0)])
def test_fused_timestep_bitwise(dim, n, precision):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1,
                          dt=2e-4 if dim == 3 else 1e-4, precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 13)

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    (ua, wa, ia), (ub, wb, ib) = run_both(once)
    assert ia == ib
    assert np.array_equal(ua, ub) and np.array_equal(wa, wb)


def run_both_mg(fn):
    from paper_1603_04570_amd import ok
    out = []
    for fuse in (0, 1):
        ok.set_option(ok.OK_OPT_FUSE_MG, fuse)
        try:
            out.append(fn())
        finally:
            ok.set_option(ok.OK_OPT_FUSE_MG, 1)
    return out


@pytest.mark.parametrize("dim,n,precision", [(2, 64, 0), (2, 256, 1), (3, 32, 0), (3, 64, 1),
                                             (3, 128, 0)])
def test_fused_multigrid_smoothers_bitwise(dim, n, precision):
    """V(2,2) cycles with the fused smoother kernels (pre-smoothing with the
    residual, post-smoothing in one pass) on every level above the coarsest
    reproduce the one-iteration kernels bit for bit over a whole timestep."""
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1,
                          dt=2e-4 if dim == 3 else 1e-4, precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 29)
    print("fused mg", dim, n, precision, flush=True)
    levels = []
    k = n
    while k > 8:  # the levels the smoothers run on (coarsest: 8 elements)
        levels.append(k)
        k //= 2
    for lev_n in levels:  # pin a shape: the levels then use the fused kernels
        for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
            ok.set_launch_shape(dim, lev_n, kern, precision, 1, 256, max(1, (lev_n + 1) // 4))

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    try:
        (ua, wa, ia), (ub, wb, ib) = run_both_mg(once)
    finally:
        for lev_n in levels:
            for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
                ok.set_launch_shape(dim, lev_n, kern, precision, 0)
    assert ia == ib
    assert np.array_equal(ua, ub) and np.array_equal(wa, wb)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("option", ["OK_OPT_ISSUE_AHEAD", "OK_OPT_TRACE_RANGES"])
def test_host_options_bitwise(precision, option):
    """Host-side options change no arithmetic.  FGMRES iterations issued one
    ahead of the host-side stop test (OK_OPT_ISSUE_AHEAD), and ROCTX ranges
    around the solver loops (OK_OPT_TRACE_RANGES), give the same iterates,
    counts and final state as the default, for a single problem and for a
    batch whose instances stop at different iterations."""
    from paper_1603_04570_amd import ok
    from paper_1603_04570_amd.inputs import sweep_instance
    p = ok.default_params(dim=3, n=32, eps=0.02, sigma=100.0, m=0.1, dt=2e-4,
                          precision=precision)
    u0, w0 = noise_state(3, 32, 0.1, 41)

    def solo():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 2)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    specs = [sweep_instance(i, sizes=(32, 64)) for i in range(4)]
    plist = [ok.default_params(dim=s["dim"], n=s["n"], eps=s["eps"], sigma=s["sigma"], m=s["m"],
                               dt=s["dt"], theta=s["theta"], precision=precision) for s in specs]

    def batch():
        Bt = ok.Batch(plist)
        for i, s in enumerate(specs):
            a, b = noise_state(s["dim"], s["n"], s["m"], s["seed"])
            Bt.set_state(i, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        Bt.timestep(1)
        out = []
        for i in range(len(specs)):
            u, w = Bt.get_state(i)
            out.append(np.concatenate([u.cpu().numpy(), w.cpu().numpy()]))
        Bt.close()
        return out

    out = []
    code = getattr(ok, option)
    for value in (0, 1):
        print(option, value, precision, flush=True)
        ok.set_option(code, value)
        try:
            out.append((solo(), batch()))
        finally:
            ok.set_option(code, 0)
    (sa, ba), (sb, bb) = out
    assert sa[2] == sb[2]
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    for x, y in zip(ba, bb):
        assert np.array_equal(x, y)
