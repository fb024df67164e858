"""Batched sweeps: many independent instances in grouped, lockstep launches.

Each instance's result in the batch must equal its solo run bit for bit
(same kernels, same per-instance arithmetic and reduction order), with the
same Newton/FGMRES iteration counts, and the solo runs agree with the oracle.
"""
import numpy as np
import pytest

from oracle.okref import Oracle
from paper_1603_04570_amd.inputs import noise_state, sweep_instance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def params_for(spec, precision):
    from paper_1603_04570_amd import ok
    return ok.default_params(dim=spec["dim"], n=spec["n"], eps=spec["eps"], sigma=spec["sigma"],
                             m=spec["m"], dt=spec["dt"], theta=spec["theta"], precision=precision)


def run_batch_and_solo(specs, precision, steps=1):
    from paper_1603_04570_amd import ok
    plist = [params_for(s, precision) for s in specs]
    B = ok.Batch(plist)
    init = []
    for i, s in enumerate(specs):
        u0, w0 = noise_state(s["dim"], s["n"], s["m"], s["seed"])
        init.append((u0, w0))
        B.set_state(i, torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda())
    bst = B.timestep(steps)
    out = []
    for i, s in enumerate(specs):
        ub, wb = B.get_state(i)
        P = ok.Problem(plist[i])
        u = torch.from_numpy(init[i][0]).cuda()
        w = torch.from_numpy(init[i][1]).cuda()
        sst = P.timestep(u, w, steps)
        out.append((ub.cpu().numpy(), wb.cpu().numpy(), u.cpu().numpy(), w.cpu().numpy(),
                    bst[i], sst))
    return B, out


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_solo_2d_sweep(precision):
    specs = [sweep_instance(i, sizes=(32, 64, 128)) for i in range(8)]
    print("batch 2D sweep", [s["n"] for s in specs], flush=True)
    B, out = run_batch_and_solo(specs, precision)
    assert B.classes() == len({s["n"] for s in specs})
    for (ub, wb, us, ws, bs, ss), s in zip(out, specs):
        assert bs.its() == ss.its(), (s, bs.its(), ss.its())
        assert np.array_equal(ub, us) and np.array_equal(wb, ws), s


def test_batch_mixed_dims_two_steps():
    specs = [sweep_instance(0, sizes=(64,)), dict(dim=3, n=16, eps=0.02, sigma=100.0, m=0.1,
                                                 theta=1.0, dt=2e-4, seed=9),
             sweep_instance(1, sizes=(64,)), dict(dim=3, n=16, eps=0.03, sigma=30.0, m=-0.2,
                                                 theta=1.0, dt=4e-4, seed=10)]
    print("batch mixed dims", flush=True)
    B, out = run_batch_and_solo(specs, 0, steps=2)
    assert B.classes() == 2
    for (ub, wb, us, ws, bs, ss), s in zip(out, specs):
        assert bs.its() == ss.its()
        assert np.array_equal(ub, us) and np.array_equal(wb, ws)


def test_batch_instance_matches_oracle():
    specs = [sweep_instance(i, sizes=(32, 64)) for i in range(3)]
    B, out = run_batch_and_solo(specs, 0)
    for (ub, wb, _, _, bs, _), s in zip(out, specs):
        o = Oracle(2, s["n"], s["eps"], s["sigma"], s["m"], s["dt"], s["theta"])
        u0, w0 = noise_state(2, s["n"], s["m"], s["seed"])
        uo, wo, info, st = o.timestep(u0, w0, 1)
        assert st == 0 and bs.its() == info.its()
        assert np.linalg.norm(ub - uo) / np.linalg.norm(uo) < 1e-10
        assert np.linalg.norm(wb - wo) / np.linalg.norm(wo) < 1e-10


@pytest.mark.parametrize("dim,n,precision", [(2, 64, 0), (3, 16, 1)])
def test_graph_replay_equals_direct_launches(dim, n, precision):
    """Captured FGMRES iterations replay the same kernels: bitwise equal to
    launching them one by one, also after a re-capture for another state
    pointer."""
    from paper_1603_04570_amd import ok
    spec = dict(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1, theta=1.0,
                dt=2e-4 if dim == 3 else 1e-4, seed=21)
    p = params_for(spec, precision)
    u0, w0 = noise_state(dim, n, spec["m"], spec["seed"])
    outs = []
    for graphs in (False, True):
        P = ok.Problem(p)
        if graphs:
            P.use_graphs(True)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 2)
        u2, w2 = u.clone(), w.clone()  # another state pointer: graphs re-captured
        st2 = P.timestep(u2, w2, 1)
        outs.append((u2.cpu().numpy(), w2.cpu().numpy(), st.its() + st2.its()))
    assert outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_batch_without_graphs_equals_with():
    from paper_1603_04570_amd import ok
    specs = [sweep_instance(i, sizes=(32, 64)) for i in range(4)]
    res = []
    for graphs in (True, False):
        plist = [params_for(s, 1) for s in specs]
        B = ok.Batch(plist)
        B.use_graphs(graphs)
        for i, s in enumerate(specs):
            u0, w0 = noise_state(s["dim"], s["n"], s["m"], s["seed"])
            B.set_state(i, torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda())
        st = B.timestep(1)
        res.append([(B.get_state(i)[0].cpu().numpy(), st[i].its()) for i in range(len(specs))])
    for a, b in zip(*res):
        assert a[1] == b[1] and np.array_equal(a[0], b[0])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_tiled_kernels_equal_solo(precision):
    """3D instances of one class (different parameters, so they stop at
    different FGMRES iterations) with the tiled fused Chebyshev pair and the
    tiled fused smoothers pinned on the two finest levels: every instance
    equals its solo run with the built-in kernels, bit for bit."""
    from paper_1603_04570_amd import ok
    specs = [dict(dim=3, n=32, eps=e, sigma=s, m=m, theta=1.0, dt=d, seed=70 + i)
             for i, (e, s, m, d) in enumerate([(0.02, 100.0, 0.1, 2e-4), (0.03, 30.0, -0.2, 4e-4),
                                                (0.025, 300.0, 0.0, 3e-4)])]
    plist = [params_for(s, precision) for s in specs]
    ref = []
    for p, s in zip(plist, specs):  # solo, no pinned shapes
        u0, w0 = noise_state(3, 32, s["m"], s["seed"])
        u, w = torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda()
        st = ok.Problem(p).timestep(u, w, 2)
        ref.append((u.cpu().numpy(), w.cpu().numpy(), st.its()))
    pins = [(ok.OK_SHAPE_CHEB2_TILE, 32, 2, 256, 5)]
    for lev_n in (32, 16):
        pins += [(ok.OK_SHAPE_MG_PRE, lev_n, 1, 256, 1), (ok.OK_SHAPE_MG_POST, lev_n, 1, 256, 1),
                 (ok.OK_SHAPE_MG_PRE_TILE, lev_n, 1, 512, 3),
                 (ok.OK_SHAPE_MG_POST_TILE, lev_n, 2, 256, 4)]
    try:
        for kern, lev_n, items, threads, zch in pins:
            ok.set_launch_shape(3, lev_n, kern, precision, items, threads, zch)
        print("batch tiled", precision, flush=True)
        B = ok.Batch(plist)
        for i, s in enumerate(specs):
            u0, w0 = noise_state(3, 32, s["m"], s["seed"])
            B.set_state(i, torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda())
        bst = B.timestep(2)
        for i in range(len(specs)):
            ub, wb = B.get_state(i)
            assert bst[i].its() == ref[i][2], i
            assert np.array_equal(ub.cpu().numpy(), ref[i][0]), i
            assert np.array_equal(wb.cpu().numpy(), ref[i][1]), i
        assert len({tuple(r[2]) for r in ref}) > 1  # the instances stopped at different iterations
    finally:
        for kern, lev_n, _, _, _ in pins:
            ok.set_launch_shape(3, lev_n, kern, precision, 0)


@pytest.mark.parametrize("precision,cfg", [(0, 1), (0, 4), (1, 2)])
def test_batch_strip_kernels_equal_solo(precision, cfg):
    """3D instances of one class with the strip kernels pinned on the two
    finest levels (the fused Chebyshev pair, pre-smoothing, and in FP64
    post-smoothing with the coarse-grid correction interpolated in the same
    pass): every instance equals its solo run with the built-in kernels, bit
    for bit, with different stopping iterations per instance."""
    from paper_1603_04570_amd import ok
    specs = [dict(dim=3, n=32, eps=e, sigma=s, m=m, theta=1.0, dt=d, seed=80 + i)
             for i, (e, s, m, d) in enumerate([(0.02, 100.0, 0.1, 2e-4), (0.03, 30.0, -0.2, 4e-4),
                                                (0.025, 300.0, 0.0, 3e-4)])]
    plist = [params_for(s, precision) for s in specs]
    ref = []
    for p, s in zip(plist, specs):  # solo, no pinned shapes
        u0, w0 = noise_state(3, 32, s["m"], s["seed"])
        u, w = torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda()
        st = ok.Problem(p).timestep(u, w, 2)
        ref.append((u.cpu().numpy(), w.cpu().numpy(), st.its()))
    pins = [(ok.OK_SHAPE_CHEB2_STRIP, 32, cfg, 256, 3)]
    for lev_n in (32, 16):
        pins += [(ok.OK_SHAPE_MG_PRE, lev_n, 1, 256, 1), (ok.OK_SHAPE_MG_POST, lev_n, 1, 256, 1),
                 (ok.OK_SHAPE_MG_PRE_STRIP, lev_n, cfg, 256, 2),
                 (ok.OK_SHAPE_MG_POST_STRIP, lev_n, cfg, 256, 5)]
    try:
        for kern, lev_n, items, threads, zch in pins:
            ok.set_launch_shape(3, lev_n, kern, precision, items, threads, zch)
        print("batch strips", precision, cfg, flush=True)
        B = ok.Batch(plist)
        for i, s in enumerate(specs):
            u0, w0 = noise_state(3, 32, s["m"], s["seed"])
            B.set_state(i, torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda())
        bst = B.timestep(2)
        for i in range(len(specs)):
            ub, wb = B.get_state(i)
            assert bst[i].its() == ref[i][2], i
            assert np.array_equal(ub.cpu().numpy(), ref[i][0]), i
            assert np.array_equal(wb.cpu().numpy(), ref[i][1]), i
        assert len({tuple(r[2]) for r in ref}) > 1
    finally:
        for kern, lev_n, _, _, _ in pins:
            ok.set_launch_shape(3, lev_n, kern, precision, 0)
