"""Launch shapes of the streaming stencil kernels (ok_set_launch_shape).

Every node's arithmetic is the same whatever the shape, so results must be
bitwise equal for every item count per thread, for 256- and 512-thread
fused blocks, for row-run and rectangular-tile blocks of the fused
Chebyshev pair, and for every split of the planes into z-ranges (one range,
uneven ranges, one plane per range).
"""
import numpy as np
import pytest

from paper_1603_04570_amd.inputs import noise_state, uniform01

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


STRIP_CFGS = (1, 2, 3, 4, 5)  # window configurations of the strip kernels (32x32/4, 32x16/2, 64x16/4, 32x24/3, 64x12/3)


def cheb_mass(P, r, nodes):
    x = torch.empty(nodes, dtype=torch.float64, device="cuda")
    P.cheb_mass(r, x)
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("dim,n", [(2, 256), (3, 64), (3, 100), (3, 128), (3, 256)])
def test_fused_chebyshev_shapes_bitwise(dim, n, precision):
    from paper_1603_04570_amd import ok
    p = ok.default_params(dim=dim, n=n, precision=precision)
    P = ok.Problem(p)
    nodes = (n + 1) ** dim
    r = torch.from_numpy(uniform01(23 + n, nodes) - 0.5).cuda()
    ok.set_option(ok.OK_OPT_FUSE_CHEB, 0)
    try:
        ref = cheb_mass(P, r, nodes)
    finally:
        ok.set_option(ok.OK_OPT_FUSE_CHEB, 1)
    shapes = [(1, 256), (2, 256)] + ([(1, 512), (2, 512)] if dim == 3 else [])
    try:
        for items, threads in shapes:
            for zch in (1, 3, 7, n + 1):
                print("fused shape", dim, n, precision, items, threads, zch, flush=True)
                ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2, precision, items, threads, zch)
                assert np.array_equal(cheb_mass(P, r, nodes), ref), (items, threads, zch)
    finally:
        ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2, precision, 0)
    if dim == 3:  # the same pairs on rectangular in-plane tiles
        try:
            for items, threads in [(1, 256), (2, 256), (1, 512), (2, 512)]:
                for zch in (1, 3, 7, n + 1):
                    print("tiled shape", n, precision, items, threads, zch, flush=True)
                    ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2_TILE, precision, items, threads,
                                        zch)
                    assert np.array_equal(cheb_mass(P, r, nodes), ref), (items, threads, zch)
        finally:
            ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2_TILE, precision, 0)
        try:  # and on overlapping windows with a column strip per thread
            for cfg in STRIP_CFGS:
                for zch in (1, 3, 7, n + 1):
                    print("strip shape", n, precision, cfg, zch, flush=True)
                    ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2_STRIP, precision, cfg, 256, zch)
                    assert np.array_equal(cheb_mass(P, r, nodes), ref), (cfg, zch)
        finally:
            ok.set_launch_shape(dim, n, ok.OK_SHAPE_CHEB2_STRIP, precision, 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_stencil_shapes_timestep_bitwise(precision):
    """A 3D 32^3 timestep (every stencil kernel of the path) with the one- and
    two-field stencil shapes of the two finest levels pinned to each item
    count and several z-splits."""
    from paper_1603_04570_amd import ok
    dim, n = 3, 32
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1, dt=2e-4,
                          precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 17)

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    ref = once()
    try:
        for items, threads, zch in [(1, 256, 1), (2, 256, 4), (4, 256, 33), (8, 256, 5),
                                    (8, 256, 1), (1, 512, 3), (2, 512, 1), (4, 512, 33)]:
            print("stencil shape", precision, items, threads, zch, flush=True)
            for lev_n in (n, n // 2):
                for word in (0, 1):  # FP64 and FP32 storage entries
                    ok.set_launch_shape(dim, lev_n, ok.OK_SHAPE_STENCIL, word, items, threads,
                                        min(zch, lev_n + 1))
                    ok.set_launch_shape(dim, lev_n, ok.OK_SHAPE_STENCIL2, word, min(items, 4),
                                        256, min(zch, lev_n + 1))
            got = once()
            assert got[2] == ref[2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), \
                (items, threads, zch)
    finally:
        for lev_n in (n, n // 2):
            for word in (0, 1):
                ok.set_launch_shape(dim, lev_n, ok.OK_SHAPE_STENCIL, word, 0)
                ok.set_launch_shape(dim, lev_n, ok.OK_SHAPE_STENCIL2, word, 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_mg_smoother_shapes_bitwise(precision):
    """The fused multigrid smoothers of the two finest levels of a 3D 64^3
    timestep pinned to every item count and thread count and several
    z-splits: results equal the one-iteration kernels bit for bit."""
    from paper_1603_04570_amd import ok
    dim, n = 3, 64
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1, dt=2e-4,
                          precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 31)

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    ok.set_option(ok.OK_OPT_FUSE_MG, 0)
    try:
        ref = once()
    finally:
        ok.set_option(ok.OK_OPT_FUSE_MG, 1)
    try:
        for items, threads, zch in [(1, 256, 1), (2, 256, 5), (1, 512, 65), (2, 512, 3)]:
            print("mg shape", precision, items, threads, zch, flush=True)
            for lev_n in (n, n // 2):
                for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
                    ok.set_launch_shape(dim, lev_n, kern, precision, items, threads,
                                        min(zch, lev_n + 1))
            got = once()
            assert got[2] == ref[2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), \
                (items, threads, zch)
    finally:
        for lev_n in (n, n // 2):
            for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
                ok.set_launch_shape(dim, lev_n, kern, precision, 0)


@pytest.mark.parametrize("n", [64, 100])
@pytest.mark.parametrize("precision", [0, 1])
def test_mg_smoother_tile_shapes_bitwise(precision, n):
    """The fused multigrid smoothers on in-plane tiles (3D), pinned on the two
    finest levels of a 64^3 timestep and of the paper's N = 100 mesh (levels
    100 and 50) for every thread and node count and several z-splits: results
    equal the one-iteration kernels bit for bit."""
    from paper_1603_04570_amd import ok
    dim = 3
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1, dt=2e-4,
                          precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 37)

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    ok.set_option(ok.OK_OPT_FUSE_MG, 0)
    try:
        ref = once()
    finally:
        ok.set_option(ok.OK_OPT_FUSE_MG, 1)
    kinds = (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST, ok.OK_SHAPE_MG_PRE_TILE,
             ok.OK_SHAPE_MG_POST_TILE)
    try:
        for items, threads, zch in [(1, 256, 1), (2, 256, 5), (1, 512, 65), (2, 512, 3)]:
            print("mg tile shape", precision, items, threads, zch, flush=True)
            for lev_n in (n, n // 2):
                # a row-run entry switches the fused smoothers on; the tile entry selects tiles
                for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
                    ok.set_launch_shape(dim, lev_n, kern, precision, 1, 256, 1)
                for kern in (ok.OK_SHAPE_MG_PRE_TILE, ok.OK_SHAPE_MG_POST_TILE):
                    ok.set_launch_shape(dim, lev_n, kern, precision, items, threads,
                                        min(zch, lev_n + 1))
            got = once()
            assert got[2] == ref[2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), \
                (items, threads, zch)
    finally:
        for lev_n in (n, n // 2):
            for kern in kinds:
                ok.set_launch_shape(dim, lev_n, kern, precision, 0)


@pytest.mark.parametrize("n", [64, 100])
@pytest.mark.parametrize("precision", [0, 1])
def test_mg_smoother_strip_shapes_bitwise(precision, n):
    """The fused multigrid smoothers on overlapping windows with a column strip
    per thread (3D), pinned on the two finest levels of a 64^3 timestep and of
    the N = 100 mesh for every window configuration and several z-splits, with
    the prolongation folded into the post-smoother (the default in FP64) and in
    a pass of its own: results equal the one-iteration kernels bit for bit."""
    from paper_1603_04570_amd import ok
    dim = 3
    p = ok.default_params(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.1, dt=2e-4,
                          precision=precision)
    u0, w0 = noise_state(dim, n, 0.1, 41)

    def once():
        P = ok.Problem(p)
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        st = P.timestep(u, w, 1)
        return u.cpu().numpy(), w.cpu().numpy(), st.its()

    ok.set_option(ok.OK_OPT_FUSE_MG, 0)
    try:
        ref = once()
    finally:
        ok.set_option(ok.OK_OPT_FUSE_MG, 1)
    kinds = (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST, ok.OK_SHAPE_MG_PRE_STRIP,
             ok.OK_SHAPE_MG_POST_STRIP)
    try:
        for cfg, zch, fold in [(1, 1, 1), (2, 5, 1), (3, 3, 1), (1, 65, 1), (2, 2, 1),
                               (3, 101, 1), (4, 7, 1), (5, 2, 1), (1, 5, 0), (4, 3, 0)]:
            print("mg strip shape", precision, n, cfg, zch, fold, flush=True)
            ok.set_option(ok.OK_OPT_FUSE_PROLONG, fold)
            for lev_n in (n, n // 2):
                # a row-run entry switches the fused smoothers on; the strip entry selects strips
                for kern in (ok.OK_SHAPE_MG_PRE, ok.OK_SHAPE_MG_POST):
                    ok.set_launch_shape(dim, lev_n, kern, precision, 1, 256, 1)
                for kern in (ok.OK_SHAPE_MG_PRE_STRIP, ok.OK_SHAPE_MG_POST_STRIP):
                    ok.set_launch_shape(dim, lev_n, kern, precision, cfg, 256,
                                        min(zch, lev_n + 1))
            got = once()
            assert got[2] == ref[2]
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), \
                (cfg, zch, fold)
    finally:
        ok.set_option(ok.OK_OPT_FUSE_PROLONG, 1)
        for lev_n in (n, n // 2):
            for kern in kinds:
                ok.set_launch_shape(dim, lev_n, kern, precision, 0)
