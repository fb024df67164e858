"""Host emulation of the index arithmetic of every z-streaming stencil kernel
(no GPU): for every launch shape the autotuner or ok_set_launch_shape can
choose, on 2D and 3D grids of N in {8, 16, 25 * 2^k, 32 ... 256} (3D) and
up to 2048 (2D), every global load and store and every LDS access lies inside
its array, the prefetch slots cover what each plane's staging needs, and
every output node is written exactly once.

Each emulation restates, in numpy, the block/thread/trip index computations
of one kernel family of paper_1603_04570_amd/csrc/k_stencil_impl.h and
k_strip2.h (block -> (plane chunk or tile, z-range), thread -> in-plane
positions, clamped prefetch addresses, LDS positions), separately for the
in-plane part (the same for every plane) and the z part (the planes each
z-range touches).  A change to a kernel's indexing must be mirrored here."""
import numpy as np
import pytest

GRIDS_3D = [8, 16, 25, 32, 50, 64, 100, 128, 200, 256]
GRIDS_2D = [8, 16, 64, 128, 256, 512, 1024, 2048]


def z_candidates(nn, per_plane_blocks):
    """The z-range counts the autotuner tries (zchunk_candidates_n), plus the
    extremes ok_set_launch_shape accepts."""
    v = [(nn + zc - 1) // zc for zc in (4, 8, 16, 32)]
    v += [t // per_plane_blocks for t in (512, 1024, 2048, 3072, 4096, 6144)]
    v += [1, 3, nn]
    return sorted({max(1, min(z, nn)) for z in v})


def zranges(nn, nzc):
    return [(z * nn // nzc, (z + 1) * nn // nzc) for z in range(nzc)]


def check_planes(N, planes):
    planes = np.asarray(planes)
    assert planes.min() >= 0 and planes.max() <= N, (planes.min(), planes.max(), N)


# ---------------------------------------------------------------- k_stencil
def stencil_shapes(dim, nf):
    """(items, threads) pairs of stencil_shape_ok."""
    out = []
    for items in (1, 2, 4, 8):
        if items == 8 and nf != 1:
            continue
        out.append((items, 256))
    if dim == 3 and nf == 1:
        out += [(1, 512), (2, 512), (4, 512)]
    return out


def emulate_stencil(dim, N, nf, items, NT):
    nn = N + 1
    plane = nn * nn if dim == 3 else nn
    halo = nn + 1 if dim == 3 else 1
    chunk = NT * items
    nchunks = (plane + chunk - 1) // chunk
    ldsn = chunk + 2 * halo
    extra = (ldsn - chunk + NT - 1) // NT
    hx = 3 if extra <= 3 else (5 if extra <= 5 else (9 if extra <= 9 else 17))
    if extra > 17 or nf * ldsn * 8 > 65536 or (dim == 3 and hx > 5):
        return None  # the launcher rejects this shape (hipErrorInvalidValue)
    F = items + hx
    assert F * NT >= ldsn  # every staged position has a prefetch slot
    written = np.zeros(plane, np.int64)
    tid = np.arange(NT)
    for c in range(nchunks):
        s0 = c * chunk
        for k in range(F):
            gq = s0 - halo + tid + NT * k
            gc = np.clip(gq, 0, plane - 1)
            assert gc.min() >= 0 and gc.max() < plane
        for p in range(items):
            q = s0 + tid + NT * p
            valid = q < plane
            L = tid + NT * p + halo
            lo = L - (nn + 1 if dim == 3 else 1)
            hi = L + (nn + 1 if dim == 3 else 1)
            assert lo.min() >= 0 and hi.max() < ldsn
            np.add.at(written, q[valid], 1)
            qc = np.where(q < plane, q, plane - 1)  # epilogue loads: clamped
            assert qc.max() < plane
    assert (written == 1).all()
    return nchunks


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("nf", [1, 2])
def test_stencil_streaming_kernel_indices(dim, nf):
    for N in (GRIDS_3D if dim == 3 else GRIDS_2D):
        nn = N + 1
        for items, NT in stencil_shapes(dim, nf):
            nch = emulate_stencil(dim, N, nf, items, NT)
            if nch is None:
                continue
            for nzc in z_candidates(nn, nch):
                for z0, z1 in zranges(nn, nzc):
                    zlast = min(z1, N)
                    planes = [max(z0 - 1, 0)] + [min(pz + 1, zlast) for pz in range(z0 - 1, z1 + 1)]
                    check_planes(N, planes)
                    check_planes(N, [max(o, z0) for o in range(z0 - 1, z1)])  # epilogue loads


# ---------------------------------------------------------- k_cheb2 / k_mg2
def emulate_rowrun_fused(dim, N, items, NT, word):
    """k_cheb2 and k_mg2: a run of NT*items nodes per block, one- and two-row
    halos; returns the number of runs per plane, or None where the launcher
    rejects the shape."""
    nn = N + 1
    plane = nn * nn if dim == 3 else nn
    H = nn + 1 if dim == 3 else 1
    CH = NT * items
    ex1 = (2 * H + NT - 1) // NT
    exa = (4 * H + NT - 1) // NT
    combos = {(1, 1)} if dim == 2 else {(1, 1), (1, 2), (2, 3), (3, 5), (5, 9)}
    if (ex1, exa) not in combos:
        return None
    lds_words = CH + 4 * H + CH + 2 * H + 4 * CH
    if lds_words * word > 65536:
        return None
    P1, FA = items + ex1, items + exa
    E1, E2 = CH + 2 * H, CH + 4 * H
    assert P1 * NT >= E1 and FA * NT >= E2
    nchunks = (plane + CH - 1) // CH
    ystep = nn if dim == 3 else 0
    tid = np.arange(NT)
    written = np.zeros(plane, np.int64)
    for c in range(nchunks):
        s0 = c * CH
        for k in range(FA):  # two-row-halo staging of the stenciled input
            gq = s0 - 2 * H + tid + NT * k
            assert np.clip(gq, 0, plane - 1).max() < plane
            t = tid + NT * k
            assert t[t < E2].max(initial=0) < E2
        for q in range(P1):  # stage 1 on the run plus a one-row halo
            e = tid + NT * q
            use = e < E1
            L = e + H  # position in the two-row-halo buffer
            assert (L[use] - ystep - 1).min(initial=0) >= 0
            assert (L[use] + ystep + 1).max(initial=0) < E2
            gq = np.clip(s0 - H + e, 0, plane - 1)
            assert gq.max() < plane
            cidx = e - H
            inrun = (cidx >= 0) & (cidx < CH) & use
            assert cidx[inrun].max(initial=0) < CH
        for p in range(items):  # stage 2 on the run
            cpos = tid + NT * p
            gq = s0 + cpos
            L = cpos + H
            assert (L - ystep - 1).min() >= 0 and (L + ystep + 1).max() < E1
            ok = gq < plane
            np.add.at(written, gq[ok], 1)
    assert (written == 1).all()
    return nchunks


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("word", [4, 8])
def test_rowrun_fused_kernel_indices(dim, word):
    for N in (GRIDS_3D if dim == 3 else GRIDS_2D):
        nn = N + 1
        for items in (1, 2):
            for NT in ((256, 512) if dim == 3 else (256,)):
                nch = emulate_rowrun_fused(dim, N, items, NT, word)
                if nch is None:
                    continue
                for nzc in z_candidates(nn, nch):
                    for z0, z1 in zranges(nn, nzc):
                        zlast = min(z1 + 1, N)
                        a = [max(z0 - 2, 0)] + [max(min(pz + 1, zlast), 0)
                                                for pz in range(z0 - 2, z1 + 2)]
                        pw = [max(z0 - 1, 0)] + [min(max(pz, 0), N) for pz in range(z0 - 2, z1 + 2)]
                        check_planes(N, a)
                        check_planes(N, pw)
                        outs = [pz - 2 for pz in range(z0 - 2, z1 + 2) if z0 <= pz - 2 < z1]
                        assert outs == list(range(z0, z1))


# -------------------------------------------------------- k_cheb2t / k_mg2t
def tile_geom(N, threads, items):
    """cheb2_tile_geom: the tiling of the N+1 columns with the fewest tiles
    per plane whose rings fit items+1 slots per thread and whose LDS fits."""
    nn = N + 1
    cap, slots = threads * items, threads * (items + 1)
    best = None
    for ntx in range(1, min(32, nn) + 1):
        tx = (nn + ntx - 1) // ntx
        ty = min(nn, cap // tx)
        while ty >= 1 and (tx + 4) * (ty + 4) > slots:
            ty -= 1
        if ty < 1:
            continue
        lds = ((tx + 4) * (ty + 4) + (tx + 2) * (ty + 2) + 4 * tx * ty) * 8
        if lds > 65536:
            continue
        ntxr, nty = (nn + tx - 1) // tx, (nn + ty - 1) // ty
        if best is None or ntxr * nty < best[4]:
            best = (tx, ty, ntxr, nty, ntxr * nty)
    return best


def emulate_tiled(N, items, NT):
    nn = N + 1
    tg = tile_geom(N, NT, items)
    if tg is None:
        return None
    TX, TY, ntx, nty, _ = tg
    P1 = items + 1
    WA, WB = TX + 4, TX + 2
    EA, E1, CH = WA * (TY + 4), WB * (TY + 2), TX * TY
    assert TX * TY <= NT * items and EA <= NT * P1 and E1 <= NT * P1
    lds_words = EA + E1 + 4 * CH
    tid = np.arange(NT)
    written = np.zeros(nn * nn, np.int64)
    for tile in range(ntx * nty):
        x0, y0 = (tile % ntx) * TX, (tile // ntx) * TY
        for k in range(P1):  # input staging with a two-node ring
            t = tid + NT * k
            ra, ca = t // WA, t % WA
            gy, gx = y0 - 2 + ra, x0 - 2 + ca
            oa = np.clip(gy, 0, N) * nn + np.clip(gx, 0, N)
            assert oa.max() < nn * nn and oa.min() >= 0
        for q in range(P1):  # stage 1 on the tile plus a one-node ring
            e = tid + NT * q
            use = e < E1
            rb, cb = e // WB, e % WB
            l1 = np.where(use, (rb + 1) * WA + cb + 1, WA + 1)
            assert (l1 - WA - 1).min() >= 0 and (l1 + WA + 1).max() < EA
            gy, gx = np.clip(y0 - 1 + rb, 0, N), np.clip(x0 - 1 + cb, 0, N)
            ci, cj = gx - x0, gy - y0
            own = use & (ci >= 0) & (ci < TX) & (cj >= 0) & (cj < TY)
            c = cj * TX + ci
            assert c[own].max(initial=0) < CH and c[own].min(initial=0) >= 0
            assert e[use].max(initial=0) < E1
        for p in range(items):  # stage 2 on the tile
            c = tid + NT * p
            a, bb = c // TX, c % TX
            gy, gx = y0 + a, x0 + bb
            valid = (c < CH) & (gy <= N) & (gx <= N)
            l2 = np.where(c < CH, (a + 1) * WB + bb + 1, WB + 1)
            assert (l2 - WB - 1).min() >= 0 and (l2 + WB + 1).max() < E1
            np.add.at(written, (gy * nn + gx)[valid], 1)
    assert (written == 1).all()
    assert lds_words * 8 <= 65536
    return ntx * nty


@pytest.mark.parametrize("items,NT", [(1, 256), (2, 256), (1, 512), (2, 512)])
def test_tiled_fused_kernel_indices(items, NT):
    for N in GRIDS_3D:
        nn = N + 1
        nt = emulate_tiled(N, items, NT)
        if nt is None:
            continue
        for nzc in z_candidates(nn, nt):
            for z0, z1 in zranges(nn, nzc):
                zlast = min(z1 + 1, N)
                check_planes(N, [max(z0 - 2, 0)] + [max(min(pz + 1, zlast), 0)
                                                    for pz in range(z0 - 2, z1 + 2)])


# ---------------------------------------------------------------- k_strip2
STRIP_CFGS = {1: (32, 32, 4, 256), 2: (32, 16, 2, 256), 3: (64, 16, 4, 256), 4: (32, 24, 3, 256),
              5: (64, 12, 3, 256)}


def emulate_strip(N, cfg):
    BX, BY, P, NT = STRIP_CFGS[cfg]
    assert BX * BY // P == NT
    nn = N + 1
    plane = nn * nn
    WA, EA = BX + 2, (BX + 2) * (BY + 2)
    KA = (EA + NT - 1) // NT
    assert KA <= 32  # one bit per slot in an unsigned mask
    assert 2 * EA * 8 <= 65536
    ntx, nty = (nn + BX - 3) // (BX - 2), (nn + BY - 3) // (BY - 2)
    tid = np.arange(NT)
    written = np.zeros(plane, np.int64)
    for tile in range(ntx * nty):
        X0, Y0 = (tile % ntx) * (BX - 2) - 1, (tile // ntx) * (BY - 2) - 1
        for k in range(KA):
            t = tid + NT * k
            gy, gx = Y0 - 1 + t // WA, X0 - 1 + t % WA
            oa = np.clip(gy, 0, N) * nn + np.clip(gx, 0, N)
            assert oa.min() >= 0 and oa.max() < plane
        cx, cy0 = tid % BX, (tid // BX) * P
        assert (cy0 + P).max() <= BY
        rows = (cy0[:, None] + np.arange(P + 2)[None, :]) * WA + cx[:, None]
        assert rows.min() >= 0 and rows.max() + 2 < EA  # partials read columns cx .. cx+2
        gx = X0 + cx
        xin = (gx >= 0) & (gx <= N)
        xout = (cx >= 1) & (cx <= BX - 2) & xin
        for p in range(P):
            cy = cy0 + p
            gy = Y0 + cy
            off = np.clip(gy, 0, N) * nn + np.clip(gx, 0, N)
            assert off.min() >= 0 and off.max() < plane
            assert ((cy + 1) * WA + cx + 1).max() < EA  # stage-1 LDS write
            out = xout & (gy >= 0) & (gy <= N) & (cy >= 1) & (cy <= BY - 2)
            np.add.at(written, off[out], 1)
    assert (written == 1).all()
    return ntx * nty


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_strip_fused_kernel_indices(cfg):
    for N in GRIDS_3D:
        nn = N + 1
        nw = emulate_strip(N, cfg)
        for nzc in z_candidates(nn, nw):
            for z0, z1 in zranges(nn, nzc):
                zlast = min(z1 + 1, N)
                check_planes(N, [max(z0 - 2, 0)] + [max(min(pz + 1, zlast), 0)
                                                    for pz in range(z0 - 2, z1 + 2)])
                # stage-1 pointwise planes q1+1 and stage-2 planes o+1, clamped
                check_planes(N, [max(z0 - 1, 0)] + [min(max(pz, 0), N)
                                                    for pz in range(z0 - 2, z1 + 2)])
                check_planes(N, [max(z0, 0)] + [min(max(pz - 1, 0), N)
                                                for pz in range(z0 - 2, z1 + 2)])


def emulate_strip_prolong(N, cfg):
    """Coarse staging of the post-smoother with the prolongation folded in
    (N = 2 Nc): every coarse value a staged fine node reads lies inside the
    CW x CH window held in LDS and is the coarse node that the interpolation
    of that fine node names."""
    BX, BY, P, NT = STRIP_CFGS[cfg]
    Nc = N // 2
    nn = N + 1
    WA, EA = BX + 2, (BX + 2) * (BY + 2)
    KA = (EA + NT - 1) // NT
    CW, CH = BX // 2 + 3, BY // 2 + 3
    CE = CW * CH
    assert (2 * EA + 2 * CE) * 8 <= 65536
    ntx, nty = (nn + BX - 3) // (BX - 2), (nn + BY - 3) // (BY - 2)
    tid = np.arange(NT)
    for tile in range(ntx * nty):
        X0, Y0 = (tile % ntx) * (BX - 2) - 1, (tile // ntx) * (BY - 2) - 1
        CI0, CJ0 = (X0 - 1) >> 1, (Y0 - 1) >> 1
        for k in range(KA):
            t = tid + NT * k
            gy, gx = Y0 - 1 + t // WA, X0 - 1 + t % WA
            va = (t < EA) & (gy >= 0) & (gy <= N) & (gx >= 0) & (gx <= N)
            cl = ((gy >> 1) - CJ0) * CW + ((gx >> 1) - CI0)
            for yb in (0, 1):
                for di in (0, 1):
                    use = va & ((yb == 0) | (gy & 1 == 1)) & ((di == 0) | (gx & 1 == 1))
                    j = cl[use] + yb * CW + di
                    assert j.size == 0 or (j.min() >= 0 and j.max() < CE)
                    cj, ci = CJ0 + j // CW, CI0 + j % CW
                    assert np.array_equal(cj, (gy[use] >> 1) + yb)
                    assert np.array_equal(ci, (gx[use] >> 1) + di)
                    assert j.size == 0 or (min(cj.min(), ci.min()) >= 0 and
                                           max(cj.max(), ci.max()) <= Nc)


def prolong_plane_schedule(N, z0, z1):
    """The two LDS coarse-plane buffers over a z-chunk's trips: each trip's
    staging finds coarse plane pz>>1 (and pz>>1 + 1 for odd pz) in place, and
    a plane is overwritten only after the last trip that reads it."""
    Nc = N // 2
    buf = [None, None]
    K0 = max(z0 - 2, 0) >> 1
    buf[K0 & 1] = K0
    buf[(K0 + 1) & 1] = K0 + 1 if K0 + 1 <= Nc else None
    for pz in range(z0 - 2, z1 + 2):
        if 0 <= pz <= N:
            K = pz >> 1
            assert buf[K & 1] == K, (N, z0, z1, pz)
            if pz & 1:
                assert buf[(K + 1) & 1] == K + 1, (N, z0, z1, pz)
            if not (pz & 1) and K + 1 <= Nc:
                # committed after this trip's first barrier: the buffer's
                # previous plane K - 1 was last read by trip pz - 1
                buf[(K + 1) & 1] = K + 1


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_strip_prolong_indices(cfg):
    for N in GRIDS_3D:
        if N % 2:
            continue
        nn = N + 1
        emulate_strip_prolong(N, cfg)
        BX, BY, _, _ = STRIP_CFGS[cfg]
        nw = ((nn + BX - 3) // (BX - 2)) * ((nn + BY - 3) // (BY - 2))
        for nzc in z_candidates(nn, nw):
            for z0, z1 in zranges(nn, nzc):
                prolong_plane_schedule(N, z0, z1)
