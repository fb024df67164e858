"""Host emulation of the index arithmetic of the multigrid transfer kernels
(no GPU): the z-streamed 3D restriction (k_restrict_zs) and the
prolongation (k_prolong_add) of paper_1603_04570_amd/csrc/k_mg.hip, for the
launch shapes launch_restrict and launch_prolong_add compute on the 3D
grids the multigrid hierarchies use.  Every global load and store and every
LDS access lies inside its array; the restriction writes every coarse node
exactly once and the prolongation updates every fine node exactly once.  A
change to either kernel's indexing must be mirrored here."""
import numpy as np
import pytest

RS_TI, RS_TJ = 64, 4
RS_FC, RS_FR = 2 * RS_TI + 1, 2 * RS_TJ + 1
RS_LOADS = (RS_FC * RS_FR + 255) // 256
PROLONG_W = 256

# coarse N of the 3D transfers between levels (fine N = 2 coarse N)
COARSE_3D = [4, 8, 13, 16, 25, 32, 50, 64, 100, 128, 200, 256]


def restrict_launch(cN, count=1):
    cnn = cN + 1
    tx = (cnn + RS_TI - 1) // RS_TI
    ti = (cnn + tx - 1) // tx
    ty = (cnn + RS_TJ - 1) // RS_TJ
    tiles = tx * ty * count
    nzc = min(cnn, max(1, (1536 + tiles - 1) // tiles))
    kc = (cnn + nzc - 1) // nzc
    nzc = (cnn + kc - 1) // kc
    return tx, ty, ti, kc, nzc


def emulate_restrict_zs(cN):
    cnn, fN = cN + 1, 2 * cN
    fnn = fN + 1
    tx, ty, ti, kc, nzc = restrict_launch(cN)
    assert ti <= RS_TI
    t = np.arange(256)
    written = np.zeros(cnn ** 3, np.int64)
    for bx in range(tx):
        for by in range(ty):
            I0, J0 = bx * ti, by * RS_TJ
            ncol = 2 * ti + 1
            nel = RS_FR * ncol
            # staging slots
            for u in range(RS_LOADS):
                e = t + 256 * u
                m = e < nel
                if not m.any():
                    continue
                row, col = e[m] // ncol, e[m] % ncol
                lw = row * RS_FC + col
                assert lw.min() >= 0 and lw.max() < RS_FR * RS_FC
                fy, fx = 2 * J0 - 1 + row, 2 * I0 - 1 + col
                ok = (fy >= 0) & (fy <= fN) & (fx >= 0) & (fx <= fN)
                off = fy[ok] * fnn + fx[ok]
                assert off.size == 0 or (off.min() >= 0 and off.max() < fnn * fnn)
            # outputs and their LDS reads
            i, j = t % RS_TI, t // RS_TI
            out = (i < ti) & (I0 + i < cnn) & (J0 + j < cnn)
            for dy in range(3):
                r = 2 * j[out] + dy
                c0 = 2 * i[out]
                assert r.max(initial=0) < RS_FR and (c0 + 2).max(initial=0) < ncol
            oq = (J0 + j[out]) * cnn + (I0 + i[out])
            for bz in range(nzc):
                K0, K1 = bz * kc, min(bz * kc + kc, cnn)
                assert K0 < cnn
                z0, z1 = max(2 * K0 - 1, 0), min(2 * K1 - 1, fN)
                assert 0 <= z0 <= z1 <= fN
                for zf in range(z0, z1 + 1):
                    K = zf >> 1
                    if zf % 2 == 0:
                        if zf == fN:
                            np.add.at(written, K * cnn * cnn + oq, 1)
                    elif K >= K0:
                        assert K < K1
                        np.add.at(written, K * cnn * cnn + oq, 1)
    assert written.min() == 1 and written.max() == 1


@pytest.mark.parametrize("cN", [c for c in COARSE_3D if c + 1 >= 33])
def test_restrict_streamed_indices(cN):
    emulate_restrict_zs(cN)


def emulate_prolong(cN):
    cnn, fN = cN + 1, 2 * cN
    fnn = fN + 1
    nseg = (cnn + PROLONG_W - 1) // PROLONG_W
    LW = PROLONG_W + 1
    cols = 2 * PROLONG_W // 256
    t = np.arange(256)
    upd = np.zeros(fnn ** 3, np.int64)
    for K in range(cnn):
        for J in range(cnn):
            for seg in range(nseg):
                I0, I1 = seg * cnn // nseg, (seg + 1) * cnn // nseg
                assert I1 - I0 <= PROLONG_W
                # staging: o < LW, clamped coarse reads
                o = np.arange(LW)
                Ic = np.minimum(I0 + o, cN)
                assert Ic.max() <= cN
                nfx = min(2 * I1, fnn) - 2 * I0
                assert nfx <= 256 * cols
                for rr in range(4):
                    a, b = rr & 1, rr >> 1
                    fj, fk = 2 * J + a, 2 * K + b
                    if fj > fN or fk > fN:
                        continue
                    for v in range(cols):
                        ix = t + 256 * v
                        ix = ix[ix < nfx]
                        fi = 2 * I0 + ix
                        li0, li1 = (fi >> 1) - I0, ((fi + 1) >> 1) - I0
                        assert li0.min(initial=0) >= 0 and li1.max(initial=0) < LW
                        q = (fk * fnn + fj) * fnn + fi
                        np.add.at(upd, q, 1)
    assert upd.min() == 1 and upd.max() == 1


@pytest.mark.parametrize("cN", [4, 8, 13, 16, 25, 32, 50, 64])
def test_prolong_indices(cN):
    emulate_prolong(cN)
