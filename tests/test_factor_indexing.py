"""Host check of the factor kernels' index arithmetic (no GPU needed).

The three factor kernels (Cholesky sweep, column-tile inverse, operand rows)
hand tiles over through a per-block buffer and write W and the whitening
operand.  This walks the same index formulas for every band count (1..320
bands, T <= 20 tiles) and asserts that every access lies inside its buffer,
that every tile is owned exactly once (in registers or, from 273 bands on,
in LDS), and that the Cholesky workgroup's LDS fits a CU.  The formulas are
restated from the kernels; a change to one must be made here too."""
import pytest

CNW, CDW, CMAXT, MAXT, CREG = 16, 3, 20, 20, 11
LDS_BYTES = 160 * 1024


def pad16(b):
    return 16 * -(-b // 16)


def lf_tiles(T):
    return T + T * (T - 1) // 2


def lf_stride(Bp):
    return 256 * lf_tiles(Bp // 16) + Bp


def tmax_for(T):
    return 8 if T <= 8 else (12 if T <= 12 else (17 if T <= 17 else 20))


def chol_lds_bytes(t_max):
    coff = -(-(t_max * (t_max - 1) // 2) // (CNW - CDW))
    clds = coff - min(coff, CREG)
    fts = 16 * 17
    # lcol, ybuf, overflow tiles, sc, diagonal staging, red, flag
    return (t_max * 64 * 32 + 2 * 64 * 32 + max(1, clds * (CNW - CDW)) * 64 * 32 + 16 * t_max * 8
            + CDW * fts * 8 + CNW * 8 + 4)


def chol_owners(T, t_max):
    cdiag = -(-t_max // CDW)
    coff = -(-(t_max * (t_max - 1) // 2) // (CNW - CDW))
    owned = {}
    for wv in range(CNW):
        ns = cdiag if wv < CDW else coff
        for s in range(ns):
            if wv < CDW:
                k = wv + CDW * s
                if k < T:
                    owned.setdefault((k, k), []).append(wv)
            else:
                u = s * (CNW - CDW) + (wv - CDW)
                if u < T * (T - 1) // 2:
                    i = 1
                    while (i + 1) * i // 2 <= u:
                        i += 1
                    j = u - i * (i - 1) // 2
                    owned.setdefault((i, j), []).append(wv)
    return owned


@pytest.mark.parametrize("t_max", [8, 12, 17, 20])
def test_cholesky_workgroup_lds_fits(t_max):
    assert chol_lds_bytes(t_max) <= LDS_BYTES


@pytest.mark.parametrize("B", range(1, 16 * CMAXT + 1))
def test_three_kernel_factor_indices_in_bounds(B):
    Bp = pad16(B)
    T = Bp // 16
    Bw = 32 * -(-Bp // 32)
    t_max = tmax_for(T)
    owned = chol_owners(T, t_max)
    assert sorted(owned) == sorted((i, j) for i in range(T) for j in range(i + 1))
    assert all(len(v) == 1 for v in owned.values())
    stride = lf_stride(Bp)
    # Cholesky: Y_k at 256 k .. +255, L_ik at 256 (T + i (i-1)/2 + k), scales after
    for k in range(T):
        assert 256 * k + 255 < 256 * T
    for i in range(T):
        for k in range(i):
            base = 256 * (T + i * (i - 1) // 2 + k)
            assert 256 * T <= base and base + 255 < 256 * lf_tiles(T)
    assert 256 * lf_tiles(T) + Bp <= stride
    # inverse: W rows 16 i + lg + 4 r, columns 16 j + lr, inside Bp x Bp; LDS tiles m < CMAXT
    for j in range(T):
        assert T - 1 < CMAXT
        for i in range(j, T):
            for lane in range(64):
                lr, lg = lane & 15, lane >> 4
                for q in range(4):
                    r, c = 16 * i + lg + 4 * q, 16 * j + lr
                    assert r * Bp + c < Bp * Bp
        # a wave's m terms of a row fit its VMT operand slots
        for i in range(j + 1, T):
            for wv in range(4):
                terms = [m for m in range(j + wv, i, 4)]
                assert len(terms) <= -(-CMAXT // 4)
    # operand rows: row tile t writes rows 16 t .. 16 t + 15, columns < 16 (t + 1) <= Bp <= Bw
    for t in range(T):
        ncol = 16 * (t + 1)
        assert ncol <= Bp <= Bw
        for wv in range(4):
            for q in range(4):
                i = 16 * t + 4 * wv + q
                assert i < Bp
                for c in range(5):
                    for lane in range(64):
                        jj = lane + 64 * c
                        if jj < ncol:
                            assert i * Bw + jj < Bp * Bw and i * Bp + jj < Bp * Bp
                        if jj <= i and jj < B:
                            assert i * Bp + jj < Bp * Bp
