"""Host check of the factor kernels' index arithmetic (no GPU needed).

The three factor kernels (Cholesky sweep, column-tile inverse, operand rows)
hand tiles over through a per-block buffer and write W and the whitening
operand.  This walks the same index formulas for every band count the
three-kernel path takes (1..272 bands, T <= 17 tiles) and for the tail of
the single-workgroup kernel kept for 273..320 bands, and asserts that every
access lies inside its buffer and that every tile is owned exactly once.
The formulas are restated from the kernels; a change to one must be made
here too."""
import pytest

CNW, CDW, CMAXT, MAXT = 16, 3, 17, 20


def pad16(b):
    return 16 * -(-b // 16)


def lf_tiles(T):
    return T + T * (T - 1) // 2


def lf_stride(Bp):
    return 256 * lf_tiles(Bp // 16) + Bp


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


@pytest.mark.parametrize("B", range(1, 16 * CMAXT + 1))
def test_three_kernel_factor_indices_in_bounds(B):
    Bp = pad16(B)
    T = Bp // 16
    Bw = 32 * -(-Bp // 32)
    t_max = 8 if T <= 8 else (12 if T <= 12 else CMAXT)
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


@pytest.mark.parametrize("B", range(16 * CMAXT + 1, 16 * MAXT + 1))
def test_single_workgroup_factor_tail_in_bounds(B):
    # the 273..320-band kernel: rows i0 = 4 wv + 32 n (< Bp), four rows each;
    # columns j = lane + 64 c (c < 5); maxima read W[i Bp + j] for j <= i, j < B;
    # the operand writes wl[i Bw + j] for j < 16 (i / 16 + 1)
    Bp = pad16(B)
    Bw = 32 * -(-Bp // 32)
    for wv in range(8):
        for i0 in range(4 * wv, Bp, 32):
            for q in range(4):
                i = i0 + q
                assert i < Bp
                for c in range(5):
                    for lane in range(64):
                        j = lane + 64 * c
                        if j <= i and j < B:
                            assert i * Bp + j < Bp * Bp
                        if j < 16 * (i // 16 + 1):
                            assert j < Bp and i * Bw + j < Bp * Bw and i * Bp + j < Bp * Bp
