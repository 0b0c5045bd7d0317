"""Index arithmetic of the direct-load covariance kernel (k_syrk3), walked on
the CPU for every padded band count: every direct load, conversion and
fragment read stays inside its LDS ring buffer, the three buffers fit the
160 KiB of LDS, and the pipeline (two chunks queued ahead, one barrier per
chunk) queues, converts and multiplies every chunk of a split once, in
order, requeueing a buffer only after its chunk was multiplied."""
import pytest

S2NT, MAXT, KC = 1024, 20, 64
S2IT = (16 * MAXT * 8 + S2NT - 1) // S2NT
S3RING = 128 * S2IT          # rows per ring buffer: S2IT load rounds of 128 rows
LDS = 160 * 1024


def ring(bp):
    return 3, S3RING


def super_tile(wv):
    i, t = 0, wv
    while t > i:
        t -= i + 1
        i += 1
    return i, t


@pytest.mark.parametrize("bp", range(16, 16 * MAXT + 1, 16))
def test_ring_accesses_stay_in_bounds(bp):
    d, cap = ring(bp)
    assert d * cap * KC * 2 + 16 * MAXT * 4 <= LDS                  # ring + shift table
    assert S2IT == 3
    for wv in range(S2NT // 64):
        for q in range(S2IT):
            rb = 128 * q + 8 * wv                                    # every round loads, also past bp
            assert 0 <= rb and rb + 8 <= cap                         # one wave's 64 x 16 bytes
        nsup = (bp + 63) // 64
        i, j = super_tile(wv)
        if i >= nsup:
            continue
        assert 64 * i + 63 < cap and 64 * j + 63 < cap               # every fragment read
        for r in range(4):
            for cgrp in range(4):
                for jc in range(cgrp, 4, 4):
                    stored = 64 * i + 16 * r < bp and 64 * j + 16 * jc < bp and (i > j or r >= jc)
                    if stored:
                        assert 64 * i + 16 * r + 15 < bp + 15 and 64 * j + 16 * jc < bp


@pytest.mark.parametrize("d", [3])
def test_ring_steps_queue_each_chunk_once(d):
    # the pipeline's order (prologue, whole rotations, last steps) queues,
    # converts and multiplies every chunk of a split exactly once, in order,
    # and a buffer is requeued only after its chunk was multiplied
    for n in range(0, 40):
        queued, conv, mult = [], [], []
        buf_of = {}
        c0, c1 = 0, n
        nxt = c0

        def queue(slot):
            nonlocal nxt
            assert slot not in buf_of.values() or all(c in mult for c, s in buf_of.items() if s == slot)
            buf_of[nxt] = slot
            queued.append(nxt)
            nxt += 1

        if c0 < c1:
            queue(0)
            if c0 + 1 < c1:
                queue(1)
            if d == 4 and c0 + 2 < c1:
                queue(2)
            conv.append(c0)
        ch = c0
        while ch + 2 * d - 2 < c1:
            for i in range(d):
                queue((i + d - 1) % d)
                assert buf_of[ch + i] == i % d and (ch + i) in conv
                mult.append(ch + i)
                conv.append(ch + i + 1)
            ch += d
        for i in range(2 * d - 1):
            c = ch + i
            if c >= c1:
                continue
            if c + d - 1 < c1:
                queue((i + d - 1) % d)
            assert buf_of[c] == i % d and c in conv
            mult.append(c)
            if c + 1 < c1:
                conv.append(c + 1)
        assert queued == list(range(n)) and conv == list(range(n)) and mult == list(range(n))
