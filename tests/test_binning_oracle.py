"""Pins of the ingest binning oracle (CPU only): brute force by plain loops
on tiny cubes, the identity at k = 1, conservation of the selected bands'
total, one band summing everything, and the 12-bit bound that keeps the
paper's four-band sums inside 16 bits."""
import numpy as np

from oracle import binning as ob
from paper_2602_13509_amd import synth


def brute(cube, b0, nb, k):
    l, b, s = cube.shape
    out = [[[0] * s for _ in range(nb // k)] for _ in range(l)]
    for li in range(l):
        for j in range(nb // k):
            for si in range(s):
                tot = 0
                for t in range(k):
                    tot += int(cube[li][b0 + j * k + t][si])
                out[li][j][si] = tot
    return np.array(out, dtype=np.int64)


def test_brute_force_tiny():
    for seed, (l, b, s, b0, nb, k) in enumerate([(2, 9, 5, 1, 8, 4), (3, 7, 3, 0, 6, 3), (1, 5, 4, 2, 3, 1)]):
        c = synth.raw_counts(seed, l, b, s)
        assert np.array_equal(ob.bin_bands(c, b0, nb, k), brute(c, b0, nb, k))


def test_identity_and_conservation():
    c = synth.raw_counts(4, 3, 30, 11)
    assert np.array_equal(ob.bin_bands(c, 5, 20, 1), c[:, 5:25, :].astype(np.int64))
    out = ob.bin_bands(c, 2, 24, 4)
    assert np.array_equal(out.sum(axis=1), c[:, 2:26, :].astype(np.int64).sum(axis=1))


def test_single_output_band_and_12_bit_bound():
    c = synth.raw_counts(5, 2, 8, 6)
    assert np.array_equal(ob.bin_bands(c, 0, 8, 8)[:, 0, :], c.astype(np.int64).sum(axis=1))
    full = np.full((1, 300, 4), 4095, np.uint16)
    out = ob.bin_bands(full, 10, 280, 4)
    assert out.shape == (1, 70, 4) and out.max() == 4 * 4095 <= 65535
