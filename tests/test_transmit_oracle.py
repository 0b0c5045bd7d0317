"""Pins of the transmission-stage oracle (CPU only).

The oracle (oracle/transmit.py) follows the paper's transmission: square
root in FP32, normalised to the cube's maximum, binary16 codes, the maximum
carried beside them; the receiver undoes the normalisation and squares
(Sections "System Implementation / Data Transmission" and "... / Ground
Control Station").  What fixes it here, independently of its own formulas:
  * worked values: delta = (k / 128)^2 for k = 0..1024 has maximum m = 8 and
    codes k / 1024 exactly, checked against Python's own IEEE half packer;
  * the largest score codes as 1.0 (0x3C00), whatever its value;
  * round trip: decoded scores are within the binary16 rounding bound of
    the inputs (relative 2^-10 plus FP32 rounding);
  * codes are monotone in the score;
  * the receiver's threshold agrees with delta / max(delta) > tau outside
    the binary16 rounding band;
  * NaN, empty and all-zero inputs.
A wrong order (normalising before the square root), a truncating cast or a
maximum taken over the wrong quantity fails at least one of these."""
import struct

import numpy as np

from oracle import transmit as tx
from paper_2602_13509_amd import synth


def half_bits(x: float) -> int:
    return struct.unpack("<H", struct.pack("<e", x))[0]


def test_worked_values_code_exactly():
    k = np.arange(1025)
    delta = ((k / 128.0) ** 2).astype(np.float32)
    codes, m = tx.encode(delta)
    assert m == np.float32(8.0)
    assert codes.dtype == np.uint16
    assert [int(c) for c in codes] == [half_bits(v / 1024.0) for v in k]
    back, _ = tx.decode(codes, m, 0.110)
    assert np.array_equal(back, delta)            # every value here is exact both ways


def test_maximum_codes_as_one():
    for seed in range(3):
        d = synth.score_sample(seed, 5000)
        codes, m = tx.encode(d)
        i = int(np.nanargmax(d))
        assert codes[i] == 0x3C00
        assert m == np.sqrt(np.float32(np.nanmax(d)))
        assert codes.view(np.float16).astype(np.float32).max() == 1.0


def test_round_trip_within_half_precision_bound():
    d = synth.score_sample(7, 200000)
    codes, m = tx.encode(d)
    back, _ = tx.decode(codes, m, 0.110)
    q = np.sqrt(d.astype(np.float64)) / float(m)
    normal = q >= 2.0 ** -14                      # binary16 normal range
    rel = np.abs(back[normal].astype(np.float64) - d[normal]) / d[normal]
    assert rel.max() <= 2.0 ** -10 + 1e-6
    # and the rounding is to nearest: the code is the nearest binary16 of sqrt(d)/m
    h = codes.view(np.float16).astype(np.float64)
    assert np.all(np.abs(h[normal] - q[normal]) <= 2.0 ** -11 * q[normal] * (1 + 1e-6))


def test_codes_are_monotone():
    d = np.sort(synth.score_sample(11, 50000))
    codes, _ = tx.encode(d)
    h = codes.view(np.float16).astype(np.float32)
    assert np.all(np.diff(h) >= 0)


def test_receiver_threshold_matches_normalised_scores():
    d = synth.score_sample(3, 100000)
    tau = 0.110
    codes, m = tx.encode(d)
    _, mask = tx.decode(codes, m, tau)
    r = d.astype(np.float64) / np.nanmax(d)
    ref = r > tau
    band = np.abs(r - tau) <= 4 * 2.0 ** -11 * tau
    assert np.array_equal(mask[~band], ref[~band])
    assert ref.sum() > 0 and (~ref).sum() > 0


def test_nan_empty_and_zero_inputs():
    d = np.array([1.0, np.nan, 4.0, 0.0], dtype=np.float32)
    codes, m = tx.encode(d)
    assert m == np.float32(2.0)
    h = codes.view(np.float16)
    assert h[0] == np.float16(0.5) and np.isnan(h[1]) and h[2] == np.float16(1.0) and h[3] == 0
    _, mask = tx.decode(codes, m, 0.110)
    assert list(mask) == [True, False, True, False]   # NaN is never marked
    codes, m = tx.encode(np.zeros(0, np.float32))
    assert codes.size == 0 and m == 0
    codes, m = tx.encode(np.zeros(5, np.float32))
    assert m == 0 and np.all(codes == 0)
    codes, m = tx.encode(np.full(3, np.nan, np.float32))
    assert m == 0 and np.all(np.isnan(codes.view(np.float16)))


def test_pack_bits_order():
    bits = tx.pack_bits(np.array([1, 0, 0, 0, 0, 0, 0, 0, 0, 1], bool))
    assert list(bits) == [1, 2]
