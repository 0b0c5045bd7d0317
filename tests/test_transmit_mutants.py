"""Planted mistakes in copies of the transmission oracle (CPU only): each is
a plausible error and must fail at least one of the checks that pin the
oracle; the real oracle passes all of them."""
import struct

import numpy as np
import pytest

from oracle import transmit as tx
from paper_2602_13509_amd import synth


def half_bits(x):
    return struct.unpack("<H", struct.pack("<e", x))[0]


def chk_worked(enc, dec):
    k = np.arange(1025)
    d = ((k / 128.0) ** 2).astype(np.float32)
    codes, m = enc(d)
    back, _ = dec(codes, m, 0.110)
    return [int(c) for c in codes] == [half_bits(v / 1024.0) for v in k] and np.array_equal(back, d)


def chk_max_one(enc, dec):
    d = synth.score_sample(1, 4000)
    codes, _ = enc(d)
    return codes[int(np.nanargmax(d))] == 0x3C00


def chk_round_trip(enc, dec):
    d = synth.score_sample(5, 50000)
    codes, m = enc(d)
    back, _ = dec(codes, m, 0.110)
    q = np.sqrt(d.astype(np.float64)) / np.sqrt(np.nanmax(d).astype(np.float64))
    nz = q >= 2.0 ** -14
    h = codes.view(np.float16).astype(np.float64)
    return (np.all(np.abs(back[nz] - d[nz]) <= (2.0 ** -10 + 1e-6) * d[nz])
            and np.all(np.abs(h[nz] - q[nz]) <= 2.0 ** -11 * q[nz] * (1 + 1e-6)))


def chk_threshold(enc, dec):
    d = synth.score_sample(3, 50000)
    codes, m = enc(d)
    _, mask = dec(codes, m, 0.110)
    r = d.astype(np.float64) / np.nanmax(d)
    band = np.abs(r - 0.110) <= 4 * 2.0 ** -11 * 0.110
    return np.array_equal(mask[~band], (r > 0.110)[~band])


def chk_nan(enc, dec):
    d = np.array([1.0, np.nan, 4.0, 0.0], dtype=np.float32)
    codes, m = enc(d)
    h = codes.view(np.float16)
    return m == 2.0 and h[0] == 0.5 and np.isnan(h[1]) and h[2] == 1.0 and h[3] == 0


CHECKS = [chk_worked, chk_max_one, chk_round_trip, chk_threshold, chk_nan]


def enc_norm_before_sqrt(d):      # header carries max(delta), values sqrt(delta / max)
    d = d.astype(np.float32)
    mx = np.float32(np.nanmax(d))
    return np.sqrt(d / mx).astype(np.float16).view(np.uint16), mx


def enc_truncate(d):              # rounding toward zero instead of to nearest
    c, m = tx.encode(d)
    s = np.sqrt(d.astype(np.float32)) / m
    h = s.astype(np.float16)
    over = np.abs(h.astype(np.float32)) > np.abs(s)
    bits = h.view(np.uint16).copy()
    bits[over] -= 1
    return bits, m


def enc_max_not_sqrt(d):          # normalised by max(delta) instead of its square root
    d = d.astype(np.float32)
    mx = np.float32(np.nanmax(d))
    return (np.sqrt(d) / mx).astype(np.float16).view(np.uint16), np.sqrt(mx)


def enc_nan_in_max(d):            # NaN not skipped in the maximum
    d = d.astype(np.float32)
    s = np.sqrt(d)
    m = np.float32(np.max(s))
    return (s / m).astype(np.float16).view(np.uint16), m


def dec_square_first(codes, m, tau):   # squares, then scales by m once
    h = codes.view(np.float16).astype(np.float32)
    return (h * h * np.float32(m)).astype(np.float32), h * h > tau


def dec_thr_on_root(codes, m, tau):    # threshold on h instead of h^2
    back, _ = tx.decode(codes, m, tau)
    h = codes.view(np.float16).astype(np.float32)
    return back, h > tau


MUTANTS = {
    "normalise_before_sqrt": (enc_norm_before_sqrt, tx.decode),
    "truncating_cast": (enc_truncate, tx.decode),
    "max_without_sqrt": (enc_max_not_sqrt, tx.decode),
    "nan_in_max": (enc_nan_in_max, tx.decode),
    "decode_square_first": (tx.encode, dec_square_first),
    "threshold_on_root": (tx.encode, dec_thr_on_root),
}


def test_real_oracle_passes_every_check():
    for chk in CHECKS:
        assert chk(tx.encode, tx.decode), chk.__name__


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    enc, dec = MUTANTS[name]
    with np.errstate(all="ignore"):
        results = [bool(chk(enc, dec)) for chk in CHECKS]
    assert not all(results), f"mutant {name} passed every check"
