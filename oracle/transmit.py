"""CPU oracle of the score transmission stage -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark may import this module.
It shares no code with the HIP library and never imports it.

What it computes (the paper, Section "System Implementation / Data
Transmission"): scores are sent as IEEE half-precision values; the square
root is taken first (the squared distance is heavily skewed towards small
values) and every value is normalised to the cube's maximum, which travels
in the packet header so the receiver can undo it.  The receiver (Section
"System Implementation / Ground Control Station") undoes the normalisation
and squares the scores; thresholded anomalies use 0.110 on the normalised
score (Section "Results / Detector Visual Analysis").

Precision: the paper computes in FP32 and transmits binary16, and the code is
an integer decided by floating point, so every step here is taken in FP32 as
the paper states (numpy's float32 square root and division are correctly
rounded; the cast to float16 rounds to nearest even).

Readings taken where the paper is silent:
  * the normalisation divides the square roots by their maximum, so the
    header value is m = max sqrt(delta) (= sqrt(max delta): the square root
    is monotone and correctly rounded);
  * NaN scores are left out of the maximum and code as NaN; with no finite
    score m = 0 and finite scores code as 0;
  * the receiver's threshold compares the normalised squared score h^2 with
    tau, strictly (the relative mode of the scoring oracle).
"""
from __future__ import annotations

import numpy as np


def encode(delta: np.ndarray) -> tuple[np.ndarray, np.float32]:
    """delta [n] (any float) -> (binary16 bit patterns uint16 [n], m float32)."""
    d = np.asarray(delta, dtype=np.float32)
    with np.errstate(invalid="ignore"):
        s = np.sqrt(d)
    fin = s[~np.isnan(s)]
    m = np.float32(fin.max()) if fin.size else np.float32(0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = (s / m).astype(np.float32) if m > 0 else np.where(np.isnan(s), s, np.float32(0.0)).astype(np.float32)
    return q.astype(np.float16).view(np.uint16), m


def decode(codes: np.ndarray, m: np.float32, tau: float) -> tuple[np.ndarray, np.ndarray]:
    """(codes, m, tau) -> (delta^ float32 [n] = (h m)^2, bool mask [n] = h^2 > tau)."""
    h = np.asarray(codes, dtype=np.uint16).view(np.float16).astype(np.float32)
    u = h * np.float32(m)
    with np.errstate(invalid="ignore"):
        mask = (h * h) > np.float32(tau)
    return (u * u).astype(np.float32), mask


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """bool [n] -> bytes, bit j of byte q = pixel 8q + j."""
    return np.packbits(np.asarray(mask, dtype=bool), bitorder="little")
