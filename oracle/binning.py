"""CPU oracle of band selection and binning at ingest -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark may import this module.
It shares no code with the HIP library and never imports it.

What it computes (the paper, Section "System Implementation / Data
Acquisition"): the out-of-range bands of the 300-band imager are discarded,
leaving 280, and every four consecutive bands of those are summed into one
band of the 70-band cube.  On a BIL cube [lines][bands][samples]:
    out[l][j][s] = sum over t < k of in[l][b0 + j k + t][s],  j < nb / k.
The paper does not say how many bands go at each end; b0 (the first kept
band) is a parameter; the reading taken is b0 = 10 (ten each side).  Counts
are integers, so the sums are exact (int64 here)."""
from __future__ import annotations

import numpy as np


def bin_bands(cube: np.ndarray, b0: int, nb: int, k: int) -> np.ndarray:
    l, b, s = cube.shape
    assert k >= 1 and nb % k == 0 and 0 <= b0 and b0 + nb <= b
    sel = np.asarray(cube[:, b0:b0 + nb, :], dtype=np.int64)
    return sel.reshape(l, nb // k, k, s).sum(axis=2)
