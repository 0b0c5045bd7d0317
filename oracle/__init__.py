"""FP64 CPU oracle for streaming global RX -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: it never loads
the native library and the library never imports it.  See rx.py (batch
definition), stream.py (line-block streaming with windows) and brute.py
(exact rationals for tiny cubes).

Parity status: every function here is pinned by tests/test_oracle_pins.py
(exact rationals, closed forms, invariants of Eq. 1 and brute force).  The
low-precision error model (stream.error_model_sd) is pinned statistically
there too: scores of inputs rounded to each format by an independent
round-to-nearest-even quantiser, computed in FP64, have the error spread the
model predicts.
"""
from . import rx, brute, stream  # noqa: F401
