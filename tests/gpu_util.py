"""Shared helpers for the GPU parity tests (HIP path vs the FP64 oracle)."""
import sys

import numpy as np

from oracle import rx as orx
from oracle.stream import RxStreamOracle


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(got, ref, bands):
    """|d_gpu - d_ref| / max(d_ref, 1e-3 B), elementwise."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(ref, 1e-3 * bands)


def err_summary(got, ref, bands):
    e = rel_err(got, ref, bands)
    return float(np.max(e)), float(np.quantile(e, 0.99))


def assert_scores(got, ref, bands, max_rel, p99_rel, label=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    nan_ref = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan_ref), f"{label}: NaN pattern differs"
    if (~nan_ref).sum() == 0:
        return
    mx, p99 = err_summary(got[~nan_ref], ref[~nan_ref], bands)
    say(f"  {label}: max rel {mx:.3e}  p99 rel {p99:.3e}  (bounds {max_rel:g}/{p99_rel:g})")
    assert mx <= max_rel, f"{label}: max rel err {mx:.3e} > {max_rel}"
    assert p99 <= p99_rel, f"{label}: p99 rel err {p99:.3e} > {p99_rel}"


def assert_mask(got_mask, ref_scores, tau_eff, tol, bands, label=""):
    """Bit-identical wherever the oracle score is farther than the tolerance
    band from the threshold; either value is accepted inside the band."""
    ref = np.asarray(ref_scores, dtype=np.float64)
    band = tol * max(tau_eff, 1e-3 * bands)
    want = orx.mask_abs(ref, tau_eff)
    decided = np.abs(ref - tau_eff) > band
    bad = np.flatnonzero(decided & (np.asarray(got_mask) != want))
    say(f"  {label}: {int((~decided).sum())} pixels inside the tolerance band, {bad.size} decided mismatches")
    assert bad.size == 0, f"{label}: mask differs at decided pixels {bad[:10]}"


def oracle_stream_scores(cube, bands, samples, block_lines=0, window_lines=0, ddof=0, rho=0.0, pushes=None,
                         causal=False, one_pass=False):
    o = RxStreamOracle(bands, samples, ddof=ddof, rho=rho, window_lines=window_lines, block_lines=block_lines,
                       causal=causal, one_pass=one_pass)
    if pushes is None:
        pushes = [cube.shape[0]]
    out, l0 = [], 0
    for n in pushes:
        out.append(o.push(cube[l0:l0 + n]))
        l0 += n
    return np.concatenate(out), o
