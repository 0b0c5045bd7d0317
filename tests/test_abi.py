"""The C-ABI library loads and exports every entry point include/rx.h
declares; host-only argument checks behave as documented.  CPU only: no
call here reaches a GPU kernel."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rx.h")
LIB = os.path.join(ROOT, "paper_2602_13509_amd", "librx.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rx_status|const char\*|int64_t)\s+(rx_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_core_calls():
    names = declared()
    for n in ("rx_init", "rx_push_lines", "rx_scores", "rx_mask", "rx_destroy", "rx_server_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(\w+)$", out, re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2602_13509_amd import rx
    assert sorted(rx.EXPORTED) == declared()


def test_config_defaults_and_host_validation():
    from paper_2602_13509_amd import rx
    cfg = rx.rx_config()
    assert rx.LIB.rx_config_init(C.byref(cfg), 270, 640) == rx.RX_OK
    assert cfg.struct_size == C.sizeof(rx.rx_config)
    assert (cfg.in_type, cfg.syrk_prec, cfg.whiten_prec, cfg.bit_depth) == (rx.RX_IN_U16, rx.RX_BF16, rx.RX_BF16, 12)
    b = C.c_size_t()
    assert rx.LIB.rx_stream_footprint(C.byref(cfg), 100, C.byref(b)) == rx.RX_OK and b.value > 0
    for field, bad in (("bands", 0), ("bands", 321), ("samples", 0), ("syrk_prec", 5),
                       ("whiten_prec", 9), ("ddof", 2), ("layout", 2), ("flags", 4), ("struct_size", 4)):
        c2 = rx.rx_config()
        C.memmove(C.byref(c2), C.byref(cfg), C.sizeof(cfg))
        setattr(c2, field, bad)
        assert rx.LIB.rx_stream_footprint(C.byref(c2), 100, C.byref(b)) == rx.RX_E_ARG, field
        assert rx.last_error()
    c3 = rx.rx_config()
    C.memmove(C.byref(c3), C.byref(cfg), C.sizeof(cfg))
    c3.ridge_rel = float("nan")
    assert rx.LIB.rx_stream_footprint(C.byref(c3), 100, C.byref(b)) == rx.RX_E_ARG


def test_null_handles_are_rejected():
    from paper_2602_13509_amd import rx
    n = C.c_int64()
    assert rx.LIB.rx_destroy(None) == rx.RX_OK
    assert rx.LIB.rx_push_lines(None, None, 1, 0, None) == rx.RX_E_ARG
    assert rx.LIB.rx_scores(None, None, 0, C.byref(n), 0, None) == rx.RX_E_ARG
    assert rx.LIB.rx_init(None, None, None) == rx.RX_E_ARG
    assert rx.LIB.rx_server_destroy(None) == rx.RX_OK


def test_footprint_accounts_for_causal_slot_and_float_validity():
    # Host logic only (no GPU): the admission footprint grows by the causal
    # mode's extra snapshot slot and by the float-input validity buffers,
    # and counters carry the non-finite and FP8 saturation fields (whitening and
    # covariance product).
    import numpy as np
    from paper_2602_13509_amd import rx
    base = rx.stream_footprint(rx.make_config(270, 640, in_dtype=np.uint16), 100)
    causal = rx.stream_footprint(rx.make_config(270, 640, in_dtype=np.uint16, causal=True), 100)
    flt = rx.stream_footprint(rx.make_config(270, 640, in_dtype=np.float32), 100)
    assert causal > base and flt > base
    assert flt - base >= 2 * 100 * 640               # two parity sets of one validity byte per pixel
    assert rx.make_config(16, 16, causal=True).flags == rx.RX_FLAG_CAUSAL
    names = [f[0] for f in rx.rx_counters._fields_]
    assert names[-3:] == ["nonfinite_px", "fp8_saturated", "fp8_syrk_saturated"]


def test_one_pass_flag_is_exclusive_with_causal_and_takes_the_extra_slot():
    # Host logic only: the one-pass flag keeps the window-before slot (same
    # footprint as causal mode) and cannot be combined with the causal flag;
    # unknown flag bits are refused.
    import numpy as np
    from paper_2602_13509_amd import rx
    assert rx.make_config(16, 16, one_pass=True).flags == rx.RX_FLAG_ONE_PASS
    causal = rx.stream_footprint(rx.make_config(270, 640, in_dtype=np.uint16, causal=True), 100)
    one = rx.stream_footprint(rx.make_config(270, 640, in_dtype=np.uint16, one_pass=True), 100)
    assert one == causal
    for flags in (rx.RX_FLAG_CAUSAL | rx.RX_FLAG_ONE_PASS, 4):
        cfg = rx.make_config(16, 16)
        cfg.flags = flags
        n = C.c_size_t()
        assert rx.LIB.rx_stream_footprint(C.byref(cfg), 16, C.byref(n)) == rx.RX_E_ARG
