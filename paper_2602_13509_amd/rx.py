"""Python binding of the C ABI in include/rx.h (ctypes; argument marshalling only).

Every step of the scoring path runs in the HIP library (librx.so, built for
gfx950).  Importing this module loads that library and fails loudly if it is
missing: there is no CPU fallback.  PyTorch is used only for device memory
and streams (tensors are passed as raw device pointers).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librx.so")

RX_OK, RX_E_ARG, RX_E_NOMEM, RX_E_NOTREADY, RX_E_SINGULAR, RX_E_DEVICE, RX_E_BUDGET, RX_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
RX_IN_U16, RX_IN_F32, RX_IN_F64 = 0, 1, 2
RX_BIL, RX_BIP = 0, 1
RX_LINES_HOST, RX_LINES_DEVICE, RX_LINES_RESIDENT = 0, 1, 2
RX_FP64, RX_FP32, RX_BF16, RX_FP16, RX_FP8_E4M3 = 0, 1, 2, 3, 4
RX_THR_ABS, RX_THR_REL_MAX, RX_THR_TOPK = 0, 1, 2
RX_FLAG_CAUSAL = 1
RX_FLAG_ONE_PASS = 2
RX_MAX_BANDS = 320
RX_MASK_NOALLOC_BYTES = 4096 + (1 << 20)
RX_MASK_NOALLOC_MAX_PX = 1 << 23

STATUS_NAMES = {0: "RX_OK", -1: "RX_E_ARG", -2: "RX_E_NOMEM", -3: "RX_E_NOTREADY", -4: "RX_E_SINGULAR",
                -5: "RX_E_DEVICE", -6: "RX_E_BUDGET", -7: "RX_E_STATE"}
PREC = {"fp64": RX_FP64, "fp32": RX_FP32, "bf16": RX_BF16, "fp16": RX_FP16, "fp8": RX_FP8_E4M3}
IN_TYPE = {np.dtype(np.uint16): RX_IN_U16, np.dtype(np.float32): RX_IN_F32, np.dtype(np.float64): RX_IN_F64}

EXPORTED = [
    "rx_config_init", "rx_init", "rx_push_lines", "rx_scores", "rx_scores_f64", "rx_mask", "rx_wait",
    "rx_sync", "rx_get_counters", "rx_destroy", "rx_last_error", "rx_get_stats", "rx_set_stats",
    "rx_get_whitener", "rx_server_create", "rx_server_destroy", "rx_stream_footprint", "rx_server_submit",
    "rx_server_step", "rx_server_poll", "rx_server_sync", "rx_server_queued", "rx_profile",
    "rx_phase_times", "rx_tx_encode", "rx_tx_decode", "rx_encode", "rx_bin_bands", "rx_split_plan",
    "rx_mask_noalloc", "rx_server_start", "rx_server_stop", "rx_server_poll_ns", "rx_clock_ns",
]


class rx_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("bands", C.c_int32), ("samples", C.c_int32), ("in_type", C.c_int32),
        ("bit_depth", C.c_int32), ("layout", C.c_int32), ("syrk_prec", C.c_int32), ("whiten_prec", C.c_int32),
        ("ddof", C.c_int32), ("block_lines", C.c_int32), ("window_lines", C.c_int64), ("ridge_rel", C.c_double),
        ("device", C.c_int32), ("flags", C.c_int32),
    ]


class rx_counters(C.Structure):
    _fields_ = [("lines_pushed", C.c_int64), ("blocks", C.c_int64), ("singular_blocks", C.c_int64),
                ("notready_blocks", C.c_int64), ("pending_px", C.c_int64), ("window_px", C.c_int64),
                ("nonfinite_px", C.c_int64), ("fp8_saturated", C.c_int64), ("fp8_syrk_saturated", C.c_int64)]


class RxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    # The library and PyTorch's ROCm build each need a HIP runtime under the
    # same soname (libamdhip64.so.7); the dynamic loader gives the whole
    # process whichever is loaded first.  Importing torch first keeps the
    # process on the runtime torch was built with, which the library also
    # runs on; the other order leaves torch on a runtime it was not built for
    # and the first kernel launch finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950) first")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    sig = {
        "rx_config_init": (I32, [C.POINTER(rx_config), I32, I32]),
        "rx_init": (I32, [C.POINTER(rx_config), P, C.POINTER(P)]),
        "rx_push_lines": (I32, [P, P, I64, I32, P]),
        "rx_scores": (I32, [P, P, I64, C.POINTER(I64), I32, P]),
        "rx_scores_f64": (I32, [P, P, I64, C.POINTER(I64), I32, P]),
        "rx_mask": (I32, [P, D, I32, I64, P, I64, C.POINTER(I64), I32, P]),
        "rx_wait": (I32, [P, P]),
        "rx_sync": (I32, [P]),
        "rx_get_counters": (I32, [P, C.POINTER(rx_counters)]),
        "rx_destroy": (I32, [P]),
        "rx_last_error": (C.c_char_p, []),
        "rx_get_stats": (I32, [P, C.POINTER(I64), P, P]),
        "rx_set_stats": (I32, [P, I64, P, P]),
        "rx_get_whitener": (I32, [P, P]),
        "rx_server_create": (I32, [SZ, I32, I32, C.POINTER(P)]),
        "rx_server_destroy": (I32, [P]),
        "rx_stream_footprint": (I32, [C.POINTER(rx_config), I32, C.POINTER(SZ)]),
        "rx_server_submit": (I32, [P, P, P, I64, U64]),
        "rx_server_step": (I32, [P, C.POINTER(I32)]),
        "rx_server_poll": (I32, [P, P, I32, C.POINTER(I32), I32]),
        "rx_server_sync": (I32, [P]),
        "rx_server_queued": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(SZ)]),
        "rx_profile": (I32, [P, I32]),
        "rx_phase_times": (I32, [P, P, P]),
        "rx_tx_encode": (I32, [P, I64, P, P, P]),
        "rx_tx_decode": (I32, [P, I64, P, C.c_float, P, P, P]),
        "rx_encode": (I32, [P, P, I64, C.POINTER(I64), P, P]),
        "rx_bin_bands": (I32, [P, I64, I32, I32, I32, I32, I32, I32, P, P]),
        "rx_split_plan": (I32, [C.POINTER(rx_config), I64, C.POINTER(I32), C.POINTER(I64)]),
        "rx_mask_noalloc": (I32, [P, D, I32, I64, P, I64, C.POINTER(I64), P]),
        "rx_server_start": (I32, [P]),
        "rx_server_stop": (I32, [P]),
        "rx_server_poll_ns": (I32, [P, P, P, I32, C.POINTER(I32), I32]),
        "rx_clock_ns": (I64, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    return lib


LIB = _load()


def last_error() -> str:
    return LIB.rx_last_error().decode(errors="replace")


def check(status: int, allow=()) -> int:
    if status != RX_OK and status not in allow:
        raise RxError(status, last_error())
    return status


def _ptr(a) -> int:
    """Raw address of a torch tensor (device or host) or numpy array."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _is_dev(a) -> int:
    return 0 if isinstance(a, np.ndarray) else int(a.is_cuda)


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def make_config(bands: int, samples: int, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ddof=0,
                ridge_rel=0.0, block_lines=0, window_lines=0, bit_depth=12, device=0, causal=False,
                layout=RX_BIL, one_pass=False) -> rx_config:
    cfg = rx_config()
    check(LIB.rx_config_init(C.byref(cfg), bands, samples))
    cfg.in_type = IN_TYPE[np.dtype(in_dtype)]
    cfg.bit_depth = bit_depth if np.dtype(in_dtype) == np.uint16 else 0
    cfg.syrk_prec = PREC[syrk] if isinstance(syrk, str) else syrk
    cfg.whiten_prec = PREC[whiten] if isinstance(whiten, str) else whiten
    cfg.ddof, cfg.ridge_rel = ddof, float(ridge_rel)
    cfg.block_lines, cfg.window_lines, cfg.device = block_lines, window_lines, device
    cfg.flags = (RX_FLAG_CAUSAL if causal else 0) | (RX_FLAG_ONE_PASS if one_pass else 0)
    cfg.layout = layout
    return cfg


class RxStream:
    """One sensor stream (rx_init ... rx_destroy)."""

    def __init__(self, cfg: rx_config, server: "RxServer | None" = None):
        self.cfg = cfg
        h = C.c_void_p()
        check(LIB.rx_init(C.byref(cfg), server.h if server else None, C.byref(h)))
        self.h = h
        self.B, self.S = cfg.bands, cfg.samples
        self.score_f64 = cfg.whiten_prec == RX_FP64

    # -- core path
    def rx_push_lines(self, lines, stream=None, allow_notready=True, guard=True, resident=False) -> int:
        """lines: BIL [n_lines][B][S] (BIP [n_lines][S][B] for an RX_BIP stream)
        torch tensor (device or host) or numpy array.

        A device tensor is read asynchronously on the library's own queues,
        after the work already on the caller's stream (torch's current one by
        default).  With guard=True the caller's stream is then made to wait
        for that work (rx_wait, no host block), so later work on it --
        including torch's reuse of the tensor's memory once it is freed --
        cannot overwrite the lines before they are read.  guard=False leaves
        the caller's stream free (so one push's tail can overlap the next
        push): the tensor must then stay alive and unchanged until rx_sync or
        an rx_wait, as the C interface states.
        resident=True (device tensors already written, e.g. after a
        synchronisation): RX_LINES_RESIDENT, the push orders itself against
        no stream and stream / guard are not used; the tensor must stay alive
        and unchanged until rx_sync."""
        n = lines.shape[0]
        shape = (self.S, self.B) if self.cfg.layout == RX_BIP else (self.B, self.S)
        assert tuple(lines.shape[1:]) == shape, lines.shape
        dev = _is_dev(lines)
        if resident:
            assert dev, "resident lines are device memory"
            return check(LIB.rx_push_lines(self.h, _ptr(lines), n, RX_LINES_RESIDENT, 0),
                         allow=(RX_E_NOTREADY,) if allow_notready else ())
        sh = _stream_handle(stream) if dev else 0
        r = check(LIB.rx_push_lines(self.h, _ptr(lines), n, RX_LINES_DEVICE if dev else RX_LINES_HOST, sh),
                  allow=(RX_E_NOTREADY,) if allow_notready else ())
        if dev and guard:
            check(LIB.rx_wait(self.h, sh))
        return r

    def rx_scores(self, out, stream=None) -> int:
        n = C.c_int64()
        dev = _is_dev(out)
        f = LIB.rx_scores_f64 if str(out.dtype).endswith("float64") else LIB.rx_scores
        check(f(self.h, _ptr(out), out.numel() if hasattr(out, "numel") else out.size, C.byref(n), dev,
                _stream_handle(stream) if dev else 0))
        return n.value

    def rx_mask(self, tau: float, mode: int, k: int, out, stream=None) -> int:
        n = C.c_int64()
        dev = _is_dev(out)
        size = out.numel() if hasattr(out, "numel") else out.size
        check(LIB.rx_mask(self.h, float(tau), mode, int(k), _ptr(out), size, C.byref(n), dev,
                          _stream_handle(stream) if dev else 0))
        return n.value

    def rx_mask_noalloc(self, tau: float, mode: int, k: int, out, stream=None) -> int:
        """rx_mask_noalloc: device output (a uint8 tensor), no allocation."""
        n = C.c_int64()
        check(LIB.rx_mask_noalloc(self.h, float(tau), mode, int(k), _ptr(out), out.numel(), C.byref(n),
                                  _stream_handle(stream)))
        return n.value

    def rx_encode(self, codes, max_out, stream=None) -> int:
        """Transmission codes of the pending scores (codes: int16/uint16
        device tensor, max_out: one-element float32 device tensor)."""
        n = C.c_int64()
        check(LIB.rx_encode(self.h, _ptr(codes), codes.numel(), C.byref(n), _ptr(max_out), _stream_handle(stream)))
        return n.value

    def rx_wait(self, stream=None):
        check(LIB.rx_wait(self.h, _stream_handle(stream)))

    def rx_sync(self, allow=()) -> int:
        return check(LIB.rx_sync(self.h), allow=allow)

    def rx_get_counters(self) -> rx_counters:
        c = rx_counters()
        check(LIB.rx_get_counters(self.h, C.byref(c)))
        return c

    def rx_get_stats(self):
        n = C.c_int64()
        mean = np.zeros(self.B)
        cov = np.zeros((self.B, self.B))
        check(LIB.rx_get_stats(self.h, C.byref(n), mean.ctypes.data, cov.ctypes.data))
        return n.value, mean, cov

    def rx_set_stats(self, n: int, mean: np.ndarray, cov: np.ndarray):
        mean = np.ascontiguousarray(mean, dtype=np.float64)
        cov = np.ascontiguousarray(cov, dtype=np.float64)
        check(LIB.rx_set_stats(self.h, int(n), mean.ctypes.data, cov.ctypes.data))

    def rx_get_whitener(self) -> np.ndarray:
        w = np.zeros((self.B, self.B))
        check(LIB.rx_get_whitener(self.h, w.ctypes.data))
        return w

    def rx_profile(self, enable: bool):
        check(LIB.rx_profile(self.h, int(enable)))

    def rx_phase_times(self):
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.int64)
        check(LIB.rx_phase_times(self.h, ms.ctypes.data, n.ctypes.data))
        return ms, n

    def rx_destroy(self):
        if self.h:
            check(LIB.rx_destroy(self.h))
            self.h = None

    # -- conveniences for tests and the benchmark
    def pending(self) -> int:
        return self.rx_get_counters().pending_px

    def scores_host(self, f64: bool = False) -> np.ndarray:
        n = self.pending()
        out = np.empty(n, dtype=np.float64 if f64 else np.float32)
        got = self.rx_scores(out)
        assert got == n
        return out

    def mask_host(self, tau: float, mode: int = RX_THR_ABS, k: int = 0) -> np.ndarray:
        n = self.pending()
        out = np.zeros((n + 7) // 8, dtype=np.uint8)
        self.rx_mask(tau, mode, k, out)
        return np.unpackbits(out, bitorder="little")[:n].astype(bool)

    def __del__(self):
        try:
            self.rx_destroy()
        except Exception:
            pass


class RxServer:
    """Many streams on one GPU (rx_server_create ... rx_server_destroy)."""

    def __init__(self, hbm_budget_bytes: int, max_streams: int, device: int = 0):
        h = C.c_void_p()
        check(LIB.rx_server_create(int(hbm_budget_bytes), int(max_streams), int(device), C.byref(h)))
        self.h = h

    def rx_server_submit(self, stream: RxStream, lines_dev, tag: int):
        check(LIB.rx_server_submit(self.h, stream.h, _ptr(lines_dev), lines_dev.shape[0], int(tag)))

    def rx_server_step(self) -> int:
        n = C.c_int32()
        check(LIB.rx_server_step(self.h, C.byref(n)))
        return n.value

    def rx_server_poll(self, block: bool = False, max_tags: int = 4096) -> list:
        tags = np.zeros(max_tags, dtype=np.uint64)
        n = C.c_int32()
        check(LIB.rx_server_poll(self.h, tags.ctypes.data, max_tags, C.byref(n), int(block)))
        return tags[: n.value].tolist()

    def rx_server_sync(self):
        check(LIB.rx_server_sync(self.h))

    def rx_server_start(self):
        check(LIB.rx_server_start(self.h))

    def rx_server_stop(self):
        check(LIB.rx_server_stop(self.h))

    def rx_server_poll_ns(self, block: bool = False, max_tags: int = 4096):
        """Finished blocks as (tags, completion stamps in ns of clock_ns())."""
        tags = np.zeros(max_tags, dtype=np.uint64)
        ts = np.zeros(max_tags, dtype=np.int64)
        n = C.c_int32()
        check(LIB.rx_server_poll_ns(self.h, tags.ctypes.data, ts.ctypes.data, max_tags, C.byref(n), int(block)))
        return tags[: n.value].tolist(), ts[: n.value].tolist()

    def rx_server_queued(self):
        q, f, u = C.c_int32(), C.c_int32(), C.c_size_t()
        check(LIB.rx_server_queued(self.h, C.byref(q), C.byref(f), C.byref(u)))
        return q.value, f.value, u.value

    def rx_server_destroy(self):
        if self.h:
            check(LIB.rx_server_destroy(self.h))
            self.h = None


def stream_footprint(cfg: rx_config, max_block_lines: int) -> int:
    b = C.c_size_t()
    check(LIB.rx_stream_footprint(C.byref(cfg), int(max_block_lines), C.byref(b)))
    return b.value


def tx_encode(scores, codes, max_out, stream=None) -> None:
    """rx_tx_encode on device tensors: scores float32 [n], codes int16/uint16
    [n] (binary16 bit patterns), max_out float32 [1]."""
    check(LIB.rx_tx_encode(_ptr(scores), scores.numel(), _ptr(codes), _ptr(max_out), _stream_handle(stream)))


def tx_decode(codes, max_in, tau: float, delta=None, bits=None, stream=None) -> None:
    """rx_tx_decode on device tensors: delta float32 [n] and bits int32
    [ceil(n/32)] are optional outputs."""
    check(LIB.rx_tx_decode(_ptr(codes), codes.numel(), _ptr(max_in), float(tau),
                           _ptr(delta) if delta is not None else None,
                           _ptr(bits) if bits is not None else None, _stream_handle(stream)))


def bin_bands(cube, b0: int, nb: int, k: int, out, bit_depth: int = 12, stream=None) -> None:
    """rx_bin_bands on device tensors: cube uint16-valued [lines][bands][samples]
    (torch int16 or uint16), out [lines][nb / k][samples] of the same dtype."""
    lines, bands, samples = cube.shape
    check(LIB.rx_bin_bands(_ptr(cube), lines, bands, samples, b0, nb, k, bit_depth, _ptr(out),
                           _stream_handle(stream)))


def split_plan(cfg: rx_config, lines: int):
    """(splits, most chunks in one split) of the covariance product for a
    block of `lines` lines under cfg (host-only query, no device work)."""
    ks, mc = C.c_int32(0), C.c_int64(0)
    check(LIB.rx_split_plan(C.byref(cfg), lines, C.byref(ks), C.byref(mc)))
    return ks.value, mc.value


def clock_ns() -> int:
    """The library's monotonic clock (ns), the time base of rx_server_poll_ns."""
    return int(LIB.rx_clock_ns())
