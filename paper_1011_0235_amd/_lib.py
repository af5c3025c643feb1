"""ctypes binding of libhistmi.so (argument marshalling only; every count is made by the HIP kernels).

Device buffers are passed as torch tensors (their data_ptr) or raw integer addresses;
streams as torch.cuda.Stream or a raw hipStream_t integer.  The library must have been
built (``python paper_1011_0235_amd/build.py`` or ``__graft_entry__.build()``); loading
fails loudly otherwise.
"""

from __future__ import annotations

import ctypes
import itertools
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhistmi.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EBUSY, EDEVICE, ENOTSUP, ETIMEDOUT, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7, -8
MODE_AUTO, MODE_AHIST, MODE_WAVEHIST, MODE_WAVEAGG = 0, 1, 2, 3
CRIT_MAXBIN, CRIT_COLLISION, CRIT_BOTH = 0, 1, 2
PAT_IDENTITY, PAT_PAPER960, PAT_FLAT = 0, 1, 2
S_MAX = 16384
RMAX_MAX = 64
AUTO_FLAT_R = 32

c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_u8p = ctypes.POINTER(ctypes.c_uint8)


class HistError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, strerror(status), status))


class Pattern(ctypes.Structure):
    _fields_ = [("word", ctypes.c_uint32 * 256), ("total_S", ctypes.c_uint32), ("rmax", ctypes.c_uint32)]

    @classmethod
    def from_words(cls, words: Sequence[int], S: int, rmax: int) -> "Pattern":
        p = cls()
        for i, w in enumerate(words):
            p.word[i] = int(w)
        p.total_S = int(S)
        p.rmax = int(rmax)
        return p

    def words(self):
        return [int(x) for x in self.word]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("cu_count", ctypes.c_int), ("clock_khz", ctypes.c_int),
                ("lds_per_cu", ctypes.c_size_t), ("hbm_bytes", ctypes.c_size_t), ("arch", ctypes.c_char * 32)]


class StreamConfig(ctypes.Structure):
    _fields_ = [("W", ctypes.c_uint32), ("theta_pct", ctypes.c_uint32), ("S", ctypes.c_uint32),
                ("rmax", ctypes.c_uint32), ("lag", ctypes.c_uint32), ("trace_cap", ctypes.c_uint32),
                ("alarm_pct", ctypes.c_uint32), ("criterion", ctypes.c_uint32), ("kappa_pct", ctypes.c_uint32)]


class IngestConfig(ctypes.Structure):
    _fields_ = [("n_hip_streams", ctypes.c_uint32), ("slot_bytes", ctypes.c_uint64)]


class StreamSnapshot(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_uint64), ("acc", ctypes.c_uint64 * 256), ("mw", ctypes.c_uint64 * 256),
                ("next_mode", ctypes.c_uint32), ("next_pattern", Pattern), ("alarms", ctypes.c_uint64),
                ("first_alarm", ctypes.c_uint64), ("last_alarm", ctypes.c_uint64),
                ("wait_timeouts", ctypes.c_uint64), ("merge_timeouts", ctypes.c_uint64)]


class Diag(ctypes.Structure):
    _fields_ = [("invalid_patterns", ctypes.c_uint64), ("wait_timeouts", ctypes.c_uint64),
                ("merge_timeouts", ctypes.c_uint64)]


class Tune(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_uint32), ("tile_kib", ctypes.c_uint32), ("merge_copies", ctypes.c_uint32),
                ("tiles_per_wg", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("n_stream_ids", ctypes.c_uint32), ("n_hip_streams", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("theta_pct", ctypes.c_uint32),
                ("S", ctypes.c_uint32), ("rmax", ctypes.c_uint32), ("idle_spin_us", ctypes.c_uint32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("stream_id", ctypes.c_uint32), ("bytes", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("bytes_done", ctypes.c_uint64), ("max_inflight_bytes", ctypes.c_uint64),
                ("max_inflight_requests", ctypes.c_uint64), ("max_concurrent_batches", ctypes.c_uint64),
                ("max_launch_ns", ctypes.c_uint64), ("max_query_ns", ctypes.c_uint64)]


# (name, restype, argtypes) of every symbol include/histmi.h declares
_VP = ctypes.c_void_p
_SIGS = [
    ("hist_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("hist_device_info", ctypes.c_int, [ctypes.POINTER(DeviceInfo)]),
    ("hist_u8", ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_int, ctypes.POINTER(Pattern), _VP]),
    ("hist_u8_u64", ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_int, ctypes.POINTER(Pattern), _VP]),
    ("hist_u8_noalloc", ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_int, ctypes.POINTER(Pattern), _VP]),
    ("hist_pattern_init", ctypes.c_int, [ctypes.POINTER(Pattern), ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]),
    ("hist_pattern_validate", ctypes.c_int, [ctypes.POINTER(Pattern)]),
    ("hist_pattern_update", ctypes.c_int, [_VP, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP]),
    ("hist_stream_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(StreamConfig)]),
    ("hist_stream_push", ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_int, _VP, _VP]),
    ("hist_stream_push_many", ctypes.c_int, [_VP, ctypes.POINTER(_VP), c_u64p, ctypes.c_uint32, ctypes.c_int, _VP, _VP]),
    ("hist_stream_read", ctypes.c_int, [_VP, ctypes.POINTER(StreamSnapshot), c_u8p, c_u32p, ctypes.c_uint32, _VP]),
    ("hist_stream_read_alarms", ctypes.c_int, [_VP, c_u8p, ctypes.c_uint32, _VP]),
    ("hist_stream_read_times", ctypes.c_int, [_VP, c_u64p, ctypes.c_uint32, _VP]),
    ("hist_stream_destroy", ctypes.c_int, [_VP]),
    ("hist_batch", ctypes.c_int, [ctypes.POINTER(_VP), c_u64p, ctypes.c_uint32, _VP, ctypes.c_int,
                                  ctypes.POINTER(Pattern), _VP]),
    ("hist_batch_graph_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(_VP), c_u64p, ctypes.c_uint32, _VP,
                                               ctypes.c_int, ctypes.POINTER(Pattern)]),
    ("hist_batch_graph_launch", ctypes.c_int, [_VP, _VP]),
    ("hist_batch_graph_destroy", ctypes.c_int, [_VP]),
    ("hist_diag_read", ctypes.c_int, [ctypes.POINTER(Diag)]),
    ("hist_read_probe", ctypes.c_int, [_VP, ctypes.c_size_t, _VP, ctypes.c_uint32, _VP]),
    ("hist_set_wait_limits", ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32]),
    ("hist_tune_set", ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(Tune)]),
    ("hist_tune_get", ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(Tune)]),
    ("hist_ingest_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(IngestConfig)]),
    ("hist_ingest_push", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_size_t, ctypes.c_int, _VP]),
    ("hist_ingest_sync", ctypes.c_int, [_VP]),
    ("hist_ingest_destroy", ctypes.c_int, [_VP]),
    ("hist_server_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(ServerConfig)]),
    ("hist_server_submit", ctypes.c_int, [_VP, ctypes.c_uint32, _VP, ctypes.c_size_t, _VP, c_u64p]),
    ("hist_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ServerResult)]),
    ("hist_server_wait", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ServerResult)]),
    ("hist_server_drain", ctypes.c_int, [_VP, ctypes.c_int64]),
    ("hist_server_stream_acc", ctypes.c_int, [_VP, ctypes.c_uint32, c_u64p]),
    ("hist_server_stats", ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    ("hist_server_destroy", ctypes.c_int, [_VP]),
]

_lib = None


def declared_symbols():
    return [name for name, _, _ in _SIGS]


TUNING_PATH = os.path.join(HERE, "tuning.json")
_FAMILIES = {"wavehist": 0, "uniform": 1, "lookup": 2, "waveagg": 3, "stream": 4, "stream_known": 5}
TUNE_STREAM = 4
TUNE_STREAM_KNOWN = 5


def apply_tuning(path: str = TUNING_PATH):
    """Apply the launch shapes an autotuner run wrote (no-op if there is none)."""
    import json
    if not os.path.exists(path):
        return
    with open(path) as f:
        t = json.load(f)
    for name, fam in t.get("families", {}).items():
        if name in _FAMILIES:
            tune_set(_FAMILIES[name], int(fam.get("blocks_per_cu", 0)), int(fam.get("tile_kib", 0)),
                     int(fam.get("merge_copies", 0)), int(fam.get("tiles_per_wg", 0)))


def load(path: Optional[str] = None, apply_tuning: bool = True):
    """Load libhistmi.so (once).  Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libhistmi.so is not built (%s); run python paper_1011_0235_amd/build.py" % p)
    # PyTorch ships its own HIP runtime.  Imported first, it provides the runtime this library
    # then binds to (same soname), so both share one; loaded the other way round, the
    # process gets ROCm's runtime under PyTorch's name and device calls fail.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    if apply_tuning:
        globals()["apply_tuning"]()
    return lib


def strerror(status: int) -> str:
    if _lib is None:
        return "status %d" % status
    return _lib.hist_strerror(int(status)).decode()


def _check(status: int, what: str):
    if status != OK:
        raise HistError(status, what)


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(s) -> int:
    if s is None:
        try:
            import torch
            return int(torch.cuda.current_stream().cuda_stream)
        except Exception:
            return 0
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _nbytes(x) -> int:
    return int(x.numel() * x.element_size())


def _in_bytes(d_in, n: Optional[int]) -> int:
    """Bytes to read from d_in: all of a tensor, or n; an n beyond a tensor's bytes is refused
    (the kernel would read past the allocation)."""
    if isinstance(d_in, int) or d_in is None:
        if n is None:
            raise ValueError("a raw address needs an explicit byte count n")
        return int(n)
    nb = _nbytes(d_in)
    if n is None:
        return nb
    if int(n) < 0 or int(n) > nb:
        raise ValueError("n = %d exceeds the input tensor's %d bytes" % (int(n), nb))
    if not d_in.is_contiguous():
        raise ValueError("the input tensor must be contiguous")
    return int(n)


def _check_out(d_out, words: int, elem_bytes: int = 4, what: str = "d_out"):
    """A tensor output must be contiguous, of elem_bytes-byte elements, and hold at least
    `words` of them (raw addresses are the caller's responsibility)."""
    if d_out is None or isinstance(d_out, int):
        return
    if d_out.element_size() != elem_bytes:
        raise ValueError("%s must have %d-byte elements" % (what, elem_bytes))
    if not d_out.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if d_out.numel() < words:
        raise ValueError("%s holds %d elements, needs at least %d" % (what, d_out.numel(), words))


# ---------------------------------------------------------------- patterns (host)

def pattern_init(kind: int, S: int = 0, rmax: int = 0) -> Pattern:
    p = Pattern()
    _check(load().hist_pattern_init(ctypes.byref(p), int(kind), int(S), int(rmax)), "hist_pattern_init")
    return p


def pattern_validate(p: Pattern) -> int:
    return load().hist_pattern_validate(ctypes.byref(p))


def pattern_update(d_hist, S: int, rmax: int, d_pat, stream=None):
    """Rule P on the device: d_hist uint64[256] (int64 tensor) -> d_pat (int32 tensor of 258 words)."""
    _check(load().hist_pattern_update(_ptr(d_hist), int(S), int(rmax), _ptr(d_pat), _stream(stream)),
           "hist_pattern_update")


# ---------------------------------------------------------------- single histograms

def hist_u8(d_in, d_out, mode: int = MODE_AUTO, pattern: Optional[Pattern] = None, stream=None, n: Optional[int] = None):
    """d_out (int32/uint32 tensor of 256, device) <- histogram of the bytes of d_in."""
    nb = _in_bytes(d_in, n)
    _check_out(d_out, 256)
    st = load().hist_u8(_ptr(d_in), nb, _ptr(d_out), int(mode), ctypes.byref(pattern) if pattern is not None else None,
                        _stream(stream))
    _check(st, "hist_u8")


def hist_u8_noalloc(d_in, d_out, mode: int = MODE_AUTO, pattern: Optional[Pattern] = None, stream=None,
                    n: Optional[int] = None):
    """hist_u8 on the library's fixed per-device scratch array: allocates no device memory.
    Calls that overlap on one device race (they share that array)."""
    nb = _in_bytes(d_in, n)
    _check_out(d_out, 256)
    st = load().hist_u8_noalloc(_ptr(d_in), nb, _ptr(d_out), int(mode),
                                ctypes.byref(pattern) if pattern is not None else None, _stream(stream))
    _check(st, "hist_u8_noalloc")


def hist_u8_u64(d_in, d_acc, mode: int = MODE_AUTO, pattern: Optional[Pattern] = None, stream=None,
                n: Optional[int] = None):
    nb = _in_bytes(d_in, n)
    _check_out(d_acc, 256, 8, "d_acc")
    st = load().hist_u8_u64(_ptr(d_in), nb, _ptr(d_acc), int(mode),
                            ctypes.byref(pattern) if pattern is not None else None, _stream(stream))
    _check(st, "hist_u8_u64")


def read_probe(d_in, d_sum, workgroups: int = 0, stream=None, n: Optional[int] = None):
    """Streaming read of d_in (HBM read roofline); adds its uint32 words to d_sum[0] (uint64)."""
    nb = _in_bytes(d_in, n)
    _check_out(d_sum, 1, 8, "d_sum")
    _check(load().hist_read_probe(_ptr(d_in), nb, _ptr(d_sum), int(workgroups), _stream(stream)),
           "hist_read_probe")


def _ptr_arrays(bufs) -> Tuple[np.ndarray, np.ndarray]:
    """Device addresses and byte counts as uint64 arrays, from an (n, 2) integer array of
    (address, nbytes) rows, a sequence of (address, nbytes) pairs, or a sequence of device
    tensors (mixed with pairs).  Arrays and pairs are converted without a per-item Python
    loop, so that marshalling thousands of buffers stays well below a launch's duration."""
    if isinstance(bufs, np.ndarray):
        if bufs.ndim != 2 or bufs.shape[1] != 2 or bufs.dtype.kind not in "iu":
            raise ValueError("an array of buffers must be (n, 2) integers: address, nbytes")
        if bufs.dtype.kind == "i" and bufs.size and int(bufs.min()) < 0:
            raise ValueError("buffer addresses and sizes must be non-negative")
        a = bufs.astype(np.uint64, copy=False)
        return np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1])
    n = len(bufs)
    if all(type(b) is tuple and len(b) == 2 for b in bufs):
        a = np.fromiter(itertools.chain.from_iterable(bufs), dtype=np.uint64, count=2 * n).reshape(n, 2)
        return np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1])
    ptrs = np.zeros(n, dtype=np.uint64)
    sizes = np.zeros(n, dtype=np.uint64)
    for i, b in enumerate(bufs):
        if isinstance(b, tuple):
            ptrs[i] = int(b[0])
            sizes[i] = int(b[1])
        else:
            ptrs[i] = _ptr(b)
            sizes[i] = _nbytes(b)
    return ptrs, sizes


def _vpp(a: np.ndarray):
    """A uint64 address array as the C side's `const void *const *`."""
    return a.ctypes.data_as(ctypes.POINTER(_VP))


def hist_batch(bufs, d_out, mode: int = MODE_AUTO, pattern: Optional[Pattern] = None, stream=None):
    """bufs: device tensors or (address, nbytes) pairs, or an (n, 2) integer array of such rows;
    d_out: int32 [n, 256] device tensor."""
    ptrs, sizes = _ptr_arrays(bufs)
    _check_out(d_out, 256 * len(ptrs))
    st = load().hist_batch(_vpp(ptrs), sizes.ctypes.data_as(c_u64p), len(ptrs), _ptr(d_out), int(mode),
                           ctypes.byref(pattern) if pattern is not None else None, _stream(stream))
    _check(st, "hist_batch")


class BatchGraph:
    """A batch captured once into a HIP graph; launch() recomputes every histogram."""

    def __init__(self, bufs, d_out, mode: int = MODE_AUTO, pattern: Optional[Pattern] = None):
        ptrs, sizes = _ptr_arrays(bufs)
        _check_out(d_out, 256 * len(ptrs))
        self._h = ctypes.c_void_p()
        st = load().hist_batch_graph_create(ctypes.byref(self._h), _vpp(ptrs), sizes.ctypes.data_as(c_u64p), len(ptrs),
                                            _ptr(d_out), int(mode),
                                            ctypes.byref(pattern) if pattern is not None else None)
        _check(st, "hist_batch_graph_create")

    def launch(self, stream=None):
        _check(load().hist_batch_graph_launch(self._h, _stream(stream)), "hist_batch_graph_launch")

    def close(self):
        if self._h:
            load().hist_batch_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- streams

class Stream:
    """A device-resident histogram stream (Accumulator, moving window, adaptive kernel switch)."""

    def __init__(self, W: int = 1, theta_pct: int = 45, S: int = 960, rmax: int = 8, lag: int = 0,
                 trace_cap: int = 1024, alarm_pct: int = 0, criterion: int = 0, kappa_pct: int = 0):
        cfg = StreamConfig(W, theta_pct, S, rmax, lag, trace_cap, alarm_pct, criterion, kappa_pct)
        self.cfg = cfg
        self._h = ctypes.c_void_p()
        _check(load().hist_stream_create(ctypes.byref(self._h), ctypes.byref(cfg)), "hist_stream_create")

    def push(self, d_chunk, mode: int = MODE_AUTO, d_out=None, stream=None, n: Optional[int] = None):
        nb = _in_bytes(d_chunk, n)
        _check_out(d_out, 256)
        _check(load().hist_stream_push(self._h, _ptr(d_chunk), nb, int(mode), _ptr(d_out), _stream(stream)),
               "hist_stream_push")

    def push_many(self, chunks, mode: int = MODE_AUTO, d_out=None, stream=None):
        ptrs, sizes = _ptr_arrays(chunks)
        _check_out(d_out, 256 * len(ptrs))
        _check(load().hist_stream_push_many(self._h, _vpp(ptrs), sizes.ctypes.data_as(c_u64p), len(ptrs), int(mode),
                                            _ptr(d_out), _stream(stream)), "hist_stream_push_many")

    def read(self, trace_len: int = 0, stream=None, allow_timeouts: bool = False):
        """(snapshot, mode trace, pattern trace).  A bounded wait that gave up raises
        HistError(ETIMEDOUT) unless allow_timeouts (the snapshot then says how many)."""
        snap = StreamSnapshot()
        modes = np.zeros(max(trace_len, 1), dtype=np.uint8)
        pats = np.zeros((max(trace_len, 1), 256), dtype=np.uint32)
        st = load().hist_stream_read(self._h, ctypes.byref(snap), modes.ctypes.data_as(c_u8p),
                                     pats.ctypes.data_as(c_u32p), int(trace_len), _stream(stream))
        if not (allow_timeouts and st == ETIMEDOUT):
            _check(st, "hist_stream_read")
        return snap, modes[:trace_len], pats[:trace_len]

    def read_alarms(self, trace_len: int, stream=None) -> np.ndarray:
        """Change detection trace: entry k is 1 iff an alarm was raised after chunk k."""
        out = np.zeros(max(trace_len, 1), dtype=np.uint8)
        _check(load().hist_stream_read_alarms(self._h, out.ctypes.data_as(c_u8p), int(trace_len), _stream(stream)),
               "hist_stream_read_alarms")
        return out[:trace_len]

    def read_times(self, trace_len: int, stream=None) -> np.ndarray:
        """Device timeline of the traced chunks: uint64[trace_len, 3] = (ns when the first
        workgroup began counting chunk k, ns when its decision was ready, the shader cycle
        counter's rate in ticks per us inside its finalizer); 0 where not traced or not run."""
        out = np.zeros((max(trace_len, 1), 3), dtype=np.uint64)
        _check(load().hist_stream_read_times(self._h, out.ctypes.data_as(c_u64p), int(trace_len), _stream(stream)),
               "hist_stream_read_times")
        return out[:trace_len]

    def close(self):
        if self._h:
            load().hist_stream_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ingest:
    """Host-ingest pipeline: pushes chunks that live in host memory (pinned for asynchronous
    copies) through device streams, copies overlapping counting over n_hip_streams HIP streams."""

    def __init__(self, n_hip_streams: int = 4, slot_bytes: int = 4 << 20):
        cfg = IngestConfig(n_hip_streams, slot_bytes)
        self.cfg = cfg
        self._h = ctypes.c_void_p()
        _check(load().hist_ingest_create(ctypes.byref(self._h), ctypes.byref(cfg)), "hist_ingest_create")

    def push(self, stream: "Stream", h_chunk, mode: int = MODE_AUTO, d_out=None, n: Optional[int] = None):
        """h_chunk: a host tensor / numpy array / host address (must stay valid until sync)."""
        if isinstance(h_chunk, np.ndarray):
            ptr, nb = int(h_chunk.ctypes.data), int(h_chunk.nbytes)
            if n is not None and not 0 <= int(n) <= nb:
                raise ValueError("n = %d exceeds the host chunk's %d bytes" % (int(n), nb))
            nb = nb if n is None else int(n)
        else:
            ptr, nb = _ptr(h_chunk), _in_bytes(h_chunk, n)
        _check_out(d_out, 256)
        _check(load().hist_ingest_push(self._h, stream._h, ptr, nb, int(mode), _ptr(d_out)), "hist_ingest_push")

    def sync(self):
        _check(load().hist_ingest_sync(self._h), "hist_ingest_sync")

    def close(self):
        if self._h:
            load().hist_ingest_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- diagnostics / tuning / device

def diag() -> Diag:
    d = Diag()
    _check(load().hist_diag_read(ctypes.byref(d)), "hist_diag_read")
    return d


def set_wait_limits(decision_polls: int = 0, merge_polls: int = 0):
    """Bounds of the in-kernel waits of later launches (0 = the library's default)."""
    _check(load().hist_set_wait_limits(int(decision_polls), int(merge_polls)), "hist_set_wait_limits")


def tune_get(family: int) -> Tune:
    t = Tune()
    _check(load().hist_tune_get(int(family), ctypes.byref(t)), "hist_tune_get")
    return t


def tune_set(family: int, blocks_per_cu: int = 0, tile_kib: int = 0, merge_copies: int = 0, tiles_per_wg: int = 0):
    t = Tune(blocks_per_cu, tile_kib, merge_copies, tiles_per_wg)
    _check(load().hist_tune_set(int(family), ctypes.byref(t)), "hist_tune_set")


def device_info() -> DeviceInfo:
    d = DeviceInfo()
    _check(load().hist_device_info(ctypes.byref(d)), "hist_device_info")
    return d


# ---------------------------------------------------------------- server

class Server:
    """Continuous-batching request server (see hist_server_* in include/histmi.h)."""

    def __init__(self, hbm_budget_bytes: int = 1 << 30, max_slots: int = 256, n_stream_ids: int = 64,
                 n_hip_streams: int = 4, max_batch: int = 64, mode: int = MODE_AUTO, theta_pct: int = 45,
                 S: int = 8192, rmax: int = 32, idle_spin_us: int = 0):
        cfg = ServerConfig(int(hbm_budget_bytes), max_slots, n_stream_ids, n_hip_streams, max_batch, mode, theta_pct,
                           S, rmax, idle_spin_us)
        self.cfg = cfg
        self._h = ctypes.c_void_p()
        _check(load().hist_server_create(ctypes.byref(self._h), ctypes.byref(cfg)), "hist_server_create")

    def submit(self, stream_id: int, d_buf, d_out=None, n: Optional[int] = None) -> int:
        nb = _in_bytes(d_buf, n)
        _check_out(d_out, 256)
        t = ctypes.c_uint64()
        _check(load().hist_server_submit(self._h, int(stream_id), _ptr(d_buf), nb, _ptr(d_out), ctypes.byref(t)),
               "hist_server_submit")
        return int(t.value)

    def try_submit(self, stream_id: int, d_buf, d_out=None, n: Optional[int] = None):
        """(status, ticket) without raising on a library status (argument errors still raise)."""
        nb = _in_bytes(d_buf, n)
        _check_out(d_out, 256)
        t = ctypes.c_uint64()
        st = load().hist_server_submit(self._h, int(stream_id), _ptr(d_buf), nb, _ptr(d_out), ctypes.byref(t))
        return st, int(t.value)

    def poll(self, ticket: int) -> ServerResult:
        r = ServerResult()
        _check(load().hist_server_poll(self._h, int(ticket), ctypes.byref(r)), "hist_server_poll")
        return r

    def wait(self, ticket: int, timeout_ns: int = -1) -> ServerResult:
        r = ServerResult()
        _check(load().hist_server_wait(self._h, int(ticket), int(timeout_ns), ctypes.byref(r)), "hist_server_wait")
        return r

    def drain(self, timeout_ns: int = -1):
        _check(load().hist_server_drain(self._h, int(timeout_ns)), "hist_server_drain")

    def stream_acc(self, stream_id: int) -> np.ndarray:
        out = np.zeros(256, dtype=np.uint64)
        _check(load().hist_server_stream_acc(self._h, int(stream_id), out.ctypes.data_as(c_u64p)),
               "hist_server_stream_acc")
        return out

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(load().hist_server_stats(self._h, ctypes.byref(s)), "hist_server_stats")
        return s

    def close(self):
        if self._h:
            load().hist_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
