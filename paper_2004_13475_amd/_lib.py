"""ctypes binding of libfractal.so (argument marshalling only).

Every function forwards to the C entry point of the same name in
include/fractal.h; all computation happens in the library's HIP kernels.
Device buffers are passed as torch tensors (or raw integer addresses) and
streams as torch streams, raw hipStream_t integers or None (torch's current
stream).  A missing library is an error: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfractal.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_AGAIN = 0, 1, 2, 3, 4
RULE_CA, RULE_HEAT = 0, 1
NBB_GASKET, NBB_CARPET, NBB_VICSEK, NBB_XFRACTAL, NBB_HFRACTAL, NBB_CANTOR = range(6)
ORDER_NATURAL, ORDER_CURVE, ORDER_CURVE_XCD = 0, 1, 2
FLAG_SEGMENTS, FLAG_NT_STORE, FLAG_PERSISTENT, FLAG_FUSE2, FLAG_FUSE4 = 1, 2, 4, 8, 16
FLAG_MARCH, FLAG_FUSE8, FLAG_FUSE16 = 32, 64, 128
FLAG_STACK2, FLAG_STACK4, FLAG_STACK8 = 256, 512, 1024
FLAG_OCC_ALT = 2048
FLAG_BLOCK = 4096
FLAG_FUSE24, FLAG_FUSE32, FLAG_FUSE36 = 8192, 16384, 32768
MAP_LAMBDA, MAP_BB, MAP_MFMA = 0, 1, 2
R_AUTO = -1

EXPORTED = [
    "fractal_grid_dims", "fractal_lambda_map", "fractal_lambda_map_mfma",
    "fractal_lambda_map_tiles", "fractal_seed_fill", "fractal_bb_step", "fractal_lambda_step",
    "fractal_lambda_step_mfma", "fractal_step_tuned", "fractal_autotune",
    "fractal_get_tuning", "fractal_set_tuning", "fractal_tuning_save", "fractal_tuning_load",
    "fractal_batch_workspace", "fractal_batch_step",
    "fractal_single_write", "fractal_reduce_workspace", "fractal_reduce",
    "fractal_reduce_noalloc", "fractal_compact_bytes", "fractal_pack", "fractal_unpack", "fractal_compact_seed_fill",
    "fractal_compact_step", "fractal_nbb_builtin", "fractal_nbb_lambda_map",
    "fractal_nbb_single_write", "fractal_nbb_reduce_workspace", "fractal_nbb_reduce",
    "fractal_nbb_ca_step",
    "fractal_now", "fractal_serve_create", "fractal_serve_set_steps_per_iter", "fractal_serve_submit",
    "fractal_serve_poll", "fractal_serve_stats", "fractal_serve_destroy", "fractal_last_error",
]


class FractalError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfractal error {code}: {msg}")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("threads", ctypes.c_int),
                ("order", ctypes.c_int), ("flags", ctypes.c_int)]

    def as_tuple(self):
        return (self.r, self.threads, self.order, self.flags)


class Nbb(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("s", ctypes.c_int),
                ("tau_x", ctypes.c_uint8 * 32), ("tau_y", ctypes.c_uint8 * 32)]

    def replicas(self):
        return [(self.tau_x[i], self.tau_y[i]) for i in range(self.k)]


class Instance(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("rule", ctypes.c_int),
                ("steps", ctypes.c_int), ("alpha", ctypes.c_float),
                ("d_buf0", ctypes.c_void_p), ("d_buf1", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("rule", ctypes.c_int),
                ("steps", ctypes.c_int), ("alpha", ctypes.c_float),
                ("seed", ctypes.c_uint32), ("h_init", ctypes.c_void_p),
                ("h_out", ctypes.c_void_p), ("t_arrival", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("reserved", ctypes.c_int),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("checksum", ctypes.c_uint64)]


class ServeReport(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("p50_latency", ctypes.c_double),
                ("p99_latency", ctypes.c_double), ("mean_latency", ctypes.c_double),
                ("cell_updates", ctypes.c_double), ("t_first_arrival", ctypes.c_double),
                ("t_last_done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Load libfractal.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with paper_2004_13475_amd.build "
            "(or __graft_entry__.build()); there is no non-HIP fallback")
    # torch carries its own copy of the HIP runtime, whose file name differs
    # from the system one the library is linked against: loaded first, torch's
    # copy satisfies the library's dependency, while loading the library
    # first would put two HIP runtimes in the process (the second one to
    # start then finds no device).  So torch, when present, is imported first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    i, u32, f, vp = ctypes.c_int, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p
    pu32 = ctypes.POINTER(u32)
    sig = {
        "fractal_grid_dims": ([i, i, pu32, pu32], i),
        "fractal_lambda_map": ([i, i, vp, vp], i),
        "fractal_lambda_map_mfma": ([i, i, vp, vp], i),
        "fractal_lambda_map_tiles": ([i, i, i, vp, vp], i),
        "fractal_seed_fill": ([i, i, u32, vp, vp], i),
        "fractal_bb_step": ([i, i, i, f, vp, vp, i, vp], i),
        "fractal_lambda_step": ([i, i, i, f, vp, vp, i, vp], i),
        "fractal_lambda_step_mfma": ([i, i, i, f, vp, vp, i, vp], i),
        "fractal_step_tuned": ([i, i, i, f, vp, vp, i, ctypes.POINTER(Tuning), vp], i),
        "fractal_autotune": ([i, i, f, vp, vp, vp, ctypes.POINTER(Tuning)], i),
        "fractal_get_tuning": ([i, i, ctypes.POINTER(Tuning)], i),
        "fractal_set_tuning": ([i, i, ctypes.POINTER(Tuning)], i),
        "fractal_tuning_save": ([ctypes.c_char_p], i),
        "fractal_tuning_load": ([ctypes.c_char_p], i),
        "fractal_batch_workspace": ([i, ctypes.POINTER(ctypes.c_size_t)], i),
        "fractal_batch_step": ([ctypes.POINTER(Instance), i, ctypes.POINTER(Tuning), vp,
                                ctypes.c_size_t, vp], i),
        "fractal_single_write": ([i, i, i, i, u32, vp, vp], i),
        "fractal_reduce_workspace": ([i, i, ctypes.POINTER(ctypes.c_size_t)], i),
        "fractal_reduce": ([i, i, i, i, vp, vp, ctypes.c_size_t, vp, vp], i),
        "fractal_reduce_noalloc": ([i, i, i, i, vp, vp, vp], i),
        "fractal_compact_bytes": ([i, i, i, ctypes.POINTER(ctypes.c_size_t)], i),
        "fractal_pack": ([i, i, i, vp, vp, vp], i),
        "fractal_unpack": ([i, i, i, vp, vp, vp], i),
        "fractal_compact_seed_fill": ([i, i, i, u32, vp, vp], i),
        "fractal_compact_step": ([i, i, i, f, vp, vp, i, i, vp], i),
        "fractal_nbb_builtin": ([i, ctypes.POINTER(Nbb)], i),
        "fractal_nbb_lambda_map": ([ctypes.POINTER(Nbb), i, vp, vp], i),
        "fractal_nbb_single_write": ([ctypes.POINTER(Nbb), i, i, i, u32, vp, vp], i),
        "fractal_nbb_reduce_workspace": ([ctypes.POINTER(Nbb), i, i, ctypes.POINTER(ctypes.c_size_t)], i),
        "fractal_nbb_reduce": ([ctypes.POINTER(Nbb), i, i, i, vp, vp, ctypes.c_size_t, vp, vp], i),
        "fractal_nbb_ca_step": ([ctypes.POINTER(Nbb), i, i, i, vp, vp, i, vp], i),
        "fractal_now": ([], ctypes.c_double),
        "fractal_serve_create": ([vp, ctypes.c_size_t, i, vp, ctypes.POINTER(vp)], i),
        "fractal_serve_set_steps_per_iter": ([vp, i], i),
        "fractal_serve_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], i),
        "fractal_serve_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(Result)], i),
        "fractal_serve_stats": ([vp, ctypes.POINTER(ServeReport)], i),
        "fractal_serve_destroy": ([vp], i),
        "fractal_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        if not hasattr(lib, name):
            continue  # reported by exported_symbols(); calls raise AttributeError
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    """Names of EXPORTED that the loaded library defines."""
    lib = load()
    return [n for n in EXPORTED if hasattr(lib, n)]


def _check(rc: int):
    if rc != OK:
        msg = load().fractal_last_error().decode(errors="replace")
        raise FractalError(rc, msg)
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def grid_dims(k: int, r: int):
    gx, gy = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().fractal_grid_dims(k, r, ctypes.byref(gx), ctypes.byref(gy)))
    return gx.value, gy.value


def lambda_map(k, r, out, stream=None):
    return _check(load().fractal_lambda_map(k, r, _ptr(out), _stream(stream)))


def lambda_map_mfma(k, r, out, stream=None):
    return _check(load().fractal_lambda_map_mfma(k, r, _ptr(out), _stream(stream)))


def lambda_map_tiles(k, r, order, out, stream=None):
    """The per-lane form of lambda the march kernels use: out[2i], out[2i+1]
    = block of tile id i in dispatch order `order`."""
    return _check(load().fractal_lambda_map_tiles(k, r, order, _ptr(out), _stream(stream)))


def seed_fill(k, rule, stream_id, buf, stream=None):
    return _check(load().fractal_seed_fill(k, rule, stream_id, _ptr(buf), _stream(stream)))


def bb_step(k, r, rule, alpha, buf0, buf1, steps, stream=None):
    return _check(load().fractal_bb_step(k, r, rule, alpha, _ptr(buf0), _ptr(buf1),
                                         steps, _stream(stream)))


def lambda_step(k, r, rule, alpha, buf0, buf1, steps, stream=None):
    return _check(load().fractal_lambda_step(k, r, rule, alpha, _ptr(buf0), _ptr(buf1),
                                             steps, _stream(stream)))


def lambda_step_mfma(k, r, rule, alpha, buf0, buf1, steps, stream=None):
    return _check(load().fractal_lambda_step_mfma(k, r, rule, alpha, _ptr(buf0),
                                                  _ptr(buf1), steps, _stream(stream)))


def step_tuned(map_, k, rule, alpha, buf0, buf1, steps, r, threads, order, flags=0,
               stream=None):
    t = Tuning(r, threads, order, flags)
    return _check(load().fractal_step_tuned(map_, k, rule, alpha, _ptr(buf0), _ptr(buf1),
                                            steps, ctypes.byref(t), _stream(stream)))


def autotune(k, rule, alpha, buf0, buf1, stream=None):
    t = Tuning()
    _check(load().fractal_autotune(k, rule, alpha, _ptr(buf0), _ptr(buf1),
                                   _stream(stream), ctypes.byref(t)))
    return t.as_tuple()


def get_tuning(k, rule):
    t = Tuning()
    _check(load().fractal_get_tuning(k, rule, ctypes.byref(t)))
    return t.as_tuple()


def set_tuning(k, rule, r, threads, order, flags=0):
    t = Tuning(r, threads, order, flags)
    return _check(load().fractal_set_tuning(k, rule, ctypes.byref(t)))


def _nbytes(buf, nbytes, what):
    """Size in bytes of a device buffer: a tensor's own size, else the
    caller's `nbytes` (required for raw addresses)."""
    if hasattr(buf, "numel"):
        size = buf.numel() * buf.element_size()
        return size if nbytes is None else min(size, int(nbytes))
    if nbytes is None:
        raise ValueError(f"{what}: a raw device address needs its size in bytes (nbytes=)")
    return int(nbytes)


def tuning_save(path):
    """Write every cached tuning to a tuning file."""
    return _check(load().fractal_tuning_save(os.fsencode(path)))


def tuning_load(path):
    """Add a tuning file's entries for the current device to the cache."""
    return _check(load().fractal_tuning_load(os.fsencode(path)))


def batch_workspace(count) -> int:
    """Bytes of device workspace batch_step needs for `count` instances."""
    b = ctypes.c_size_t()
    _check(load().fractal_batch_workspace(count, ctypes.byref(b)))
    return b.value


def batch_step(instances, tuning=None, work=None, stream=None, work_bytes=None):
    """instances: list of (k, rule, steps, alpha, buf0, buf1).  `work`: the
    device workspace of batch_workspace(len(instances)) bytes (a tensor, or a
    raw address with its size in `work_bytes`).  When None, a torch tensor
    of that size is allocated on the current device and marked as used by
    the (torch) stream, so torch does not hand its memory out again before
    the batch's work on that stream has run; a raw stream needs an explicit
    workspace."""
    arr = (Instance * len(instances))()
    for j, (k, rule, steps, alpha, b0, b1) in enumerate(instances):
        arr[j] = Instance(k, rule, steps, alpha, _ptr(b0), _ptr(b1))
    tp = None
    if tuning is not None:
        tp = ctypes.byref(Tuning(*tuning) if len(tuning) == 4 else Tuning(*tuning, 0))
    if work is None:
        if isinstance(stream, int):
            raise ValueError("batch_step on a raw stream needs an explicit workspace")
        import torch
        work = torch.empty(max(batch_workspace(len(instances)), 16), dtype=torch.uint8,
                           device="cuda")
        work.record_stream(torch.cuda.current_stream() if stream is None else stream)
    nbytes = _nbytes(work, work_bytes, "batch_step workspace")
    return _check(load().fractal_batch_step(arr, len(instances), tp, _ptr(work), nbytes,
                                            _stream(stream)))


def single_write(map_, k, r, rule, value, buf, stream=None):
    """Test SW: `value` (uint8 low byte / float32 bit pattern) on every
    gasket cell of `buf`."""
    return _check(load().fractal_single_write(map_, k, r, rule, int(value) & 0xFFFFFFFF,
                                              _ptr(buf), _stream(stream)))


def reduce_workspace(k, r) -> int:
    """Bytes of device workspace `reduce` needs."""
    b = ctypes.c_size_t()
    _check(load().fractal_reduce_workspace(k, r, ctypes.byref(b)))
    return b.value


def reduce(map_, k, r, rule, buf, work, out, stream=None, work_bytes=None):
    """Test RD: the sum of the gasket cells of `buf` into the 8-byte device
    buffer `out` (uint64 for uint8 cells, float64 for float32 cells); `work`
    is a device buffer of at least reduce_workspace(k, r) bytes (a tensor,
    or a raw address with its size in `work_bytes`)."""
    nbytes = _nbytes(work, work_bytes, "reduce workspace")
    return _check(load().fractal_reduce(map_, k, r, rule, _ptr(buf), _ptr(work), nbytes,
                                        _ptr(out), _stream(stream)))


def reduce_noalloc(map_, k, r, rule, buf, out, stream=None):
    """Test RD as `reduce`, with the library's static per-device scratch in
    place of a caller workspace (nothing is allocated; k - r <= 13; calls
    that overlap on one device race on that scratch)."""
    return _check(load().fractal_reduce_noalloc(map_, k, r, rule, _ptr(buf), _ptr(out),
                                                _stream(stream)))


def compact_bytes(k, r, rule) -> int:
    """Bytes of one compact state (tiles of side 2^r kept in lambda order)."""
    b = ctypes.c_size_t()
    _check(load().fractal_compact_bytes(k, r, rule, ctypes.byref(b)))
    return b.value


def pack(k, r, rule, embedded, compact, stream=None):
    return _check(load().fractal_pack(k, r, rule, _ptr(embedded), _ptr(compact),
                                      _stream(stream)))


def unpack(k, r, rule, compact, embedded, stream=None):
    return _check(load().fractal_unpack(k, r, rule, _ptr(compact), _ptr(embedded),
                                        _stream(stream)))


def compact_seed_fill(k, r, rule, stream_id, compact, stream=None):
    return _check(load().fractal_compact_seed_fill(k, r, rule, stream_id, _ptr(compact),
                                                   _stream(stream)))


def compact_step(k, r, rule, alpha, buf0, buf1, steps, flags=0, stream=None):
    return _check(load().fractal_compact_step(k, r, rule, alpha, _ptr(buf0), _ptr(buf1), steps,
                                              flags, _stream(stream)))


def nbb_builtin(which) -> Nbb:
    """A built-in NBB table (FRACTAL_NBB_*)."""
    f = Nbb()
    _check(load().fractal_nbb_builtin(which, ctypes.byref(f)))
    return f


def nbb_make(k, s, replicas) -> Nbb:
    """An NBB table from a list of (tau_x, tau_y) replica offsets."""
    f = Nbb()
    f.k, f.s = k, s
    for i, (x, y) in enumerate(replicas):
        f.tau_x[i], f.tau_y[i] = x, y
    return f


def nbb_lambda_map(f, rb, out, stream=None):
    return _check(load().fractal_nbb_lambda_map(ctypes.byref(f), rb, _ptr(out), _stream(stream)))


def nbb_single_write(f, map_, level, r, value, buf, stream=None):
    return _check(load().fractal_nbb_single_write(ctypes.byref(f), map_, level, r,
                                                  int(value) & 0xFF, _ptr(buf), _stream(stream)))


def nbb_reduce_workspace(f, level, r) -> int:
    b = ctypes.c_size_t()
    _check(load().fractal_nbb_reduce_workspace(ctypes.byref(f), level, r, ctypes.byref(b)))
    return b.value


def nbb_reduce(f, map_, level, r, buf, work, out, stream=None, work_bytes=None):
    nbytes = _nbytes(work, work_bytes, "nbb_reduce workspace")
    return _check(load().fractal_nbb_reduce(ctypes.byref(f), map_, level, r, _ptr(buf),
                                            _ptr(work), nbytes, _ptr(out), _stream(stream)))


def nbb_ca_step(f, map_, level, r, buf0, buf1, steps, stream=None):
    return _check(load().fractal_nbb_ca_step(ctypes.byref(f), map_, level, r, _ptr(buf0),
                                             _ptr(buf1), steps, _stream(stream)))


def now() -> float:
    return load().fractal_now()


class Server:
    """Handle on a libfractal request server (continuous batching)."""

    def __init__(self, arena, arena_bytes, max_slots, steps_per_iter=None, stream=None):
        h = ctypes.c_void_p()
        _check(load().fractal_serve_create(_ptr(arena), arena_bytes, max_slots,
                                           _stream(stream), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        if steps_per_iter is not None:
            self.set_steps_per_iter(steps_per_iter)

    def set_steps_per_iter(self, steps_per_iter):
        """Steps each admitted request advances per scheduling iteration."""
        _check(load().fractal_serve_set_steps_per_iter(self._h, steps_per_iter))

    def submit(self, k, rule, steps, alpha=0.2, seed=0, h_init=None, h_out=None,
               t_arrival=-1.0):
        """h_init / h_out: numpy arrays (kept alive until the ticket is polled)."""
        rq = Request(k, rule, steps, alpha, seed,
                     None if h_init is None else h_init.ctypes.data,
                     None if h_out is None else h_out.ctypes.data, t_arrival)
        t = ctypes.c_uint64()
        _check(load().fractal_serve_submit(self._h, ctypes.byref(rq), ctypes.byref(t)))
        self._keep[t.value] = (h_init, h_out)
        return t.value

    def poll(self, ticket):
        """Result (status, t_arrival, t_admit, t_done, checksum) or None."""
        res = Result()
        rc = load().fractal_serve_poll(self._h, ticket, ctypes.byref(res))
        if rc == E_AGAIN:
            return None
        _check(rc)
        self._keep.pop(ticket, None)
        return (res.status, res.t_arrival, res.t_admit, res.t_done, res.checksum)

    def stats(self):
        """Latency (p50, p99, mean of done minus arrival) and throughput of
        the requests completed so far, as a dict."""
        rep = ServeReport()
        _check(load().fractal_serve_stats(self._h, ctypes.byref(rep)))
        return rep.as_dict()

    def close(self):
        if self._h is not None and self._h.value:
            _check(load().fractal_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
