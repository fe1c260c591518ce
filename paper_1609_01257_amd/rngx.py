"""ctypes binding of librngx.so (the C ABI declared in include/rngx.h).

Argument marshalling only: every computation runs in the library's HIP
kernels and host code. Functions take torch tensors for device buffers and
torch streams (or raw handles) for streams, and raise :class:`RngxError` on a
non-zero status. The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librngx.so")

RNGX_OK = 0
RNGX_E_INVAL = -1
RNGX_E_NOINIT = -2
RNGX_E_HIP = -3
RNGX_E_NOMEM = -4
RNGX_E_BUSY = -5
RNGX_E_ABORTED = -6
COPY_KERNEL = 0
COPY_RUNTIME = 1
EXPORT_TABLE = 0
EXPORT_TRACE = 1
SCRAMBLE_NONE = 0
SCRAMBLE_STAR = 1

CONSUME_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                              ctypes.c_size_t)

PROF_NAME = 32
PROF_MAX_AGG = 16
PROF_MAX_OVERLAP = 32


class RngxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (strerror(code), msg))
        self.code = code


class BatchCfg(ctypes.Structure):
    _fields_ = [("values_per_lane", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("blocks", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("row_values", ctypes.c_uint32), ("run_items", ctypes.c_uint32),
                ("per_item", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("group_steps", ctypes.c_uint32), ("pace_gbs", ctypes.c_uint32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("cfg", BatchCfg), ("ms", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", BatchCfg), ("best_ms", ctypes.c_double), ("best_gbs", ctypes.c_double),
                ("n_tried", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("tried", TuneEntry * 128), ("confirm", TuneEntry * 4)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("chunks", ctypes.c_uint32),
                ("nontemporal", ctypes.c_uint32), ("pace_gbs", ctypes.c_uint32)]


class PlainTuneEntry(ctypes.Structure):
    _fields_ = [("cfg", Launch), ("ms", ctypes.c_double)]


class PlainTuneResult(ctypes.Structure):
    _fields_ = [("best", Launch), ("best_ms", ctypes.c_double), ("best_gbs", ctypes.c_double),
                ("n_tried", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("tried", PlainTuneEntry * 128), ("confirm", PlainTuneEntry * 4)]


class ServeReport(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "released", "pending",
                                                "admitted", "inflight_batches", "batches",
                                                "bytes")] + \
               [(k, ctypes.c_double) for k in ("elapsed_s", "gbs", "lat_p50_us", "lat_p99_us",
                                                "lat_max_us", "lat_mean_us", "wait_p50_us",
                                                "wait_p99_us", "launch_p50_us", "launch_p99_us",
                                                "exec_p50_us", "exec_p99_us")] + \
               [("max_pending", ctypes.c_uint64), ("admission_stalls", ctypes.c_uint64),
                ("mean_batch_requests", ctypes.c_double), ("pool_bytes", ctypes.c_uint64),
                ("pool_used_bytes", ctypes.c_uint64), ("pool_peak_bytes", ctypes.c_uint64),
                ("lag_p50_us", ctypes.c_double), ("lag_p99_us", ctypes.c_double),
                ("lag_max_us", ctypes.c_double)]


class ProfEvent(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * PROF_NAME), ("queue", ctypes.c_uint64),
                ("start_ns", ctypes.c_uint64), ("end_ns", ctypes.c_uint64)]


class ProfAgg(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * PROF_NAME), ("count", ctypes.c_uint64),
                ("abs_s", ctypes.c_double), ("rel_pct", ctypes.c_double)]


class ProfOverlap(ctypes.Structure):
    _fields_ = [("name1", ctypes.c_char * PROF_NAME), ("name2", ctypes.c_char * PROF_NAME),
                ("overlap_s", ctypes.c_double)]


class ProfStats(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_uint64), ("n_dropped", ctypes.c_uint64),
                ("n_agg", ctypes.c_uint32), ("n_overlap", ctypes.c_uint32),
                ("total_s", ctypes.c_double), ("overlap_s", ctypes.c_double),
                ("eff_s", ctypes.c_double), ("elapsed_s", ctypes.c_double),
                ("device_pct", ctypes.c_double), ("host_pct", ctypes.c_double),
                ("agg", ProfAgg * PROF_MAX_AGG), ("overlap", ProfOverlap * PROF_MAX_OVERLAP)]


_lib = None

_u32, _u64, _int, _p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
_SIGS = {
    "rngx_init": ([_u64, _u32], _int),
    "rngx_generate": ([_u32, _p, _p], _int),
    "rngx_generate_u32": ([_u32, _p, _p], _int),
    "rngx_info": ([_p, _p, _p], _int),
    "rngx_get_state": ([_p, _u32, _p, _p], _int),
    "rngx_set_scrambler": ([_int], _int),
    "rngx_get_scrambler": ([_p], _int),
    "rngx_set_state": ([_u64, _p, _u32, _u64], _int),
    "rngx_shutdown": ([], _int),
    "rngx_last_error": ([], ctypes.c_char_p),
    "rngx_strerror": ([_int], ctypes.c_char_p),
    "rngx_hip_notes": ([ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.c_char_p,
                        ctypes.c_size_t, _int], _int),
    "rngx_set_launch": ([_int, ctypes.POINTER(Launch)], _int),
    "rngx_get_launch": ([_int, ctypes.POINTER(Launch)], _int),
    "rngx_stream_to_host": ([_u32, _u32, _int, _p, _p, ctypes.c_size_t, _p, _u32, CONSUME_FN,
                             _p, _p, _p], _int),
    "rngx_set_copy_mode": ([_int, _u32], _int),
    "rngx_inject_copy_failure": ([_u64], _int),
    "rngx_get_copy_mode": ([ctypes.POINTER(_int), ctypes.POINTER(_u32)], _int),
    "rngx_generate_batch": ([_p, _u32, _p, _u64, _p], _int),
    "rngx_generate_batch_noalloc": ([_p, _u32, _p, _u64, _p], _int),
    "rngx_set_batch_cfg": ([ctypes.POINTER(BatchCfg)], _int),
    "rngx_get_batch_cfg": ([ctypes.POINTER(BatchCfg)], _int),
    "rngx_autotune_batch": ([_p, _u32, _p, _u64, _u32, _p, ctypes.POINTER(TuneResult)], _int),
    "rngx_checksum": ([_p, _u64, _p, ctypes.POINTER(_u64)], _int),
    "rngx_autotune_plain": ([_u32, _int, _p, _u32, _p, ctypes.POINTER(PlainTuneResult)], _int),
    "rngx_tune_cache_save": ([ctypes.c_char_p], _int),
    "rngx_tune_cache_load": ([ctypes.c_char_p, ctypes.POINTER(_u32)], _int),
    "rngx_initial_state": ([_u64, _u32, ctypes.POINTER(_u64)], _int),
    "rngx_jump_ahead": ([_u64, _u64, ctypes.POINTER(_u64)], _int),
    "rngx_serve_start": ([_u64, _u32, _p, _u64, _u32, _u32], _int),
    "rngx_serve_submit": ([_u32, _u64, _u32, ctypes.POINTER(_u64)], _int),
    "rngx_serve_try_submit": ([_u32, _u64, _u32, ctypes.POINTER(_u64)], _int),
    "rngx_serve_submit_many": ([_p, _p, _u64, _u32, _p], _int),
    "rngx_serve_poll": ([_u64, ctypes.POINTER(_p), ctypes.POINTER(_int)], _int),
    "rngx_serve_wait": ([_u64, ctypes.c_double, ctypes.POINTER(_p)], _int),
    "rngx_serve_release": ([_u64], _int),
    "rngx_serve_stats": ([ctypes.POINTER(ServeReport)], _int),
    "rngx_serve_reset_stats": ([], _int),
    "rngx_serve_run_trace": ([_p, _p, _p, _u64, ctypes.c_double, ctypes.POINTER(ServeReport)],
                             _int),
    "rngx_serve_set_max_pending": ([_u64], _int),
    "rngx_serve_set_max_inflight": ([_u32], _int),
    "rngx_serve_stop": ([], _int),
    "rngx_profile_start": ([], _int),
    "rngx_profile_reset": ([], _int),
    "rngx_profile_stop": ([], _int),
    "rngx_profile_enable": ([_int], _int),
    "rngx_profile": ([], ctypes.c_char_p),
    "rngx_profile_stats": ([ctypes.POINTER(ProfStats)], _int),
    "rngx_profile_events": ([_p, _u32, ctypes.POINTER(_u32)], _int),
    "rngx_profile_analyze": ([_p, _u32, ctypes.c_double, ctypes.POINTER(ProfStats)], _int),
    "rngx_profile_write": ([_p, _u32, ctypes.c_char_p, _int], _int),
    "rngx_profile_export": ([ctypes.c_char_p, _int], _int),
}


def lib():
    """Load librngx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librngx.so is not built (expected at %s); run "
                               "`python -m paper_1609_01257_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().rngx_strerror(code).decode()


def last_error() -> str:
    return lib().rngx_last_error().decode()


def hip_notes(clear: bool = False) -> dict:
    """HIP errors no call could return: failures on the library's release
    paths ("released") and errors found pending before a launch ("stray"),
    with the most recent notes as text."""
    rel, stray = _u64(), _u64()
    buf = ctypes.create_string_buffer(8192)
    _check(lib().rngx_hip_notes(ctypes.byref(rel), ctypes.byref(stray), buf, len(buf),
                                int(bool(clear))))
    return {"released": rel.value, "stray": stray.value,
            "notes": [l for l in buf.value.decode().split("\n") if l]}


def _check(rc: int):
    if rc != RNGX_OK:
        raise RngxError(rc, last_error())


def stream_handle(stream) -> int:
    """hipStream_t of a torch stream, a raw integer handle, or the current stream."""
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _device_buffer(t, esize: int, need: int) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("output must be a CUDA (HIP) torch tensor")
    if t.element_size() != esize or t.dtype.is_floating_point:
        raise TypeError("output must be a %d-byte integer tensor" % esize)
    if not t.is_contiguous():
        raise ValueError("output must be contiguous")
    if t.numel() < need:
        raise ValueError("output holds %d elements, %d needed" % (t.numel(), need))
    return t.data_ptr()


# --- generator --------------------------------------------------------------

def init(seed: int, n_states: int):
    _check(lib().rngx_init(seed & (2**64 - 1), n_states))


def info():
    s, n, c = _u64(), _u32(), _u64()
    _check(lib().rngx_info(ctypes.byref(s), ctypes.byref(n), ctypes.byref(c)))
    return s.value, n.value, c.value


def set_scrambler(scrambler: int):
    """Output word of the plain path: SCRAMBLE_NONE (the paper's) or SCRAMBLE_STAR."""
    _check(lib().rngx_set_scrambler(scrambler))


def get_scrambler() -> int:
    v = ctypes.c_int()
    _check(lib().rngx_get_scrambler(ctypes.byref(v)))
    return v.value


def get_state():
    """Checkpoint: (states as a uint64 numpy array, seed, cursor)."""
    import numpy as np
    n = info()[1]
    st = np.empty(n, dtype=np.uint64)
    s, c = _u64(), _u64()
    _check(lib().rngx_get_state(st.ctypes.data, n, ctypes.byref(s), ctypes.byref(c)))
    return st, s.value, c.value


def set_state(seed: int, states, cursor: int):
    """Resume from a checkpoint taken by get_state (any process, any device)."""
    import numpy as np
    st = np.ascontiguousarray(states, dtype=np.uint64)
    _check(lib().rngx_set_state(seed & (2**64 - 1), st.ctypes.data, len(st), cursor))


def generate(n_iters: int, out, stream=None):
    """out[k * n + g] = V(seed, g, cursor + k) for k < n_iters (uint64/int64 tensor)."""
    n = info()[1]
    ptr = _device_buffer(out, 8, n_iters * n) if n_iters else (out.data_ptr() if out is not None else 0)
    _check(lib().rngx_generate(n_iters, ptr, stream_handle(stream)))


def generate_u32(n_iters: int, out, stream=None):
    """Low 32-bit halves of :func:`generate` (uint32/int32 tensor)."""
    n = info()[1]
    ptr = _device_buffer(out, 4, n_iters * n) if n_iters else (out.data_ptr() if out is not None else 0)
    _check(lib().rngx_generate_u32(n_iters, ptr, stream_handle(stream)))


def generate_ptr(n_iters: int, ptr: int, stream: int = 0, u32: bool = False) -> int:
    """Raw call (returns the status instead of raising); for ABI tests."""
    f = lib().rngx_generate_u32 if u32 else lib().rngx_generate
    return f(n_iters, ptr, stream)


def stream_to_host(n_steps: int, iters_per_step: int, dev0, dev1, host, host_slots: int,
                   consume=None, u32: bool = False, gen_stream=None, copy_stream=None):
    """Stream n_steps * iters_per_step iterations to `host` (a pinned CPU
    tensor of host_slots slots) through device buffers dev0/dev1, generation
    and copies overlapped on two streams. `consume(step, array)` (optional)
    receives each step as a numpy view of its host slot, in order; returning
    a true value stops the stream (raises RngxError with RNGX_E_ABORTED), and
    an exception it raises stops the stream and is re-raised here."""
    import numpy as np
    n = info()[1]
    esize = 4 if u32 else 8
    step_elems = iters_per_step * n
    for d in (dev0, dev1):
        _device_buffer(d, esize, step_elems)
    if host.is_cuda or not host.is_contiguous() or host.element_size() != esize:
        raise TypeError("host must be a contiguous CPU tensor of %d-byte integers" % esize)
    if host.numel() < step_elems * host_slots:
        raise ValueError("host holds %d elements, %d needed" % (host.numel(), step_elems * host_slots))
    dev_bytes = min(dev0.numel(), dev1.numel()) * esize
    cb = CONSUME_FN()
    raised = []
    if consume is not None:
        npdt = np.uint32 if u32 else np.uint64

        def _cb(user, step, ptr, nbytes):
            try:
                arr = np.ctypeslib.as_array((ctypes.c_uint8 * nbytes).from_address(ptr)).view(npdt)
                return 1 if consume(step, arr) else 0
            except BaseException as e:  # stop the stream; re-raised below
                raised.append(e)
                return 1
        cb = CONSUME_FN(_cb)
    gs = stream_handle(gen_stream) if gen_stream is not None else 0
    cs = stream_handle(copy_stream) if copy_stream is not None else 0
    rc = lib().rngx_stream_to_host(n_steps, iters_per_step, int(u32), dev0.data_ptr(),
                                   dev1.data_ptr(), dev_bytes, host.data_ptr(), host_slots,
                                   cb, None, gs, cs)
    if raised:
        raise raised[0]
    _check(rc)


def inject_copy_failure(step: int):
    """Make the copy of `step` fail in the next stream_to_host call (test
    hook; 2**64 - 1 disarms it)."""
    _check(lib().rngx_inject_copy_failure(step))


def set_copy_mode(mode: int, blocks: int = 16):
    _check(lib().rngx_set_copy_mode(mode, blocks))


def get_copy_mode():
    m, b = _int(), _u32()
    _check(lib().rngx_get_copy_mode(ctypes.byref(m), ctypes.byref(b)))
    return m.value, b.value


# --- batched streams ----------------------------------------------------------

def req_dtype():
    import numpy as np
    return np.dtype([("seed", "<u8"), ("offset", "<u8"), ("length", "<u8"),
                     ("gid", "<u4"), ("reserved", "<u4")])


def make_reqs(seeds, gids, offsets, lengths):
    """Pack a request table (the rngx_req layout) from four sequences."""
    import numpy as np
    r = np.zeros(len(lengths), dtype=req_dtype())
    r["seed"] = np.asarray(seeds, dtype=np.uint64)
    r["gid"] = np.asarray(gids, dtype=np.uint32)
    r["offset"] = np.asarray(offsets, dtype=np.uint64)
    r["length"] = np.asarray(lengths, dtype=np.uint64)
    return r


def _reqs_arg(reqs):
    import numpy as np
    reqs = np.ascontiguousarray(reqs, dtype=req_dtype())
    return reqs, (reqs.ctypes.data if len(reqs) else None)


def generate_batch(reqs, out, stream=None):
    """out[base_j + t] = V(seed_j, gid_j, offset_j + t), packed in request order."""
    reqs, ptr = _reqs_arg(reqs)
    total = int(reqs["length"].sum()) if len(reqs) else 0
    optr = _device_buffer(out, 8, total) if total else (out.data_ptr() if out is not None else 0)
    cap = out.numel() if out is not None else 0
    _check(lib().rngx_generate_batch(ptr, len(reqs), optr, cap, stream_handle(stream)))
    return total


NOALLOC_MAX_REQS = 4096


def generate_batch_noalloc(reqs, out, stream=None):
    """generate_batch through the entry point that allocates nothing (its
    request table is a static device array; at most NOALLOC_MAX_REQS
    requests; calls that overlap on one device race)."""
    reqs, ptr = _reqs_arg(reqs)
    total = int(reqs["length"].sum()) if len(reqs) else 0
    optr = _device_buffer(out, 8, total) if total else (out.data_ptr() if out is not None else 0)
    cap = out.numel() if out is not None else 0
    _check(lib().rngx_generate_batch_noalloc(ptr, len(reqs), optr, cap, stream_handle(stream)))
    return total


def set_batch_cfg(values_per_lane=256, waves_per_block=4, blocks=0, use_graph=True,
                  row_values=16, run_items=1, per_item=False, group=0, group_steps=0,
                  pace_gbs=0):
    """Batch launch configuration; group > 0 selects the grouped order (groups of
    `group` wavefronts, `group_steps` steps per region, optional row schedule).
    The arguments default to the persistent grid with S = 256; the library's
    own default configuration (before any call) is the grouped order."""
    cfg = BatchCfg(values_per_lane, waves_per_block, blocks, int(bool(use_graph)), row_values,
                   run_items, int(bool(per_item)), group, group_steps, pace_gbs)
    _check(lib().rngx_set_batch_cfg(ctypes.byref(cfg)))


def get_batch_cfg():
    c = BatchCfg()
    _check(lib().rngx_get_batch_cfg(ctypes.byref(c)))
    return _cfg_dict(c)


def _cfg_dict(c):
    return {"values_per_lane": c.values_per_lane, "waves_per_block": c.waves_per_block,
            "blocks": c.blocks, "use_graph": bool(c.use_graph), "row_values": c.row_values,
            "run_items": c.run_items, "per_item": bool(c.per_item), "group": c.group,
            "group_steps": c.group_steps, "pace_gbs": c.pace_gbs}


def autotune_batch(reqs, out, reps=2, stream=None):
    """Time every batch launch configuration on this table; keep the fastest."""
    reqs, ptr = _reqs_arg(reqs)
    total = int(reqs["length"].sum())
    optr = _device_buffer(out, 8, total)
    res = TuneResult()
    _check(lib().rngx_autotune_batch(ptr, len(reqs), optr, out.numel(), reps,
                                     stream_handle(stream), ctypes.byref(res)))
    n = min(res.n_tried, 128)
    return {"best": _cfg_dict(res.best), "best_ms": res.best_ms, "best_gbs": res.best_gbs,
            "tried": [(_cfg_dict(res.tried[i].cfg), res.tried[i].ms) for i in range(n)],
            "confirm": [(_cfg_dict(res.confirm[i].cfg), res.confirm[i].ms)
                        for i in range(4) if res.confirm[i].cfg.values_per_lane]}


def _launch_dict(c):
    return {"block": c.block, "chunks": c.chunks, "nontemporal": bool(c.nontemporal),
            "pace_gbs": c.pace_gbs}


def autotune_plain(n_iters, out, reps=2, u32=False, stream=None):
    """Time every plain launch configuration at the current generator's shape
    for n_iters iterations; keep the fastest (state and cursor unchanged;
    `out` receives the next n_iters iterations)."""
    n = info()[1]
    optr = _device_buffer(out, 4 if u32 else 8, n_iters * n)
    res = PlainTuneResult()
    _check(lib().rngx_autotune_plain(n_iters, int(bool(u32)), optr, reps, stream_handle(stream),
                                     ctypes.byref(res)))
    k = min(res.n_tried, 128)
    return {"best": _launch_dict(res.best), "best_ms": res.best_ms, "best_gbs": res.best_gbs,
            "tried": [(_launch_dict(res.tried[i].cfg), res.tried[i].ms) for i in range(k)],
            "confirm": [(_launch_dict(res.confirm[i].cfg), res.confirm[i].ms)
                        for i in range(4) if res.confirm[i].cfg.block]}


def tune_cache_save(path):
    _check(lib().rngx_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path) -> int:
    n = _u32()
    _check(lib().rngx_tune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def checksum(t, n=None, stream=None) -> int:
    """sum_i t[i] * (2 i + 1) mod 2^64 over the first n uint64 values, on the device."""
    n = t.numel() if n is None else n
    ptr = _device_buffer(t, 8, n) if n else t.data_ptr()
    r = _u64()
    _check(lib().rngx_checksum(ptr, n, stream_handle(stream), ctypes.byref(r)))
    return r.value


def initial_state(seed: int, gid: int) -> int:
    r = _u64()
    _check(lib().rngx_initial_state(seed & (2**64 - 1), gid, ctypes.byref(r)))
    return r.value


def jump_ahead(state: int, k: int) -> int:
    r = _u64()
    _check(lib().rngx_jump_ahead(state, k, ctypes.byref(r)))
    return r.value


# --- serving --------------------------------------------------------------------

SERVE_AUTORELEASE = 1


def serve_start(seed: int, n_states: int, pool, n_streams: int = 4, max_batch: int = 1024):
    """Start the server over a caller-owned device pool (a CUDA tensor)."""
    if not pool.is_cuda or not pool.is_contiguous():
        raise TypeError("pool must be a contiguous device tensor")
    _check(lib().rngx_serve_start(seed & (2**64 - 1), n_states, pool.data_ptr(),
                                  pool.numel() * pool.element_size(), n_streams, max_batch))


def serve_submit(stream_id: int, length: int, autorelease: bool = False, wait: bool = True) -> int:
    t = _u64()
    f = lib().rngx_serve_submit if wait else lib().rngx_serve_try_submit
    _check(f(stream_id, length, SERVE_AUTORELEASE if autorelease else 0, ctypes.byref(t)))
    return t.value


def serve_submit_many(stream_ids, lengths, autorelease: bool = False):
    """Submit many requests at once; returns their tickets (numpy uint64)."""
    import numpy as np
    g = np.ascontiguousarray(stream_ids, dtype=np.uint32)
    n = np.ascontiguousarray(lengths, dtype=np.uint64)
    if len(g) != len(n):
        raise ValueError("stream_ids and lengths differ in length")
    t = np.zeros(len(g), dtype=np.uint64)
    _check(lib().rngx_serve_submit_many(g.ctypes.data, n.ctypes.data, len(g),
                                        SERVE_AUTORELEASE if autorelease else 0, t.ctypes.data))
    return t


def serve_poll(ticket: int):
    """(device address of the values or None, done)."""
    p, d = _p(), _int()
    _check(lib().rngx_serve_poll(ticket, ctypes.byref(p), ctypes.byref(d)))
    return p.value, bool(d.value)


def serve_wait(ticket: int, timeout_s: float = 30.0) -> int:
    p = _p()
    _check(lib().rngx_serve_wait(ticket, timeout_s, ctypes.byref(p)))
    return p.value


def serve_release(ticket: int):
    _check(lib().rngx_serve_release(ticket))


def _report(r: ServeReport) -> dict:
    return {name: getattr(r, name) for name, _ in ServeReport._fields_}


def serve_stats() -> dict:
    r = ServeReport()
    _check(lib().rngx_serve_stats(ctypes.byref(r)))
    return _report(r)


def serve_reset_stats():
    _check(lib().rngx_serve_reset_stats())


def serve_run_trace(arrival_s, stream_id, length, timeout_s: float = 600.0) -> dict:
    """Open-loop load: request i at arrival_s[i] seconds; returns the trace's stats."""
    import numpy as np
    a = np.ascontiguousarray(arrival_s, dtype=np.float64)
    g = np.ascontiguousarray(stream_id, dtype=np.uint32)
    n = np.ascontiguousarray(length, dtype=np.uint64)
    if not (len(a) == len(g) == len(n)):
        raise ValueError("trace arrays differ in length")
    r = ServeReport()
    _check(lib().rngx_serve_run_trace(a.ctypes.data, g.ctypes.data, n.ctypes.data, len(a),
                                      timeout_s, ctypes.byref(r)))
    return _report(r)


def serve_set_max_inflight(max_inflight: int):
    _check(lib().rngx_serve_set_max_inflight(max_inflight))


def serve_set_max_pending(n: int):
    _check(lib().rngx_serve_set_max_pending(n))


def serve_stop():
    _check(lib().rngx_serve_stop())


def shutdown():
    _check(lib().rngx_shutdown())


def set_launch(u32: bool, block: int, chunks: int, nontemporal: bool = False, pace_gbs: int = 0):
    """Launch configuration of rngx_generate (u32: rngx_generate_u32); pace_gbs > 0
    runs the row-scheduled persistent kernel at that write rate."""
    cfg = Launch(block, chunks, int(bool(nontemporal)), pace_gbs)
    _check(lib().rngx_set_launch(int(u32), ctypes.byref(cfg)))


def get_launch(u32: bool):
    cfg = Launch()
    _check(lib().rngx_get_launch(int(u32), ctypes.byref(cfg)))
    return _launch_dict(cfg)


# --- profiling ----------------------------------------------------------------

def profile_start():
    _check(lib().rngx_profile_start())


def profile_reset():
    """Same as :func:`profile_start`."""
    _check(lib().rngx_profile_reset())


def profile_stop():
    _check(lib().rngx_profile_stop())


def profile_enable(on: bool):
    _check(lib().rngx_profile_enable(int(bool(on))))


def profile() -> str:
    s = lib().rngx_profile()
    if s is None:
        raise RngxError(RNGX_E_INVAL, last_error())
    return s.decode()


def _stats_dict(st: ProfStats) -> dict:
    return {
        "n_events": st.n_events, "n_dropped": st.n_dropped,
        "total_s": st.total_s, "overlap_s": st.overlap_s, "eff_s": st.eff_s,
        "elapsed_s": st.elapsed_s, "device_pct": st.device_pct, "host_pct": st.host_pct,
        "agg": [(st.agg[i].name.decode(), st.agg[i].count, st.agg[i].abs_s, st.agg[i].rel_pct)
                for i in range(st.n_agg)],
        "overlaps": [(st.overlap[i].name1.decode(), st.overlap[i].name2.decode(),
                      st.overlap[i].overlap_s) for i in range(st.n_overlap)],
    }


def profile_stats() -> dict:
    st = ProfStats()
    _check(lib().rngx_profile_stats(ctypes.byref(st)))
    return _stats_dict(st)


def profile_events() -> list:
    n = _u32()
    _check(lib().rngx_profile_events(None, 0, ctypes.byref(n)))
    arr = (ProfEvent * max(1, n.value))()
    _check(lib().rngx_profile_events(arr, n.value, ctypes.byref(n)))
    return [(arr[i].name.decode(), arr[i].queue, arr[i].start_ns, arr[i].end_ns)
            for i in range(n.value)]


def _event_array(events):
    arr = (ProfEvent * max(1, len(events)))()
    qid = {}
    for i, (name, q, s, e) in enumerate(events):
        arr[i].name = name.encode()[:PROF_NAME - 1]
        arr[i].queue = q if isinstance(q, int) else qid.setdefault(q, len(qid))
        arr[i].start_ns = s
        arr[i].end_ns = e
    return arr


def profile_write(events, path: str, fmt: int = EXPORT_TABLE):
    """Write (name, queue, start_ns, end_ns) rows as a table or trace file."""
    _check(lib().rngx_profile_write(_event_array(events), len(events), os.fsencode(path), fmt))


def profile_export(path: str, fmt: int = EXPORT_TABLE):
    """Write the current profiling window's events as a table or trace file."""
    _check(lib().rngx_profile_export(os.fsencode(path), fmt))


def profile_analyze(events, elapsed_s: float) -> dict:
    """Analyse (name, queue, start_ns, end_ns) rows with the library's code."""
    arr = _event_array(events)
    st = ProfStats()
    _check(lib().rngx_profile_analyze(arr, len(events), elapsed_s, ctypes.byref(st)))
    return _stats_dict(st)
