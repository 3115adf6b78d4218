"""Thin ctypes binding of libphos (include/phos.h): argument marshalling only.

Every function has the C name and raises PhosError on a non-OK status.  All
compute happens in libphos's gfx950 kernels; there is no fallback: if the
library is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphos.so")

OK, E_INVAL, E_NOMEM, E_HIP, E_STATE, E_OVERFLOW, E_MISSPEC, E_TIMEOUT = range(8)
R, W = 1, 2
ARG_SCALAR, ARG_PTR_CONST, ARG_PTR_MUT, ARG_STRUCT, ARG_RANGE = 0, 1, 2, 3, 4
V_READS, V_WRITES, V_TRACK, V_SYNC = 1, 2, 4, 8
COW, RECOPY = 1, 2
CKPT_DEFER_BACKGROUND = 1
STAGE_HOST_DIRECT, STAGE_BLOCK = 0, 1
RST_DEFER_BACKGROUND, RST_PREFETCH_SPEC = 1, 2

STATUS_NAMES = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_STATE", 5: "E_OVERFLOW",
                6: "E_MISSPEC", 7: "E_TIMEOUT"}

VIOLATION_DTYPE = np.dtype([("index", "<u8"), ("addr", "<u8"), ("launch_id", "<u4"),
                            ("is_write", "u1"), ("reason", "u1"), ("_p", "<u2"),
                            ("victim", "<i4"), ("_q", "<u4")])
INTERVAL_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8"), ("mode", "<u4"), ("_pad", "<u4")])
SEG_DTYPE = np.dtype([("src", "<u8"), ("dst", "<u8"), ("bytes", "<u8"), ("req", "<u4"),
                      ("_p", "<u4")])


class PhosError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class phos_buffer(ctypes.Structure):
    _fields_ = [("base", ctypes.c_uint64), ("bytes", ctypes.c_uint64)]


class phos_arg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("value", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("host_struct", ctypes.c_void_p)]


class phos_ckpt_stats(ctypes.Structure):
    _fields_ = [("bg_pages", ctypes.c_uint64), ("cow_pages", ctypes.c_uint64),
                ("recopy_pages", ctypes.c_uint64), ("image_bytes", ctypes.c_uint64),
                ("precopy_pages", ctypes.c_uint64), ("staged_pages", ctypes.c_uint64),
                ("bg_read_pages", ctypes.c_uint64), ("bg_ms", ctypes.c_double),
                ("stage_batches", ctypes.c_uint64)]


class phos_rst_stats(ctypes.Structure):
    _fields_ = [("bg_pages", ctypes.c_uint64), ("demand_pages", ctypes.c_uint64),
                ("dma_pages", ctypes.c_uint64), ("asked_pages", ctypes.c_uint64),
                ("dma_ms", ctypes.c_double), ("dma_first_ms", ctypes.c_double),
                ("dma_first_issue_ms", ctypes.c_double), ("dma_first_copy_ms", ctypes.c_double),
                ("bg_ms", ctypes.c_double)]


class phos_batch_cfg(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_uint64), ("wg_per_cu", ctypes.c_uint32),
                ("threads", ctypes.c_uint32)]


P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
PP = ctypes.POINTER(ctypes.c_void_p)

# (name, argtypes) of every exported entry point, in header order.
SIGNATURES = [
    ("phos_create", [ctypes.c_int, U64, U64, U32, PP]),
    ("phos_destroy", [P]),
    ("phos_buffers_register", [P, P, U32]),
    ("phos_image_bytes", [P, ctypes.POINTER(U64)]),
    ("phos_spec_register", [P, U32, P, U32, ctypes.POINTER(U32)]),
    ("phos_spec_intervals", [P, U32, P, U32, ctypes.POINTER(U32)]),
    ("phos_spec_release", [P, U32]),
    ("phos_validate", [P, U32, P, U64, U32, P, U64, P, P]),
    ("phos_validate_noalloc", [P, U32, P, U64, U32, P, U64, P, P]),
    ("phos_twin_scale_add", [P, U32, P, P, P, U64, U32, P, U64, P, P]),
    ("phos_validate_batch", [P, P, P, P, U32, U32, P, U64, P, P]),
    ("phos_stream_status", [P, P]),
    ("phos_track_reset", [P, P]),
    ("phos_track_read", [P, U32, P, U64]),
    ("phos_ckpt_begin", [P, U32, U32, P, P, P, PP]),
    ("phos_ckpt_cow", [P, U32, P]),
    ("phos_ckpt_recopy", [P, P]),
    ("phos_ckpt_precopy", [P, P]),
    ("phos_ckpt_precopy_final", [P, P, U32, U32, P]),
    ("phos_ckpt_staging", [P, P, U64]),
    ("phos_ckpt_staging_policy", [P, P, U64, U32]),
    ("phos_ckpt_start", [P, P]),
    ("phos_ckpt_start_pair", [P, P, P]),
    ("phos_ckpt_end", [P, P, P]),
    ("phos_ckpt_copied", [P, P, U64]),
    ("phos_restore_begin", [P, U32, P, P, PP]),
    ("phos_manifest_write", [P, U32, P, U64, ctypes.POINTER(U64)]),
    ("phos_manifest_check", [P, P, U64]),
    ("phos_restore_begin_manifest", [P, U32, P, P, U64, P, PP]),
    ("phos_restore_begin_chunked", [P, U32, P, U32, U64, P, PP]),
    ("phos_restore_on_demand", [P, U32, P, U64, P, P]),
    ("phos_restore_present", [P, P, U64]),
    ("phos_restore_end", [P, P, P]),
    ("phos_batch_create", [ctypes.c_int, U64, U32, P, PP]),
    ("phos_batch_destroy", [P]),
    ("phos_batch_load", [P, P, U64, P]),
    ("phos_batch_run", [P, P]),
    ("phos_batch_copy", [P, P, U64, P]),
    ("phos_batch_done_bytes", [P, PP]),
    ("phos_batch_times", [P, P, U32]),
    ("phos_batch_get_cfg", [P, P]),
    ("phos_batch_set_cfg", [P, P]),
    ("phos_seglist_create", [ctypes.c_int, P, U64, PP]),
    ("phos_seglist_destroy", [P]),
    ("phos_copy_plain", [P, U64, U32, P]),
    ("phos_copy_batch", [P, P, U64, P]),
    ("phos_copy_batch_tuned", [P, P, U64, P]),
    ("phos_batch_tune", [ctypes.c_int, P, U64, ctypes.c_char_p, P, ctypes.POINTER(ctypes.c_double)]),
]

_lib = None


def _torch_first():
    """Load torch's HIP runtime before libphos.so when torch is installed.
    torch ships its own HSA runtime (soname libhsa-runtime64.so.1, asked for
    as libhsa-runtime64.so); loaded first, it satisfies libphos.so's need for
    libhsa-runtime64.so.1 and the process has one HSA runtime.  In the other
    order each library gets its own, and the one initialized second finds no
    device."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        _torch_first()
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.phos_last_error.argtypes = []
        L.phos_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _call(name: str, *args) -> None:
    st = getattr(lib(), name)(*args)
    if st != OK:
        raise PhosError(st, name, lib().phos_last_error().decode(errors="replace"))


def _stream(s) -> Optional[int]:
    """torch.cuda.Stream | int handle | None (null stream) -> handle."""
    if s is None:
        return None
    return int(getattr(s, "cuda_stream", s))


def _ptr(x) -> Optional[int]:
    """torch tensor / numpy array / int / None -> address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


# ---------------------------------------------------------------- context
def phos_create(device: int, pool_base: int, pool_bytes: int, page_bytes: int) -> int:
    out = ctypes.c_void_p()
    _call("phos_create", device, pool_base, pool_bytes, page_bytes, ctypes.byref(out))
    return out.value


def phos_destroy(ctx: int) -> None:
    _call("phos_destroy", ctx)


def phos_buffers_register(ctx: int, bufs: Sequence[Tuple[int, int]]) -> None:
    arr = (phos_buffer * max(1, len(bufs)))(*[phos_buffer(b, n) for b, n in bufs])
    _call("phos_buffers_register", ctx, arr, len(bufs))


def phos_image_bytes(ctx: int) -> int:
    v = U64()
    _call("phos_image_bytes", ctx, ctypes.byref(v))
    return v.value


# ------------------------------------------------------------ speculation
def make_args(args: Sequence[Tuple[int, int, int, int]], structs=None):
    """args: (kind, mode, value, bytes); structs: {position: bytes}. Returns (array, keepalive)."""
    structs = structs or {}
    arr = (phos_arg * max(1, len(args)))()
    keep = []
    for j, (kind, mode, value, nbytes) in enumerate(args):
        arr[j].kind, arr[j].mode, arr[j].value, arr[j].bytes = kind, mode, value, nbytes
        if j in structs:
            buf = ctypes.create_string_buffer(structs[j], len(structs[j]))
            keep.append(buf)
            arr[j].host_struct = ctypes.addressof(buf)
            arr[j].bytes = len(structs[j])
    return arr, keep


def phos_spec_register(ctx: int, launch_id: int, args, structs=None) -> int:
    arr, keep = make_args(args, structs)
    out = U32()
    _call("phos_spec_register", ctx, launch_id, arr, len(args), ctypes.byref(out))
    del keep
    return out.value


def phos_spec_intervals(ctx: int, spec: int) -> np.ndarray:
    n = U32()
    out = np.zeros(64, dtype=INTERVAL_DTYPE)
    _call("phos_spec_intervals", ctx, spec, out.ctypes.data, 64, ctypes.byref(n))
    return out[: n.value].copy()


def phos_spec_release(ctx: int, spec: int) -> None:
    _call("phos_spec_release", ctx, spec)


# ------------------------------------------------------------- validation
def phos_validate(ctx, spec, d_records, n, flags, out, cap, n_violations, stream=None) -> None:
    _call("phos_validate", ctx, spec, _ptr(d_records), n, flags, _ptr(out), cap,
          _ptr(n_violations), _stream(stream))


def phos_validate_noalloc(ctx, spec, d_records, n, flags, out, cap, n_violations,
                          stream=None) -> None:
    _call("phos_validate_noalloc", ctx, spec, _ptr(d_records), n, flags, _ptr(out), cap,
          _ptr(n_violations), _stream(stream))


def _array(vals, dtype):
    """A contiguous numpy array of `vals` (kept alive by the caller)."""
    if isinstance(vals, np.ndarray) and vals.dtype == dtype and vals.flags.c_contiguous:
        return vals
    return np.ascontiguousarray(vals, dtype=dtype)


def phos_validate_batch(ctx, specs, d_records, n, flags, out, cap, n_violations,
                        stream=None) -> None:
    """specs, d_records (integer addresses or tensors) and n: sequences or
    numpy arrays (uint32, uint64, uint64) of one entry per launch."""
    k = len(specs)
    sp = _array(specs, np.uint32)
    if isinstance(d_records, np.ndarray):
        rp = _array(d_records, np.uint64)
    else:
        rp = np.fromiter((_ptr(r) or 0 for r in d_records), dtype=np.uint64, count=k)
    nn = _array(n, np.uint64)
    if k == 0:
        sp, rp, nn = np.zeros(1, np.uint32), np.zeros(1, np.uint64), np.zeros(1, np.uint64)
    _call("phos_validate_batch", ctx, sp.ctypes.data, rp.ctypes.data, nn.ctypes.data, k, flags,
          _ptr(out), cap, _ptr(n_violations), _stream(stream))


def phos_twin_scale_add(ctx, spec, x, y, idx, n, flags, out=None, cap=0, n_violations=None,
                        stream=None) -> None:
    _call("phos_twin_scale_add", ctx, spec, _ptr(x), _ptr(y), _ptr(idx), n, flags, _ptr(out), cap,
          _ptr(n_violations), _stream(stream))


def phos_stream_status(ctx, stream=None) -> None:
    _call("phos_stream_status", ctx, _stream(stream))


def phos_track_reset(ctx, stream=None) -> None:
    _call("phos_track_reset", ctx, _stream(stream))


def phos_track_read(ctx, which: int, n_pages: int) -> np.ndarray:
    nw = (n_pages + 31) // 32
    out = np.zeros(nw, dtype=np.uint32)
    _call("phos_track_read", ctx, which, out.ctypes.data, nw)
    return out


# ------------------------------------------------------------- checkpoint
def phos_ckpt_begin(ctx, protocol, flags, image, host_image, copy_stream) -> int:
    out = ctypes.c_void_p()
    _call("phos_ckpt_begin", ctx, protocol, flags, _ptr(image), _ptr(host_image),
          _stream(copy_stream), ctypes.byref(out))
    return out.value


def phos_ckpt_cow(ck, spec, app_stream) -> None:
    _call("phos_ckpt_cow", ck, spec, _stream(app_stream))


def phos_ckpt_recopy(ck, app_stream) -> None:
    _call("phos_ckpt_recopy", ck, _stream(app_stream))


def phos_ckpt_start(ck, after=None) -> None:
    _call("phos_ckpt_start", ck, _stream(after))


def phos_ckpt_start_pair(cow, recopy, after=None) -> None:
    _call("phos_ckpt_start_pair", cow, recopy, _stream(after))


def phos_ckpt_staging(ck, staging, nbytes) -> None:
    _call("phos_ckpt_staging", ck, _ptr(staging), nbytes)


def phos_ckpt_staging_policy(ck, staging, nbytes, policy) -> None:
    _call("phos_ckpt_staging_policy", ck, _ptr(staging), nbytes, policy)


def phos_ckpt_precopy(ck, app_stream) -> None:
    _call("phos_ckpt_precopy", ck, _stream(app_stream))


def phos_ckpt_precopy_final(ck, upcoming, n_validated_ahead, app_stream) -> None:
    k = len(upcoming)
    sp = _array(upcoming, np.uint32) if k else np.zeros(1, np.uint32)
    _call("phos_ckpt_precopy_final", ck, sp.ctypes.data, k, n_validated_ahead,
          _stream(app_stream))


def phos_ckpt_end(ck, app_stream) -> phos_ckpt_stats:
    st = phos_ckpt_stats()
    _call("phos_ckpt_end", ck, _stream(app_stream), ctypes.byref(st))
    return st


def phos_ckpt_copied(ck, n_pages: int) -> np.ndarray:
    nw = (n_pages + 31) // 32
    out = np.zeros(nw, dtype=np.uint32)
    _call("phos_ckpt_copied", ck, out.ctypes.data, nw)
    return out


# ---------------------------------------------------------------- restore
def phos_restore_begin(ctx, flags, image, copy_stream) -> int:
    out = ctypes.c_void_p()
    _call("phos_restore_begin", ctx, flags, _ptr(image), _stream(copy_stream), ctypes.byref(out))
    return out.value


def phos_manifest_write(ctx, protocol: int = 0) -> bytes:
    n = U64()
    _call("phos_manifest_write", ctx, protocol, None, 0, ctypes.byref(n))
    buf = ctypes.create_string_buffer(n.value)
    _call("phos_manifest_write", ctx, protocol, buf, n.value, ctypes.byref(n))
    return buf.raw[:n.value]


def phos_manifest_check(ctx, manifest: bytes) -> None:
    _call("phos_manifest_check", ctx, manifest, len(manifest))


def phos_restore_begin_manifest(ctx, flags, image, manifest: bytes, copy_stream) -> int:
    out = ctypes.c_void_p()
    _call("phos_restore_begin_manifest", ctx, flags, _ptr(image), manifest, len(manifest),
          _stream(copy_stream), ctypes.byref(out))
    return out.value


def phos_restore_begin_chunked(ctx, flags, chunks, chunk_bytes, copy_stream) -> int:
    tab = (ctypes.c_void_p * len(chunks))(*[_ptr(x) for x in chunks])
    out = ctypes.c_void_p()
    _call("phos_restore_begin_chunked", ctx, flags, tab, len(chunks), chunk_bytes,
          _stream(copy_stream), ctypes.byref(out))
    return out.value


def phos_restore_on_demand(rs, spec, d_records, n, app_stream, d_faulted=None) -> None:
    _call("phos_restore_on_demand", rs, spec, _ptr(d_records), n, _stream(app_stream),
          _ptr(d_faulted))


def phos_restore_present(rs, n_pages: int) -> np.ndarray:
    nw = (n_pages + 31) // 32
    out = np.zeros(nw, dtype=np.uint32)
    _call("phos_restore_present", rs, out.ctypes.data, nw)
    return out


def phos_restore_end(rs, app_stream) -> phos_rst_stats:
    st = phos_rst_stats()
    _call("phos_restore_end", rs, _stream(app_stream), ctypes.byref(st))
    return st


# ------------------------------------------------------------------ batch
def seg_array(segs) -> np.ndarray:
    a = np.ascontiguousarray(segs, dtype=SEG_DTYPE) if not isinstance(segs, np.ndarray) \
        else np.ascontiguousarray(segs.astype(SEG_DTYPE, copy=False))
    return a


def phos_batch_create(device, max_segs, max_reqs, cfg: Optional[phos_batch_cfg] = None) -> int:
    out = ctypes.c_void_p()
    _call("phos_batch_create", device, max_segs, max_reqs,
          ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(out))
    return out.value


def phos_batch_destroy(b) -> None:
    _call("phos_batch_destroy", b)


def phos_batch_load(b, segs: np.ndarray, stream=None) -> None:
    a = seg_array(segs)
    _call("phos_batch_load", b, a.ctypes.data, a.shape[0], _stream(stream))


def phos_batch_run(b, stream=None) -> None:
    _call("phos_batch_run", b, _stream(stream))


def phos_batch_copy(b, segs: np.ndarray, stream=None) -> None:
    a = seg_array(segs)
    _call("phos_batch_copy", b, a.ctypes.data, a.shape[0], _stream(stream))


def phos_batch_done_bytes(b) -> int:
    out = ctypes.c_void_p()
    _call("phos_batch_done_bytes", b, ctypes.byref(out))
    return out.value


def phos_batch_times(b, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    _call("phos_batch_times", b, out.ctypes.data, n)
    return out


def phos_batch_get_cfg(b) -> phos_batch_cfg:
    c = phos_batch_cfg()
    _call("phos_batch_get_cfg", b, ctypes.byref(c))
    return c


def phos_batch_set_cfg(b, cfg: phos_batch_cfg) -> None:
    _call("phos_batch_set_cfg", b, ctypes.byref(cfg))


def phos_seglist_create(device, segs: np.ndarray) -> int:
    a = seg_array(segs)
    out = ctypes.c_void_p()
    _call("phos_seglist_create", device, a.ctypes.data, a.shape[0], ctypes.byref(out))
    return out.value


def phos_seglist_destroy(l) -> None:
    _call("phos_seglist_destroy", l)


def phos_copy_plain(l, chunk_bytes: int, threads: int, stream=None) -> None:
    _call("phos_copy_plain", l, chunk_bytes, threads, _stream(stream))


def phos_copy_batch(ctx, d_segs, nseg: int, stream=None) -> None:
    """d_segs: device memory holding nseg SEG_DTYPE entries."""
    _call("phos_copy_batch", ctx, _ptr(d_segs), nseg, _stream(stream))


def phos_copy_batch_tuned(ctx, d_segs, nseg: int, stream=None) -> None:
    _call("phos_copy_batch_tuned", ctx, _ptr(d_segs), nseg, _stream(stream))


def phos_batch_tune(device, segs: np.ndarray, cache_path: Optional[str] = None):
    a = seg_array(segs)
    best = phos_batch_cfg()
    ms = ctypes.c_double()
    _call("phos_batch_tune", device, a.ctypes.data, a.shape[0],
          cache_path.encode() if cache_path else None, ctypes.byref(best), ctypes.byref(ms))
    return best, ms.value


# ---------------------------------------------------------------- serving
SERVE_PLAIN, SERVE_BATCHED = 0, 1
REQ_CKPT, REQ_RESTORE, REQ_BURST = 0, 1, 2


class phos_serve_req(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("type", ctypes.c_uint32), ("nseg", ctypes.c_uint32),
                ("bytes", ctypes.c_uint64), ("segs", ctypes.c_void_p),
                ("d_records", ctypes.c_void_p), ("nrec", ctypes.c_uint64),
                ("d_state", ctypes.c_void_p), ("image", ctypes.c_uint64)]


class phos_serve_cfg(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("page_bytes", ctypes.c_uint32),
                ("budget_bytes", ctypes.c_uint64), ("d_arena", ctypes.c_void_p),
                ("quantum_bytes", ctypes.c_uint64), ("iter_bytes", ctypes.c_uint64),
                ("cfg", phos_batch_cfg), ("keep", ctypes.c_uint32), ("_pad", ctypes.c_uint32),
                ("small_bytes", ctypes.c_uint64)]


class phos_serve_out(ctypes.Structure):
    _fields_ = [("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("dst_off", ctypes.c_uint64)]


class phos_serve_stats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("bytes", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("max_active", ctypes.c_uint32)]


SIGNATURES += [("phos_batch_run_plain", [P, P]),
               ("phos_serve_run", [ctypes.c_int, P, P, U32, P, P])]


def phos_batch_run_plain(b, stream=None) -> None:
    _call("phos_batch_run_plain", b, _stream(stream))


def phos_serve_run(device: int, cfg: phos_serve_cfg, reqs, n: int):
    """reqs: ctypes array of phos_serve_req (the caller keeps segment arrays alive)."""
    out = (phos_serve_out * max(1, n))()
    st = phos_serve_stats()
    _call("phos_serve_run", device, ctypes.byref(cfg), reqs, n, out, ctypes.byref(st))
    return out, st
