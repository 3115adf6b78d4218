"""CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct definitions of what the validated-speculation
checkpoint/restore hot path computes (PhoenixOS, arXiv 2405.12079).  Only the
tests, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may use
it; the product library never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, linear scans, one thread); this
file marshals arguments and composes the per-launch definitions into the
protocol-level results the paper defines:

* Section 4.1 — speculated interval sets and runtime validation;
* Section 4.2 — soft copy-on-write: the image equals a stop-the-world snapshot
  at the checkpoint start t1, and a launch's pre-launch copy set is the pages
  it may write that have not been copied yet;
* Section 4.3 — soft recopy: the image equals a snapshot at the re-quiesce
  t2; the recopy set is the dirty pages plus the victim pages;
* Section 6 — concurrent restore: before a launch, the pages it touches that
  are not present yet are brought in.

Parity pins: every function here is pinned by ``tests/test_oracle_pins.py``
(exhaustive tiny pools, injected-equals-flagged, closed-form special cases,
library bisection, snapshot invariants, golden spec cases).
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

R, W = 1, 2
V_READS, V_WRITES = 1, 2
ARG_SCALAR, ARG_PTR_CONST, ARG_PTR_MUT, ARG_STRUCT, ARG_RANGE = 0, 1, 2, 3, 4

INTERVAL_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8"), ("mode", "<u4"), ("_pad", "<u4")])
VIOLATION_DTYPE = np.dtype([("index", "<u8"), ("addr", "<u8"), ("launch_id", "<u4"),
                            ("is_write", "u1"), ("reason", "u1"), ("_p", "<u2"),
                            ("victim", "<i4"), ("_q", "<u4")])
assert VIOLATION_DTYPE.itemsize == 32 and INTERVAL_DTYPE.itemsize == 24


class _Arg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("value", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("host_struct", ctypes.c_void_p)]


_lib = None
P = ctypes.c_void_p
U64, U32 = ctypes.c_uint64, ctypes.c_uint32


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} missing: run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        L.orc_spec_build.argtypes = [P, P, U32, P, U32, P, U32]
        L.orc_spec_build.restype = U32
        L.orc_check.argtypes = [P, U32, U64, ctypes.c_int]
        L.orc_check.restype = ctypes.c_int
        L.orc_victim.argtypes = [P, P, U32, U64]
        L.orc_victim.restype = ctypes.c_int32
        L.orc_validate.argtypes = [P, U32, P, U64, U32, U32, P, P, U32, P, U64]
        L.orc_validate.restype = U64
        L.orc_track.argtypes = [P, U32, P, U64, P, P, U32, U64, U64, U64, P, P]
        L.orc_write_interval_pages.argtypes = [P, U32, U64, U64, U64, P]
        L.orc_touched_pages.argtypes = [P, U64, P, P, U32, U64, U64, U64, P]
        L.orc_snapshot.argtypes = [P, U64, P, P, U32, P]
        L.orc_snapshot.restype = U64
        L.orc_restore.argtypes = [P, U64, P, P, U32, P]
        L.orc_gather.argtypes = [P, P, P, P, P, U64]
        _lib = L
    return _lib


class Table:
    """Allocation table (absolute bases, ascending) kept alive for C calls."""

    def __init__(self, bases: Sequence[int], sizes: Sequence[int]):
        self.base = np.ascontiguousarray(np.asarray(bases, dtype=np.uint64))
        self.bytes = np.ascontiguousarray(np.asarray(sizes, dtype=np.uint64))
        self.n = int(self.base.shape[0])

    @classmethod
    def from_world(cls, world, pool_base: int) -> "Table":
        return cls(world.alloc_off.astype(np.uint64) + np.uint64(pool_base), world.alloc_bytes)

    def c(self):
        return self.base.ctypes.data, self.bytes.ctypes.data, self.n


def spec_build(table: Table, args: Sequence[Tuple[int, int, int, int]],
               structs: Optional[Dict[int, bytes]] = None) -> np.ndarray:
    """args: (kind, mode, value, bytes); structs maps arg position -> struct bytes."""
    structs = structs or {}
    arr = (_Arg * max(1, len(args)))()
    keep = []
    for j, (kind, mode, value, nbytes) in enumerate(args):
        arr[j].kind, arr[j].mode, arr[j].value, arr[j].bytes = kind, mode, value, nbytes
        if j in structs:
            buf = ctypes.create_string_buffer(structs[j], len(structs[j]))
            keep.append(buf)
            arr[j].host_struct = ctypes.addressof(buf)
            arr[j].bytes = len(structs[j])
    cap = sum(max(1, (len(structs.get(j, b"")) // 8)) for j in range(len(args))) + 1
    out = np.zeros(cap, dtype=INTERVAL_DTYPE)
    n = lib().orc_spec_build(*table.c(), arr, len(args), out.ctypes.data, cap)
    return out[:n].copy()


def check(iv: np.ndarray, addr: int, is_write: int) -> int:
    iv = np.ascontiguousarray(iv, dtype=INTERVAL_DTYPE)
    return lib().orc_check(iv.ctypes.data, iv.shape[0], addr, is_write)


def victim(table: Table, addr: int) -> int:
    return lib().orc_victim(*table.c(), addr)


def validate(iv: np.ndarray, rec: np.ndarray, table: Table, launch_id: int = 0,
             flags: int = V_READS | V_WRITES, cap: Optional[int] = None) -> np.ndarray:
    iv = np.ascontiguousarray(iv, dtype=INTERVAL_DTYPE)
    rec = np.ascontiguousarray(rec, dtype=np.uint64)
    cap = rec.shape[0] if cap is None else cap
    out = np.zeros(max(cap, 1), dtype=VIOLATION_DTYPE)
    n = lib().orc_validate(iv.ctypes.data, iv.shape[0], rec.ctypes.data, rec.shape[0], flags,
                           launch_id, *table.c(), out.ctypes.data, cap)
    return out[: min(n, cap)].copy()


def track(iv: np.ndarray, rec: np.ndarray, table: Table, pool_base: int, page_bytes: int,
          n_pages: int, dirty: np.ndarray, victim_pages: np.ndarray) -> None:
    """OR one launch's dirty and victim pages into the byte-per-page arrays."""
    iv = np.ascontiguousarray(iv, dtype=INTERVAL_DTYPE)
    rec = np.ascontiguousarray(rec, dtype=np.uint64)
    assert dirty.dtype == np.uint8 and victim_pages.dtype == np.uint8
    lib().orc_track(iv.ctypes.data, iv.shape[0], rec.ctypes.data, rec.shape[0], *table.c(),
                    pool_base, page_bytes, n_pages, dirty.ctypes.data, victim_pages.ctypes.data)


def write_interval_pages(iv: np.ndarray, pool_base: int, page_bytes: int, n_pages: int,
                         pages: np.ndarray) -> None:
    iv = np.ascontiguousarray(iv, dtype=INTERVAL_DTYPE)
    lib().orc_write_interval_pages(iv.ctypes.data, iv.shape[0], pool_base, page_bytes, n_pages,
                                   pages.ctypes.data)


def touched_pages(rec: np.ndarray, table: Table, pool_base: int, page_bytes: int, n_pages: int,
                  pages: np.ndarray) -> None:
    rec = np.ascontiguousarray(rec, dtype=np.uint64)
    lib().orc_touched_pages(rec.ctypes.data, rec.shape[0], *table.c(), pool_base, page_bytes,
                            n_pages, pages.ctypes.data)


def snapshot(pool: np.ndarray, pool_base: int, table: Table) -> np.ndarray:
    img = np.empty(int(table.bytes.sum()), dtype=np.uint8)
    lib().orc_snapshot(pool.ctypes.data, pool_base, *table.c(), img.ctypes.data)
    return img


def restore(pool: np.ndarray, pool_base: int, table: Table, image: np.ndarray) -> None:
    lib().orc_restore(pool.ctypes.data, pool_base, *table.c(), image.ctypes.data)


def gather(src: np.ndarray, dst: np.ndarray, src_off, dst_off, nbytes) -> None:
    s = np.ascontiguousarray(src_off, dtype=np.uint64)
    d = np.ascontiguousarray(dst_off, dtype=np.uint64)
    b = np.ascontiguousarray(nbytes, dtype=np.uint64)
    lib().orc_gather(src.ctypes.data, dst.ctypes.data, s.ctypes.data, d.ctypes.data,
                     b.ctypes.data, s.shape[0])


def page_set(pages: np.ndarray) -> np.ndarray:
    """Byte-per-page array -> sorted page indices."""
    return np.flatnonzero(pages).astype(np.uint64)


def pages_to_bitmap(pages: np.ndarray, n_pages: int) -> np.ndarray:
    """Byte-per-page array -> little-endian 32-bit words, bit p%32 of word p//32."""
    nwords = (n_pages + 31) // 32
    padded = np.zeros(nwords * 32, dtype=np.uint8)
    padded[:n_pages] = pages[:n_pages] != 0
    return np.packbits(padded, bitorder="little").view(np.uint32).copy()


# --------------------------------------------------------------------------
# Protocol-level definitions
# --------------------------------------------------------------------------
class StreamResult:
    """Everything the oracle derives from one application stream."""

    def __init__(self):
        self.intervals: List[np.ndarray] = []
        self.violations: List[np.ndarray] = []
        self.snapshots: Dict[int, np.ndarray] = {}
        self.dirty: Optional[np.ndarray] = None
        self.victim: Optional[np.ndarray] = None
        self.cow_sets: List[np.ndarray] = []  # per launch in the CoW window
        self.fault_sets: List[np.ndarray] = []


def run_stream(world, launches, pool_base: int, records_fn, apply_fn, pool: np.ndarray,
               snap_before: Sequence[int] = (), window: Optional[Tuple[int, int]] = None,
               cow_window: Optional[Tuple[int, int]] = None, flags: int = V_READS | V_WRITES,
               keep_violations: bool = True) -> StreamResult:
    """Replay launches on a host pool.

    snap_before: launch positions j at which the image is snapshotted before
    launch j runs (len(launches) = after the last launch).
    window = (j0, j1): launches j0..j1-1 are tracked (dirty / victim pages).
    cow_window = (j0, j1): for launch j in it, the pre-launch copy set is
    (pages of its write intervals U pages of its violating writes inside
    buffers) minus everything copied by earlier launches of the window
    (Section 4.2 with the background copy paused).
    """
    table = Table.from_world(world, pool_base)
    res = StreamResult()
    npg = world.n_pages
    if window is not None:
        res.dirty = np.zeros(npg, np.uint8)
        res.victim = np.zeros(npg, np.uint8)
    copied = np.zeros(npg, np.uint8)
    for j, L in enumerate(launches):
        if j in snap_before:
            res.snapshots[j] = snapshot(pool, pool_base, table)
        iv = spec_build(table, L.arg_values(pool_base))
        res.intervals.append(iv)
        rec = records_fn(L)
        if keep_violations:
            res.violations.append(validate(iv, rec, table, L.k, flags))
        if window is not None and window[0] <= j < window[1]:
            track(iv, rec, table, pool_base, world.page_bytes, npg, res.dirty, res.victim)
        if cow_window is not None and cow_window[0] <= j < cow_window[1]:
            want = np.zeros(npg, np.uint8)
            write_interval_pages(iv, pool_base, world.page_bytes, npg, want)
            d = np.zeros(npg, np.uint8)
            v = np.zeros(npg, np.uint8)
            track(iv, rec, table, pool_base, world.page_bytes, npg, d, v)
            want |= v
            new = want & (1 - copied)
            res.cow_sets.append(page_set(new))
            copied |= new
        apply_fn(pool, L, rec)
    if len(launches) in snap_before:
        res.snapshots[len(launches)] = snapshot(pool, pool_base, table)
    return res
