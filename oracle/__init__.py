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
        L.orc_page_hash.argtypes = [P, U64, U64]
        L.orc_page_hash.restype = U64
        L.orc_hash_pages.argtypes = [P, U64, U64, U64, P]
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


def page_hash(page: np.ndarray, index: int) -> int:
    """64-bit fingerprint of one page's bytes at page index `index` (oracle.h)."""
    page = np.ascontiguousarray(page, dtype=np.uint8)
    return int(lib().orc_page_hash(page.ctypes.data, page.nbytes, index))


def hash_pages(buf: np.ndarray, page_bytes: int, index0: int = 0) -> np.ndarray:
    """Fingerprints of the whole pages of a contiguous host buffer, the first
    numbered index0."""
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    n = buf.nbytes // page_bytes
    out = np.empty(n, dtype=np.uint64)
    if n:
        lib().orc_hash_pages(buf.ctypes.data, page_bytes, n, index0, out.ctypes.data)
    return out


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
        self.hashes: Dict[int, np.ndarray] = {}  # run_stream_hashed: fingerprints of snapshots
        self.last: Optional[np.ndarray] = None   # run_stream_hashed: last victim launch per page


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


# --------------------------------------------------------------------------
# Page sets of the recopy rounds (Sections 4.3 and 7)
# --------------------------------------------------------------------------
def buffer_pages(table: Table, pool_base: int, page_bytes: int, n_pages: int) -> np.ndarray:
    """Byte per pool page: 1 iff some byte of the page belongs to an allocated
    buffer.  Only those pages have a place in the image (Section 2.2: the
    checkpointed state is the buffers), so only they are ever copied."""
    out = np.zeros(n_pages, np.uint8)
    for b, nb in zip(table.base.tolist(), table.bytes.tolist()):
        if nb == 0 or b + nb <= pool_base:
            continue
        lo = max(b, pool_base) - pool_base
        hi = b + nb - pool_base
        out[lo // page_bytes:min((hi - 1) // page_bytes + 1, n_pages)] = 1
    return out


def write_pages(table: Table, arg_lists, pool_base: int, page_bytes: int,
                n_pages: int) -> np.ndarray:
    """Union over launches of the pages of their speculated write intervals:
    what those launches may write without a violation (Section 4.1)."""
    m = np.zeros(n_pages, np.uint8)
    for args in arg_lists:
        write_interval_pages(spec_build(table, args), pool_base, page_bytes, n_pages, m)
    return m


def track_launches(table: Table, n: int, item_fn, pool_base: int, page_bytes: int,
                   n_pages: int, threads: int = 1):
    """Write-set tracking (Section 4.3) of launches 0..n-1, item_fn(j) giving
    launch j's (args, records).  Returns (dirty, victim, last): the OR of
    every launch's dirty and victim pages, and per page the last launch j
    with a failing write inside a buffer there (-1: none).  Launches are
    tracked independently and combined by OR and max, which is what the
    per-launch definition composes to; `threads` only splits the launches."""
    import concurrent.futures as cf

    def part(js):
        d, v = np.zeros(n_pages, np.uint8), np.zeros(n_pages, np.uint8)
        last = np.full(n_pages, -1, np.int64)
        for j in js:
            args, rec = item_fn(j)
            vj = np.zeros(n_pages, np.uint8)
            track(spec_build(table, args), rec, table, pool_base, page_bytes, n_pages, d, vj)
            v |= vj
            last[vj != 0] = j
        return d, v, last

    threads = max(1, min(threads, n)) if n else 1
    parts = [list(range(n))[i::threads] for i in range(threads)]
    dirty, victim = np.zeros(n_pages, np.uint8), np.zeros(n_pages, np.uint8)
    last = np.full(n_pages, -1, np.int64)
    with cf.ThreadPoolExecutor(threads) as ex:
        for d, v, lp in ex.map(part, parts):
            dirty |= d
            victim |= v
            last = np.maximum(last, lp)
    return dirty, victim, last


def precopy_rounds(dirty_per_launch: Sequence[np.ndarray], rounds: Sequence[int],
                   inbuf: np.ndarray):
    """Plain pre-copy rounds of a recopy checkpoint (Sections 4.3 and 7): a
    round before launch r copies every page marked dirty so far and unmarks
    it; later writes mark pages again.  dirty_per_launch[j]: launch j's dirty
    pages.  Returns (the dirty map left for the final recopy, the number of
    image pages the rounds copied)."""
    cur = np.zeros_like(inbuf, dtype=np.uint8)
    copied = 0
    for j, d in enumerate(dirty_per_launch):
        if j in rounds:
            copied += int((cur & inbuf).astype(bool).sum())
            cur[:] = 0
        cur |= d
    return cur, copied


def final_rounds(dirty: np.ndarray, victim: np.ndarray, last: np.ndarray,
                 rounds: Sequence[int], upcoming_pages, inbuf: np.ndarray):
    """Final-page pre-copy rounds (Sections 4.3 and 7, with every launch of the
    window validated up front).  Before launch r, a page is final when no
    launch from r on may write it validly (outside upcoming_pages(r), the
    write-interval pages of launches r, r+1, ...): the dirty pages and the
    victim pages whose last failing write came from a launch before r
    (last[p] < r) are copied and unmarked.  Returns the dirty and victim maps
    left for the recopy at the re-quiesce and the number of image pages the
    rounds copied (a page can be copied by several rounds)."""
    dirty, victim, inbuf = dirty.astype(bool), victim.astype(bool), inbuf.astype(bool)
    copied = 0
    for r in rounds:
        up = upcoming_pages(r).astype(bool)
        fin_v = victim & (last >= 0) & (last < r)
        listed = (dirty | fin_v) & ~up
        copied += int((listed & inbuf).sum())
        dirty &= ~listed
        victim &= ~(fin_v & ~up)
    return dirty, victim, copied


def needed_pages(table: Table, args, rec: np.ndarray, pool_base: int, page_bytes: int,
                 n_pages: int, prefetch: bool = False) -> np.ndarray:
    """Section 6: the pages a launch needs present before it runs: those its
    accesses touch inside buffers; with speculative prefetch, also every page
    of its speculated intervals (read and write) that lies in a buffer."""
    t = np.zeros(n_pages, np.uint8)
    touched_pages(rec, table, pool_base, page_bytes, n_pages, t)
    if prefetch:
        iv = spec_build(table, args).copy()
        iv["mode"] |= W  # every speculated interval, whatever its mode
        s = np.zeros(n_pages, np.uint8)
        write_interval_pages(iv, pool_base, page_bytes, n_pages, s)
        t |= s & buffer_pages(table, pool_base, page_bytes, n_pages)
    return t


def recopy_pages(dirty: np.ndarray, victim: np.ndarray, inbuf: np.ndarray) -> int:
    """Image pages the recopy at the re-quiesce copies: the dirty pages and the
    victim pages (Section 4.3), those inside buffers."""
    return int(((dirty.astype(bool) | victim.astype(bool)) & inbuf.astype(bool)).sum())


# --------------------------------------------------------------------------
# Full-size comparisons: fingerprints of images and pools, and the replay of
# an application stream on a host pool
# --------------------------------------------------------------------------
def _pool_map(fn, items, threads):
    import concurrent.futures as cf
    if threads <= 1:
        return [fn(x) for x in items]
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, items))


def image_hashes_from_pool(pool: np.ndarray, pool_base: int, table: Table, page_bytes: int,
                           threads: int = 1) -> np.ndarray:
    """Page fingerprints of the image a stop-the-world checkpoint of `pool`
    writes (orc_snapshot's layout: buffers back to back in ascending base
    order), in image page order, without building the image.  Buffers are
    whole pages, so image page i is one pool page."""
    n_img = int(table.bytes.sum()) // page_bytes
    out = np.empty(n_img, np.uint64)
    jobs, ip = [], 0
    for b, nb in zip(table.base.tolist(), table.bytes.tolist()):
        assert b % page_bytes == pool_base % page_bytes and nb % page_bytes == 0
        jobs.append((b - pool_base, nb, ip))
        ip += nb // page_bytes

    def one(job):
        off, nb, i0 = job
        out[i0:i0 + nb // page_bytes] = hash_pages(pool[off:off + nb], page_bytes, i0)

    _pool_map(one, jobs, threads)
    return out


def hash_chunks(read_fn, nbytes: int, page_bytes: int, chunk_bytes: int,
                threads: int = 1) -> np.ndarray:
    """Page fingerprints of nbytes of data read chunk by chunk: read_fn(off, n)
    returns bytes [off, off + n) as a host array; page i is numbered i."""
    assert nbytes % page_bytes == 0 and chunk_bytes % page_bytes == 0
    out = np.empty(nbytes // page_bytes, np.uint64)
    off = 0
    while off < nbytes:
        n = min(chunk_bytes, nbytes - off)
        host = read_fn(off, n)
        step = max(page_bytes, (n // max(1, threads)) // page_bytes * page_bytes)
        parts = [(o, min(step, n - o)) for o in range(0, n, step)]

        def one(part, host=host, base=off):
            o, m = part
            i0 = (base + o) // page_bytes
            out[i0:i0 + m // page_bytes] = hash_pages(host[o:o + m], page_bytes, i0)

        _pool_map(one, parts, threads)
        off += n
    return out


def apply_stream(pool: np.ndarray, launches, records_fn, apply_fn, threads: int = 1,
                 ahead: int = 32, log=None, log_every: int = 5000) -> None:
    """Apply launches' writes to a host pool in launch order (the application,
    not the method: each write stores a value fixed by the launch and the
    address).  records_fn(L) is pure, so up to `ahead` launches' records are
    drawn on `threads` host threads while earlier ones are applied.  log(j),
    if given, is called every `log_every` launches."""
    import concurrent.futures as cf
    if threads <= 1:
        for j, L in enumerate(launches):
            apply_fn(pool, L, records_fn(L))
            if log is not None and j % log_every == log_every - 1:
                log(j + 1)
        return
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {}
        nxt = 0
        for j, L in enumerate(launches):
            while nxt < len(launches) and nxt < j + ahead:
                futs[nxt] = ex.submit(records_fn, launches[nxt])
                nxt += 1
            apply_fn(pool, L, futs.pop(j).result())
            if log is not None and j % log_every == log_every - 1:
                log(j + 1)


def validate_launches(table: Table, pool_base: int, launches, records_fn, flags: int = V_READS | V_WRITES,
                      threads: int = 1) -> List[np.ndarray]:
    """Section 4.1 violations of every launch (list in launch order); launches
    are independent, so `threads` only splits them."""
    def one(L):
        return validate(spec_build(table, L.arg_values(pool_base)), records_fn(L), table, L.k, flags)

    return _pool_map(one, list(launches), threads)


def run_stream_hashed(world, launches, pool_base: int, records_fn, apply_fn, pool: np.ndarray,
                      hash_before: Sequence[int] = (), window: Optional[Tuple[int, int]] = None,
                      flags: int = V_READS | V_WRITES, threads: int = 1,
                      ahead: int = 16, log=None) -> StreamResult:
    """run_stream for windows too large to snapshot twice on the host: the same
    per-launch definitions (speculation, validation, tracking, then the
    launch's writes, in launch order), with each launch's records drawn,
    validated and tracked on host threads ahead of the in-order application
    of the writes, and every snapshot replaced by its page fingerprints
    (res.hashes[j], as image_hashes_from_pool).  res.last[p] is the last
    launch position in the window with a failing write inside a buffer on
    page p (-1: none).  log(j), if given, is called every 100 launches (a
    long replay reports its progress)."""
    import concurrent.futures as cf
    table = Table.from_world(world, pool_base)
    npg, page = world.n_pages, world.page_bytes
    res = StreamResult()
    if window is not None:
        res.dirty = np.zeros(npg, np.uint8)
        res.victim = np.zeros(npg, np.uint8)
        res.last = np.full(npg, -1, np.int64)

    def prep(j):
        L = launches[j]
        iv = spec_build(table, L.arg_values(pool_base))
        rec = records_fn(L)
        viol = validate(iv, rec, table, L.k, flags)
        dv = None
        if window is not None and window[0] <= j < window[1]:
            d, v = np.zeros(npg, np.uint8), np.zeros(npg, np.uint8)
            track(iv, rec, table, pool_base, page, npg, d, v)
            dv = (np.flatnonzero(d), np.flatnonzero(v))
        return iv, rec, viol, dv

    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        futs, nxt = {}, 0
        for j, L in enumerate(launches):
            while nxt < len(launches) and nxt < j + ahead:
                futs[nxt] = ex.submit(prep, nxt)
                nxt += 1
            if j in hash_before:
                res.hashes[j] = image_hashes_from_pool(pool, pool_base, table, page, threads)
            iv, rec, viol, dv = futs.pop(j).result()
            res.intervals.append(iv)
            res.violations.append(viol)
            if dv is not None:
                res.dirty[dv[0]] = 1
                res.victim[dv[1]] = 1
                res.last[dv[1]] = j
            apply_fn(pool, L, rec)
            if log is not None and j % 100 == 99:
                log(j + 1)
    if len(launches) in hash_before:
        res.hashes[len(launches)] = image_hashes_from_pool(pool, pool_base, table, page, threads)
    return res


def image_hashes_from_reader(read_fn, pool_base: int, table: Table, page_bytes: int,
                             chunk_bytes: int = 1 << 30, threads: int = 1) -> np.ndarray:
    """As image_hashes_from_pool, for a pool read piece by piece: read_fn(off,
    n) returns pool bytes [off, off + n) (pool-relative) as a host array."""
    n_img = int(table.bytes.sum()) // page_bytes
    out = np.empty(n_img, np.uint64)
    ip = 0
    for b, nb in zip(table.base.tolist(), table.bytes.tolist()):
        assert nb % page_bytes == 0
        off = b - pool_base
        for o in range(0, nb, chunk_bytes):
            n = min(chunk_bytes, nb - o)
            host = read_fn(off + o, n)
            i0 = ip + o // page_bytes
            step = max(page_bytes, (n // max(1, threads)) // page_bytes * page_bytes)

            def one(p, host=host, i0=i0, n=n):
                m = min(step, n - p)
                out[i0 + p // page_bytes:i0 + (p + m) // page_bytes] = hash_pages(
                    host[p:p + m], page_bytes, i0 + p // page_bytes)

            _pool_map(one, range(0, n, step), threads)
        ip += nb // page_bytes
    return out


def gather_hashes(src_fn, src_off, dst_off, nbytes, page_bytes: int, n_dst_pages: int,
                  threads: int = 1, piece_bytes: int = 64 << 20) -> np.ndarray:
    """Page fingerprints of the destination of orc_gather's segment copy
    (dst[dst_off[i] ..) = src[src_off[i] ..), bytes[i] each) without building
    it: src_fn(off, n) returns source bytes [off, off + n) as a host array.
    Segments are whole pages at page-aligned destinations; destination pages
    no segment writes keep the fingerprint 0."""
    out = np.zeros(n_dst_pages, np.uint64)
    jobs = []
    for s, d, n in zip(np.asarray(src_off).tolist(), np.asarray(dst_off).tolist(),
                       np.asarray(nbytes).tolist()):
        assert d % page_bytes == 0 and n % page_bytes == 0
        for o in range(0, n, piece_bytes):
            jobs.append((s + o, d + o, min(piece_bytes, n - o)))

    def one(job):
        s, d, n = job
        out[d // page_bytes:(d + n) // page_bytes] = hash_pages(src_fn(s, n), page_bytes,
                                                                d // page_bytes)

    _pool_map(one, jobs, threads)
    return out
