"""Seeded synthetic workloads (inputs only; no checkpoint/restore arithmetic).

This module describes the *application* whose GPU memory is checkpointed: the
buffer layout of its device pool, its kernel launches (arguments and the
8-byte access records each launch issues), the initial pool contents, and the
values its kernels store.  Both the CPU oracle and the GPU harness draw their
inputs from here, so they see bit-identical inputs.

* Integer draws: splitmix64 output function over a Weyl counter
  (Steele, Lea, Flood, OOPSLA 2014) and Lemire's multiply-high reduction
  (ACM TOMACS 2019).  ``synth_gen.h`` holds the C/HIP versions; the Python
  versions below are the same formulas for the small host-side draws.
* Log-uniform real draws (``lo * (hi/lo)**u``, ``u = (r >> 11) * 2**-53``)
  happen only here, on the host, when a layout is built; the layout is then a
  plain integer table that both sides read.

The workload shapes follow the paper's evaluation: buffer counts and sizes of
its applications (Table ``tab:app-data-full``), per-kernel argument lists with
a handful of buffers (Section 4.1), and the write-set share of a training step.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30

# stream tags shared with synth_gen.h
T_INJ, T_KIND, T_POS, T_RW, T_POS2, T_CONTENT, T_WVAL, T_PRESENT = 1, 2, 3, 4, 5, 6, 7, 8
# host-only layout / launch tags
T_L_SIZE, T_L_GAP, T_L_PERM, T_L_WSET = 16, 17, 18, 19
T_LN, T_LB, T_LM, T_LI, T_LO, T_LS, T_LSV, T_LW = 20, 21, 22, 23, 24, 25, 26, 27
T_R_SIZE, T_R_NBUF, T_R_SHARE, T_R_FRAC, T_R_ORDER, T_R_SCAT = 32, 33, 34, 35, 36, 37
T_S_ARR, T_S_TYPE, T_S_SIZE, T_S_SRC, T_S_FRAC, T_S_RUNS, T_S_PARTS = 48, 49, 50, 51, 52, 53, 54

# argument kinds (same meaning as the launch-argument kinds of the library)
ARG_SCALAR, ARG_PTR_CONST, ARG_PTR_MUT, ARG_STRUCT, ARG_RANGE = 0, 1, 2, 3, 4
MODE_R, MODE_W = 1, 2

INJ_PER_MILLE_DEFAULT = 1  # 0.1 % of accesses are injected out of speculation


def mix(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def key(seed: int, tag: int, a: int) -> int:
    s = mix((seed + GOLDEN * (tag + 1)) & M64)
    return mix((s + GOLDEN * (a + 1)) & M64)


def at(k: int, b: int) -> int:
    return mix((k + GOLDEN * (b + 1)) & M64)


def draw(seed: int, tag: int, a: int, b: int) -> int:
    return at(key(seed, tag, a), b)


def below(r: int, n: int) -> int:
    return (r * n) >> 64


def unit(r: int) -> float:
    return (r >> 11) * (2.0 ** -53)


def loguniform(r: int, lo: float, hi: float) -> float:
    return lo * (hi / lo) ** unit(r)


def round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def inj_threshold(per_mille: float) -> int:
    """Records whose draw is below this are injected: floor(2^64 * p)."""
    return int(per_mille * (1 << 64)) // 1000


# --------------------------------------------------------------------------
# World = pool layout
# --------------------------------------------------------------------------
@dataclass
class World:
    seed: int
    pool_bytes: int
    page_bytes: int
    alloc_off: np.ndarray  # uint64, ascending
    alloc_bytes: np.ndarray  # uint64
    inj_per_mille: float = INJ_PER_MILLE_DEFAULT
    name: str = "world"
    free_off: np.ndarray = field(init=False)
    free_bytes: np.ndarray = field(init=False)
    free_cum: np.ndarray = field(init=False)

    def __post_init__(self):
        self.alloc_off = np.asarray(self.alloc_off, dtype=np.uint64)
        self.alloc_bytes = np.asarray(self.alloc_bytes, dtype=np.uint64)
        fo, fb = [], []
        cur = 0
        for o, b in zip(self.alloc_off.tolist(), self.alloc_bytes.tolist()):
            if o > cur:
                fo.append(cur)
                fb.append(o - cur)
            cur = o + b
        if self.pool_bytes > cur:
            fo.append(cur)
            fb.append(self.pool_bytes - cur)
        self.free_off = np.asarray(fo, dtype=np.uint64)
        self.free_bytes = np.asarray(fb, dtype=np.uint64)
        cum = np.zeros(len(fb), dtype=np.uint64)
        if len(fb) > 1:
            cum[1:] = np.cumsum(np.asarray(fb[:-1], dtype=np.uint64))
        self.free_cum = cum

    @property
    def n_alloc(self) -> int:
        return int(self.alloc_off.shape[0])

    @property
    def free_total(self) -> int:
        return int(self.free_bytes.sum()) if self.free_bytes.size else 0

    @property
    def image_bytes(self) -> int:
        return int(self.alloc_bytes.sum())

    @property
    def n_pages(self) -> int:
        return self.pool_bytes // self.page_bytes

    def buffers(self, pool_base: int) -> List[Tuple[int, int]]:
        return [(pool_base + int(o), int(b)) for o, b in zip(self.alloc_off, self.alloc_bytes)]


def layout_from_sizes(seed: int, sizes: Sequence[int], page: int, pool_bytes: int,
                      name: str, inj_per_mille: float = INJ_PER_MILLE_DEFAULT,
                      max_gap_pages: int = 2) -> World:
    """Place buffers in the given order: gap_i = page * U{0..max_gap_pages}, then buffer i."""
    for attempt in range(64):
        offs, cur = [], 0
        for i, s in enumerate(sizes):
            cur += page * below(draw(seed, T_L_GAP, attempt, i), max_gap_pages + 1)
            offs.append(cur)
            cur += int(s)
        if cur <= pool_bytes:
            return World(seed, pool_bytes, page, np.asarray(offs, np.uint64),
                         np.asarray(sizes, np.uint64), inj_per_mille, name)
    raise ValueError("buffers do not fit in the pool")


def layout_random(seed: int, n_buffers: int, page: int, pool_bytes: int, lo: int, hi: int,
                  name: str = "random", inj_per_mille: float = INJ_PER_MILLE_DEFAULT) -> World:
    """n buffers with sizes log-uniform in [lo, hi] rounded up to pages (redrawn if too big)."""
    for attempt in range(64):
        sizes = [round_up(int(loguniform(draw(seed, T_L_SIZE, attempt, i), lo, hi)), page)
                 for i in range(n_buffers)]
        if sum(sizes) + n_buffers * 2 * page <= pool_bytes:
            return layout_from_sizes(seed, sizes, page, pool_bytes, name, inj_per_mille)
    raise ValueError("cannot draw a layout that fits")


def permutation(seed: int, tag: int, n: int) -> List[int]:
    p = list(range(n))
    for i in range(n - 1, 0, -1):
        j = below(draw(seed, tag, 0, i), i + 1)
        p[i], p[j] = p[j], p[i]
    return p


# --------------------------------------------------------------------------
# Launches
# --------------------------------------------------------------------------
@dataclass
class Launch:
    k: int
    named: List[Tuple[int, int]]  # (allocation index, mutable?) in naming order
    args: List[Tuple[int, int, int, int]]  # (kind, mode, value (offset for pointers), bytes)
    n_records: int

    def arg_values(self, pool_base: int) -> List[Tuple[int, int, int, int]]:
        out = []
        for kind, mode, v, b in self.args:
            if kind in (ARG_PTR_CONST, ARG_PTR_MUT, ARG_RANGE):
                v = (v + pool_base) & M64
            out.append((kind, mode, v, b))
        return out


def _named_args(seed: int, world: World, k: int, named: List[Tuple[int, int]],
                interior: bool = True) -> List[Tuple[int, int, int, int]]:
    args = []
    for j, (idx, mut) in enumerate(named):
        off = int(world.alloc_off[idx])
        nb = int(world.alloc_bytes[idx])
        if interior and below(draw(seed, T_LI, k, j), 4) == 0:
            off += 8 * below(draw(seed, T_LO, k, j), nb // 8)
        args.append((ARG_PTR_MUT if mut else ARG_PTR_CONST, 0, off, 0))
    ns = below(draw(seed, T_LS, k, 0), 3)
    for s in range(ns):
        args.append((ARG_SCALAR, 0, below(draw(seed, T_LSV, k, s), 1 << 20), 0))
    return args


def _pick_distinct(seed: int, k: int, n: int, universe: int) -> List[int]:
    picks, c = [], 0
    n = min(n, universe)
    while len(picks) < n:
        idx = below(draw(seed, T_LB, k, c), universe)
        c += 1
        if idx not in picks:
            picks.append(idx)
    return picks


def launches_uniform(world: World, n_launch: int, n_records: int, k0: int = 0,
                     max_named: int = 8) -> List[Launch]:
    """Each launch names U{1..max_named} distinct buffers, each mutable with p = 1/2."""
    out = []
    for k in range(k0, k0 + n_launch):
        nk = 1 + below(draw(world.seed, T_LN, k, 0), max_named)
        picks = _pick_distinct(world.seed, k, nk, world.n_alloc)
        named = [(idx, draw(world.seed, T_LM, k, j) & 1) for j, idx in enumerate(picks)]
        out.append(Launch(k, named, _named_args(world.seed, world, k, named), n_records))
    return out


def launch_custom(world: World, k: int, named: List[Tuple[int, int]], n_records: int,
                  extra_args: Sequence[Tuple[int, int, int, int]] = ()) -> Launch:
    args = [(ARG_PTR_MUT if m else ARG_PTR_CONST, 0, int(world.alloc_off[i]), 0) for i, m in named]
    return Launch(k, list(named), args + list(extra_args), n_records)


# --------------------------------------------------------------------------
# The five workload shapes
# --------------------------------------------------------------------------
CFG_SEED = 0x50484F53


def config1_world(seed: int = CFG_SEED + 1) -> World:
    """64 MiB pool, 256 buffers log-uniform 4 KiB..1 MiB, 4 KiB pages."""
    return layout_random(seed, 256, 4 * KiB, 64 * MiB, 4 * KiB, 1 * MiB, name="plain-tiny-64MiB")


def config1_launches(world: World, n_launch: int = 100, n_records: int = 1_000_000) -> List[Launch]:
    return launches_uniform(world, n_launch, n_records)


def config2_world(seed: int = CFG_SEED + 2) -> World:
    """16 GiB of buffers: 12 layers of bf16 weights 4096x4096 / 4096x14336 with fp32 Adam
    moments of equal element counts, 80 activations (8..256 MiB, scaled so the total is
    exactly 16 GiB) and 1,848 small buffers (64 KiB..4 MiB); 64 KiB pages."""
    page = 64 * KiB
    named = []
    for _layer in range(12):
        a, b = 4096 * 4096, 4096 * 14336
        named += [2 * a, 2 * b, 4 * a, 4 * a, 4 * b, 4 * b]
    small = [round_up(int(loguniform(draw(seed, T_L_SIZE, 2, i), 64 * KiB, 4 * MiB)), page)
             for i in range(1848)]
    act_raw = [loguniform(draw(seed, T_L_SIZE, 1, i), 8 * MiB, 256 * MiB) for i in range(80)]
    target = 16 * GiB - sum(named) - sum(small)
    f = target / sum(act_raw)
    act = [round_up(int(x * f), page) for x in act_raw[:-1]]
    act.append(target - sum(act))
    assert act[-1] > 0 and act[-1] % page == 0
    sizes = named + act + small
    perm = permutation(seed, T_L_PERM, len(sizes))
    sizes = [sizes[p] for p in perm]
    return layout_from_sizes(seed, sizes, page, 16 * GiB + 320 * MiB, "training-step-16GiB")


def config2_write_set(world: World) -> List[int]:
    """A seeded set of buffers holding 30 % +- 1 % of the pool's buffer bytes."""
    total = world.image_bytes
    lo, hi = int(0.29 * total), int(0.31 * total)
    acc, ws = 0, []
    for idx in permutation(world.seed, T_L_WSET, world.n_alloc):
        b = int(world.alloc_bytes[idx])
        if acc + b <= hi:
            ws.append(idx)
            acc += b
        if acc >= lo:
            break
    return sorted(ws)


def config2_launches(world: World, n_launch: int = 1000, n_records: int = 1_000_000,
                     write_set: Optional[List[int]] = None) -> List[Launch]:
    """Only write-set buffers may be named through mutable pointers; with p = 0.8 a
    launch names at least one write-set buffer mutably."""
    ws = write_set if write_set is not None else config2_write_set(world)
    wss = set(ws)
    out = []
    for k in range(n_launch):
        nk = 1 + below(draw(world.seed, T_LN, k, 0), 8)
        picks = _pick_distinct(world.seed, k, nk, world.n_alloc)
        named = [(idx, (draw(world.seed, T_LM, k, j) & 1) if idx in wss else 0)
                 for j, idx in enumerate(picks)]
        if below(draw(world.seed, T_LW, k, 0), 10) < 8 and not any(m for _, m in named):
            c = 0
            while True:
                cand = ws[below(draw(world.seed, T_LW, k, 1 + c), len(ws))]
                c += 1
                if cand not in picks or named[0][0] == cand:
                    break
            named[0] = (cand, 1)
        out.append(Launch(k, named, _named_args(world.seed, world, k, named), n_records))
    return out


def config5_world(seed: int = CFG_SEED + 5) -> World:
    """70 GiB image of 500 buffers (16..512 MiB, scaled to exactly 70 GiB); 64 KiB pages."""
    page = 64 * KiB
    raw = [loguniform(draw(seed, T_L_SIZE, 0, i), 16 * MiB, 512 * MiB) for i in range(500)]
    target = 70 * GiB
    f = target / sum(raw)
    sizes = [round_up(int(x * f), page) for x in raw[:-1]]
    sizes.append(target - sum(sizes))
    assert sizes[-1] > 0
    return layout_from_sizes(seed, sizes, page, 70 * GiB + 128 * MiB, "cold-start-70GiB")


def config5_roles(world: World) -> Tuple[List[int], List[int]]:
    """(read-only weight buffers, KV/activation buffers) in base order; the smallest
    10 % of buffers are the KV/activation buffers."""
    order = sorted(range(world.n_alloc), key=lambda i: (int(world.alloc_bytes[i]), i))
    wset = set(order[: world.n_alloc // 10])
    rl = [i for i in range(world.n_alloc) if i not in wset]
    wl = [i for i in range(world.n_alloc) if i in wset]
    return rl, wl


def config5_launches(world: World, n_launch: int = 40_000, n_records: int = 262_144,
                     k0: int = 0) -> List[Launch]:
    """Decode-like sweep in base order: each launch names 1..5 consecutive weight
    buffers (read-only) and the layer's KV/activation buffer (mutable)."""
    rl, wl = config5_roles(world)
    wbases = [int(world.alloc_off[i]) for i in wl]
    out, cur = [], 0
    # replay the cursor deterministically up to k0
    for k in range(0, k0 + n_launch):
        nk = 2 + below(draw(world.seed, T_LN, k, 0), 5)
        picks = [rl[(cur + j) % len(rl)] for j in range(nk - 1)]
        cur = (cur + nk - 1) % len(rl)
        if k < k0:
            continue
        b0 = int(world.alloc_off[picks[0]])
        wi = next((j for j, b in enumerate(wbases) if b >= b0), 0)
        named = [(i, 0) for i in picks] + [(wl[wi], 1)]
        out.append(Launch(k, named, _named_args(world.seed, world, k, named, interior=False),
                          n_records))
    return out


# --------------------------------------------------------------------------
# C structs and bindings
# --------------------------------------------------------------------------
class SynthWorld(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("pool_base", ctypes.c_uint64),
                ("inj_threshold", ctypes.c_uint64), ("n_alloc", ctypes.c_uint32),
                ("n_free", ctypes.c_uint32), ("alloc_off", ctypes.c_void_p),
                ("alloc_bytes", ctypes.c_void_p), ("free_off", ctypes.c_void_p),
                ("free_cum", ctypes.c_void_p), ("free_total", ctypes.c_uint64)]


class SynthLaunch(ctypes.Structure):
    _fields_ = [("n_named", ctypes.c_uint32), ("n_const", ctypes.c_uint32),
                ("named_bytes_total", ctypes.c_uint64), ("const_bytes_total", ctypes.c_uint64),
                ("named_off", ctypes.c_uint64 * 8), ("named_bytes", ctypes.c_uint64 * 8),
                ("named_mut", ctypes.c_uint32 * 8), ("named_idx_sorted", ctypes.c_uint32 * 8)]


def c_launch(world: World, L: Launch) -> SynthLaunch:
    s = SynthLaunch()
    s.n_named = len(L.named)
    tot = ctot = nconst = 0
    for j, (idx, mut) in enumerate(L.named):
        s.named_off[j] = int(world.alloc_off[idx])
        s.named_bytes[j] = int(world.alloc_bytes[idx])
        s.named_mut[j] = int(mut)
        tot += int(world.alloc_bytes[idx])
        if not mut:
            nconst += 1
            ctot += int(world.alloc_bytes[idx])
    for j, idx in enumerate(sorted(i for i, _ in L.named)):
        s.named_idx_sorted[j] = idx
    s.n_const, s.named_bytes_total, s.const_bytes_total = nconst, tot, ctot
    return s


def c_launch_array(world: World, launches: Sequence[Launch]):
    arr = (SynthLaunch * len(launches))()
    for j, L in enumerate(launches):
        arr[j] = c_launch(world, L)
    return arr


_host = None


def host_lib():
    global _host
    if _host is None:
        path = os.path.join(HERE, "libsynth_host.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} missing: run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        lib.synth_records_host.argtypes = [ctypes.POINTER(SynthWorld), ctypes.POINTER(SynthLaunch),
                                           ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_void_p]
        lib.synth_content_host.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_void_p]
        lib.synth_apply_writes_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                                ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                                ctypes.c_uint64]
        for f in ("synth_mix_host",):
            getattr(lib, f).argtypes = [ctypes.c_uint64]
            getattr(lib, f).restype = ctypes.c_uint64
        lib.synth_draw_host.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64]
        lib.synth_draw_host.restype = ctypes.c_uint64
        lib.synth_present_host.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                           ctypes.c_void_p]
        lib.synth_below_host.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_below_host.restype = ctypes.c_uint64
        _host = lib
    return _host


class HostWorld:
    """A World bound to a pool base, with its C-side tables kept alive."""

    def __init__(self, world: World, pool_base: int):
        self.world, self.pool_base = world, pool_base
        self._keep = [np.ascontiguousarray(a, dtype=np.uint64) for a in
                      (world.alloc_off, world.alloc_bytes, world.free_off, world.free_cum)]
        self.c = SynthWorld(world.seed, pool_base, inj_threshold(world.inj_per_mille),
                            world.n_alloc, len(world.free_off),
                            *[a.ctypes.data for a in self._keep], world.free_total)


def records_host(hw: HostWorld, L: Launch, i0: int = 0, n: Optional[int] = None) -> np.ndarray:
    n = L.n_records - i0 if n is None else n
    out = np.empty(n, dtype=np.uint64)
    cl = c_launch(hw.world, L)
    host_lib().synth_records_host(ctypes.byref(hw.c), ctypes.byref(cl), L.k, i0, n,
                                  out.ctypes.data)
    return out


def content_host(seed: int, byte0: int, nbytes: int) -> np.ndarray:
    out = np.empty(nbytes, dtype=np.uint8)
    host_lib().synth_content_host(seed, byte0, nbytes, out.ctypes.data)
    return out


def content_host_parallel(seed: int, byte0: int, nbytes: int, threads: int = 16,
                          out: Optional[np.ndarray] = None) -> np.ndarray:
    """content_host in slices on host threads (the C generator releases the GIL)."""
    import concurrent.futures as cf
    out = np.empty(nbytes, dtype=np.uint8) if out is None else out
    step = max(4, (nbytes // max(1, threads) + 3) // 4 * 4)
    L = host_lib()

    def one(o):
        n = min(step, nbytes - o)
        L.synth_content_host(seed, byte0 + o, n, out[o:o + n].ctypes.data)

    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(one, range(0, nbytes, step)))
    return out


def apply_writes_host(pool: np.ndarray, pool_base: int, seed: int, k: int, rec: np.ndarray):
    rec = np.ascontiguousarray(rec, dtype=np.uint64)
    host_lib().synth_apply_writes_host(pool.ctypes.data, pool_base, pool.nbytes, seed, k,
                                       rec.ctypes.data, rec.shape[0])


# --------------------------------------------------------------------------
# Device side (HIP): the same generator on the GPU, driven through torch
# tensors for memory and streams.
# --------------------------------------------------------------------------
_dev = None


def dev_lib():
    global _dev
    if _dev is None:
        path = os.path.join(HERE, "libsynth_dev.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} missing: run __graft_entry__.build()")
        # torch's HSA runtime first, so that the process has only one (it
        # satisfies this library's libhsa-runtime64.so.1)
        import torch  # noqa: F401
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.synth_dev_records.argtypes = [ctypes.POINTER(SynthWorld), P, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint64, P, P]
        lib.synth_dev_content.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, P]
        lib.synth_dev_apply_writes.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_uint32, P, ctypes.c_uint64, P]
        lib.synth_dev_present.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, P]
        for f in (lib.synth_dev_records, lib.synth_dev_content, lib.synth_dev_apply_writes,
                  lib.synth_dev_present):
            f.restype = ctypes.c_int
        _dev = lib
    return _dev


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what}: hipError {rc}")


def _sh(stream):
    return None if stream is None else int(getattr(stream, "cuda_stream", stream))


class DeviceWorld:
    """A World bound to a device pool; its tables live in device memory."""

    def __init__(self, world: World, pool_base: int, device: str = "cuda"):
        import torch
        self.world, self.pool_base = world, pool_base
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)
                                      if a.size else np.zeros(1, np.int64)).to(device)
        self._keep = [t(world.alloc_off), t(world.alloc_bytes), t(world.free_off), t(world.free_cum)]
        self.c = SynthWorld(world.seed, pool_base, inj_threshold(world.inj_per_mille),
                            world.n_alloc, len(world.free_off),
                            *[x.data_ptr() for x in self._keep], world.free_total)


def records_device(dw: DeviceWorld, launches: Sequence[Launch], n_per: int, out=None, stream=None):
    """Records of consecutive launches (launches[j].k == launches[0].k + j), n_per each,
    into a (len(launches) * n_per,) int64 tensor (bit pattern = uint64 records)."""
    import torch
    ks = [L.k for L in launches]
    assert ks == list(range(ks[0], ks[0] + len(ks))), "launches must be consecutive"
    arr = c_launch_array(dw.world, launches)
    d_l = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to("cuda")
    if out is None:
        out = torch.empty(len(launches) * n_per, dtype=torch.int64, device="cuda")
    _check(dev_lib().synth_dev_records(ctypes.byref(dw.c), d_l.data_ptr(), len(launches), ks[0],
                                       n_per, out.data_ptr(), _sh(stream)), "synth_dev_records")
    if stream is None:
        torch.cuda.synchronize()
    else:
        stream.synchronize()
    del d_l
    return out


def content_device(pool, seed: int, stream=None):
    _check(dev_lib().synth_dev_content(pool.data_ptr(), pool.numel() * pool.element_size(), seed,
                                       _sh(stream)), "synth_dev_content")


def apply_writes_device(pool_ptr: int, pool_base: int, pool_bytes: int, seed: int, k: int,
                        rec_ptr: int, n: int, stream=None):
    _check(dev_lib().synth_dev_apply_writes(pool_ptr, pool_base, pool_bytes, seed, k, rec_ptr, n,
                                            _sh(stream)), "synth_dev_apply_writes")


# --------------------------------------------------------------------------
# Batched checkpoint requests (many processes' dirty pages at once)
# --------------------------------------------------------------------------
@dataclass
class Request:
    r: int
    pages: int            # image size in pages
    dirty_start: np.ndarray  # run starts (pages, ascending)
    dirty_len: np.ndarray    # run lengths (pages)
    src_off: int = 0      # offset of the request's memory in the source arena
    dst_off: int = 0      # offset of its delta in the destination arena

    @property
    def dirty_pages(self) -> int:
        return int(self.dirty_len.sum())


def request_dirty_runs(seed: int, r: int, pages: int, frac_lo: float = 0.05,
                       frac_hi: float = 0.60) -> Tuple[np.ndarray, np.ndarray]:
    """Dirty pages of one request: U{50..5000} buffers with log-uniform shares
    (>= 1 page each); whole buffers in a seeded order while they fit in 0.9 f,
    then scattered single pages up to f, f ~ U(frac_lo, frac_hi)."""
    nb = min(pages, 50 + below(draw(seed, T_R_NBUF, r, 0), 4951))
    rng = np.random.Generator(np.random.PCG64(draw(seed, T_R_SHARE, r, 0)))
    raw = np.exp(rng.random(nb) * math.log(1000.0))
    sizes = np.maximum(1, np.floor(raw / raw.sum() * (pages - nb)).astype(np.int64) + 1)
    sizes[np.argmax(sizes)] += pages - int(sizes.sum())
    assert sizes.min() >= 1 and int(sizes.sum()) == pages
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    f = frac_lo + (frac_hi - frac_lo) * unit(draw(seed, T_R_FRAC, r, 0))
    target = int(f * pages)
    dirty = np.zeros(pages, dtype=bool)
    acc = 0
    for b in rng.permutation(nb):
        if acc + sizes[b] <= 0.9 * target:
            dirty[starts[b]:starts[b] + sizes[b]] = True
            acc += int(sizes[b])
    free = np.flatnonzero(~dirty)
    need = max(0, target - acc)
    if need:
        dirty[rng.choice(free, size=min(need, free.size), replace=False)] = True
    d = np.concatenate([[False], dirty, [False]]).astype(np.int8)
    edges = np.diff(d)
    rs = np.flatnonzero(edges == 1)
    re_ = np.flatnonzero(edges == -1)
    return rs.astype(np.int64), (re_ - rs).astype(np.int64)


def batch_requests(seed: int, n_req: int, lo: int, hi: int, page: int) -> List[Request]:
    """n requests, image sizes log-uniform in [lo, hi] rounded to pages; sources
    and compact deltas laid out back to back in two arenas."""
    reqs, so, do = [], 0, 0
    for r in range(n_req):
        size = round_up(int(loguniform(draw(seed, T_R_SIZE, r, 0), lo, hi)), page)
        pages = size // page
        st, ln = request_dirty_runs(seed, r, pages)
        q = Request(r, pages, st, ln, so, do)
        so += size
        do += q.dirty_pages * page
        reqs.append(q)
    return reqs


def config3_requests(seed: int = CFG_SEED + 3, n_req: int = 64) -> List[Request]:
    """64 checkpoint requests, images 100 MiB .. 8 GiB, 64 KiB pages."""
    return batch_requests(seed, n_req, 100 * MiB, 8 * GiB, 64 * KiB)


def request_segments(reqs: Sequence[Request], src_base: int, dst_base: int, page: int,
                     req_ids: Optional[Sequence[int]] = None) -> np.ndarray:
    """Copy segments (src, dst, bytes, req) of the requests' dirty runs: each
    run of the source copied, in ascending page order, into the compact delta."""
    dt = np.dtype([("src", "<u8"), ("dst", "<u8"), ("bytes", "<u8"), ("req", "<u4"),
                   ("_p", "<u4")])
    parts = []
    for j, q in enumerate(reqs):
        n = q.dirty_start.shape[0]
        a = np.zeros(n, dtype=dt)
        ln = q.dirty_len.astype(np.uint64) * np.uint64(page)
        a["src"] = np.uint64(src_base + q.src_off) + q.dirty_start.astype(np.uint64) * np.uint64(page)
        pre = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
        a["dst"] = np.uint64(dst_base + q.dst_off) + pre
        a["bytes"] = ln
        a["req"] = q.r if req_ids is None else req_ids[j]
        parts.append(a)
    return np.concatenate(parts) if parts else np.zeros(0, dtype=dt)


def present_device(state, seed: int, r: int, stream=None):
    """Claim words of burst r's pages: 2 (present) with p = 1/2, else 0."""
    _check(dev_lib().synth_dev_present(state.data_ptr(), state.numel(), seed, r, _sh(stream)),
           "synth_dev_present")


def present_host(seed: int, r: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    host_lib().synth_present_host(seed, r, n, out.ctypes.data)
    return out


# --------------------------------------------------------------------------
# Serving trace: Poisson arrivals of checkpoint / restore / fault-burst requests
# --------------------------------------------------------------------------
REQ_CKPT, REQ_RESTORE, REQ_BURST = 0, 1, 2


@dataclass
class ServeReq:
    r: int
    arrival_s: float
    type: int
    size: int            # bytes (page multiple)
    src_off: int         # offset of the request's memory / image in the source arena
    runs: Optional[Tuple[np.ndarray, np.ndarray]] = None  # checkpoint: dirty runs (pages)
    parts: Optional[List[int]] = None                     # burst: named eighths of the region
    n_rec: int = 0


def serving_trace(seed: int, rate: float, duration_s: float, lo: int, hi: int, page: int,
                  arena_bytes: int, mix=(0.7, 0.2, 0.1), burst_records: int = 65536,
                  frac_lo: float = 0.05, frac_hi: float = 0.60) -> List[ServeReq]:
    """Poisson arrivals (rate per second) over duration_s; sizes log-uniform in
    [lo, hi]; checkpoints copy dirty runs (f ~ U(frac_lo, frac_hi), 16..255 runs)
    into a resident image; restores copy the whole image into the process;
    bursts fault in the pages their accesses touch over 1..8 eighths of the
    region, with half the pages present beforehand."""
    out, t, r = [], 0.0, 0
    while True:
        t += -math.log(1.0 - unit(draw(seed, T_S_ARR, r, 0))) / rate
        if t > duration_s:
            return out
        v = unit(draw(seed, T_S_TYPE, r, 0))
        ty = REQ_CKPT if v < mix[0] else (REQ_RESTORE if v < mix[0] + mix[1] else REQ_BURST)
        size = round_up(int(loguniform(draw(seed, T_S_SIZE, r, 0), lo, hi)), page)
        size = min(size, arena_bytes // page * page)
        src_off = page * below(draw(seed, T_S_SRC, r, 0), (arena_bytes - size) // page + 1)
        q = ServeReq(r, t, ty, size, src_off)
        pages = size // page
        if ty == REQ_CKPT:
            f = frac_lo + (frac_hi - frac_lo) * unit(draw(seed, T_S_FRAC, r, 0))
            target = max(1, int(f * pages))
            nr = min(target, 16 + below(draw(seed, T_S_RUNS, r, 0), 240))
            rng = np.random.Generator(np.random.PCG64(draw(seed, T_S_RUNS, r, 1)))
            st = np.sort(rng.choice(pages, size=nr, replace=False)).astype(np.int64)
            nxt = np.append(st[1:], pages)
            ln = np.minimum(target // nr, nxt - st).astype(np.int64)
            keep = ln > 0
            q.runs = (st[keep], ln[keep])
        elif ty == REQ_BURST:
            k = 1 + below(draw(seed, T_S_PARTS, r, 0), 8)
            q.parts = sorted(permutation(seed + r, T_S_PARTS, 8)[:k])
            q.n_rec = burst_records
        out.append(q)
        r += 1


def burst_world(q: ServeReq, page: int) -> World:
    """The burst's region as a pool of 8 equal buffers (whole pages)."""
    pages = q.size // page
    per = max(1, pages // 8)
    offs = [i * per * page for i in range(8)]
    sizes = [per * page] * 7 + [(pages - 7 * per) * page]
    keep = [i for i in range(8) if sizes[i] > 0]
    return World(q.r, q.size, page, np.asarray([offs[i] for i in keep], np.uint64),
                 np.asarray([sizes[i] for i in keep], np.uint64), 0.0, f"burst{q.r}")


def burst_launch(q: ServeReq, w: World) -> Launch:
    named = [(i, 1) for i in q.parts if i < w.n_alloc]
    return launch_custom(w, q.r, named, q.n_rec)
