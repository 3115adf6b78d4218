"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* generator: published splitmix64 outputs;
* speculation: hand-derived interval sets (tests/golden/spec_cases.json) from
  the rules of Section 4.1 and Section 6;
* validation: exhaustive enumeration over a tiny pool with a set-membership
  brute force; "every out-of-speculation access is flagged" — the flagged
  records are exactly those the generator injected; closed-form special
  cases (a launch naming every buffer flags exactly the free-space accesses;
  a launch naming nothing flags everything); victim lookup = bisection;
* tracking: page size = pool gives one bit, page size = 8 bytes gives the exact
  written-word set; dirty pages lie inside write intervals;
* images: a hand-written snapshot, restore(snapshot) identity;
* copy-on-write (Section 4.2) and restore (Section 6) page sets: every page
  written in the window is copied no later than its first writing launch;
  restore sets are disjoint and cover exactly the touched pages.
"""
import bisect
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
POOL_BASE = 0x7F12_3400_0000


def test_splitmix64_published_outputs():
    # splitmix64 seeded with 0: the first three outputs of the reference generator.
    assert synth.mix(1 * synth.GOLDEN) == 0xE220A8397B1DCDAF
    assert synth.mix(2 * synth.GOLDEN) == 0x6E789E6AA1B965F4
    assert synth.mix(3 * synth.GOLDEN & synth.M64) == 0x06C45D188009454F
    L = synth.host_lib()
    for z in (0, 1, synth.GOLDEN, 12345678901234567):
        assert L.synth_mix_host(z) == synth.mix(z)
    for r, n in ((2**63, 3), (2**64 - 1, 1000), (12345, 7)):
        assert L.synth_below_host(r, n) == (r * n) >> 64


def _golden_cases():
    with open(os.path.join(GOLDEN, "spec_cases.json")) as f:
        return json.load(f)


def _case_structs(case):
    structs = {}
    for pos, vals in case.get("struct", {}).items():
        structs[int(pos)] = b"".join(int(v).to_bytes(8, "little") for v in vals)
    for pos, hx in case.get("struct_raw", {}).items():
        structs[int(pos)] = bytes.fromhex(hx[2:])
    return structs


@pytest.mark.parametrize("idx", range(len(_golden_cases()["cases"])))
def test_spec_golden(idx):
    g = _golden_cases()
    case = g["cases"][idx]
    table = oracle.Table([b for b, _ in g["buffers"]], [n for _, n in g["buffers"]])
    iv = oracle.spec_build(table, [tuple(a) for a in case["args"]], _case_structs(case))
    got = [[int(x["lo"]), int(x["hi"]), int(x["mode"])] for x in iv]
    assert got == case["expect"], case["name"]


# ---------------------------------------------------------------- validation
def _brute_valid(intervals, addr, is_write):
    """Set-membership definition: the 8-byte access is allowed iff its start is one
    of the 8-aligned starts enumerated inside an interval holding the mode."""
    allowed, inside = set(), set()
    for lo, hi, mode in intervals:
        starts = set(range(lo + (-lo % 8), hi - 7, 8))
        inside |= starts
        if mode & (2 if is_write else 1):
            allowed |= starts
    if addr in allowed:
        return 0
    return 2 if addr in inside else 1


def test_validate_exhaustive_tiny_pool():
    bufs = [(64, 64), (192, 128), (384, 64)]
    table = oracle.Table([b for b, _ in bufs], [n for _, n in bufs])
    addrs = list(range(0, 512, 8))
    rec_all = np.array([a | w for a in addrs for w in (0, 1)], dtype=np.uint64)
    # every assignment of {absent, R, R|W} to the three buffers, plus ranges
    specs = []
    for code in range(27):
        c, parts = code, []
        for b in bufs:
            m = c % 3
            c //= 3
            if m:
                parts.append((b[0], b[0] + b[1], 1 if m == 1 else 3))
        specs.append(parts)
    specs += [[(100, 180, 2)], [(0, 512, 1), (200, 216, 2)], [(8, 12, 3)], [(0, 8, 2), (0, 8, 1)]]
    for parts in specs:
        iv = np.zeros(len(parts), dtype=oracle.INTERVAL_DTYPE)
        for j, (lo, hi, m) in enumerate(parts):
            iv[j] = (lo, hi, m, 0)
        v = oracle.validate(iv, rec_all, table)
        got = {int(x["index"]): int(x["reason"]) for x in v}
        for i, r in enumerate(rec_all.tolist()):
            want = _brute_valid(parts, r & ~7, r & 1)
            assert got.get(i, 0) == want, (parts, r)
        for x in v:  # victim: bisection over the sorted bases
            a = int(x["addr"])
            j = bisect.bisect_right([b for b, _ in bufs], a) - 1
            expect = j if j >= 0 and a < bufs[j][0] + bufs[j][1] else -1
            assert int(x["victim"]) == expect


def _small_world():
    return synth.layout_random(0xC0FFEE, 48, 4096, 4 << 20, 4096, 64 << 10, name="small")


def test_flagged_equals_injected():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    thr = synth.inj_threshold(w.inj_per_mille)
    total_inj = 0
    for L in synth.launches_uniform(w, 30, 20000):
        rec = synth.records_host(hw, L)
        iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
        v = oracle.validate(iv, rec, table, L.k)
        inj = [i for i in range(L.n_records) if synth.draw(w.seed, synth.T_INJ, L.k, i) < thr]
        assert v["index"].tolist() == inj
        assert (v["launch_id"] == L.k).all()
        total_inj += len(inj)
    assert 400 < total_inj < 800  # 0.1 % of 600k accesses


def test_naming_every_buffer_flags_exactly_free_space():
    w = _small_world()
    table = oracle.Table.from_world(w, POOL_BASE)
    args = [(synth.ARG_PTR_MUT, 0, POOL_BASE + int(o), 0) for o in w.alloc_off]
    iv = oracle.spec_build(table, args)
    assert len(iv) == w.n_alloc
    rng = np.random.default_rng(5)
    addrs = (rng.integers(0, w.pool_bytes // 8, 200000, dtype=np.uint64) * 8 + POOL_BASE)
    rec = addrs | rng.integers(0, 2, addrs.shape[0], dtype=np.uint64)
    v = oracle.validate(iv, rec, table)
    off = addrs - np.uint64(POOL_BASE)
    j = np.searchsorted(w.alloc_off, off, side="right").astype(np.int64) - 1
    inside = (j >= 0) & (off < w.alloc_off[np.maximum(j, 0)] + w.alloc_bytes[np.maximum(j, 0)])
    assert v["index"].tolist() == np.flatnonzero(~inside).tolist()
    assert (v["reason"] == 1).all() and (v["victim"] == -1).all()


def test_naming_nothing_flags_everything():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    L = synth.Launch(7, [], [(synth.ARG_SCALAR, 0, 99, 0)], 5000)
    rec = synth.records_host(hw, L)
    iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
    v = oracle.validate(iv, rec, table, 7)
    assert len(iv) == 0 and v["index"].tolist() == list(range(5000))
    assert (v["reason"] == 1).all()


def test_flags_select_reads_and_writes():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    L = synth.launches_uniform(w, 1, 50000, k0=3)[0]
    rec = synth.records_host(hw, L)
    iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
    both = oracle.validate(iv, rec, table, L.k)
    r = oracle.validate(iv, rec, table, L.k, flags=oracle.V_READS)
    wr = oracle.validate(iv, rec, table, L.k, flags=oracle.V_WRITES)
    assert (r["is_write"] == 0).all() and (wr["is_write"] == 1).all()
    assert sorted(r["index"].tolist() + wr["index"].tolist()) == both["index"].tolist()


def test_mode_violations_are_injected_writes_to_read_only_buffers():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    for L in synth.launches_uniform(w, 10, 20000, k0=40):
        rec = synth.records_host(hw, L)
        iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
        v = oracle.validate(iv, rec, table, L.k)
        named_ro = {i for i, m in L.named if not m}
        for x in v:
            if x["reason"] == 2:
                assert x["is_write"] == 1 and int(x["victim"]) in named_ro


# ------------------------------------------------------------------ tracking
def test_track_page_equal_pool_is_any_valid_write():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    for L in synth.launches_uniform(w, 6, 3000, k0=100):
        rec = synth.records_host(hw, L)
        iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
        d = np.zeros(1, np.uint8)
        vv = np.zeros(1, np.uint8)
        oracle.track(iv, rec, table, POOL_BASE, w.pool_bytes, 1, d, vv)
        flagged = set(oracle.validate(iv, rec, table, L.k)["index"].tolist())
        any_valid_write = any((int(r) & 1) and i not in flagged for i, r in enumerate(rec))
        assert bool(d[0]) == any_valid_write


def test_track_page_8_bytes_is_exact_written_word_set():
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    table = oracle.Table.from_world(w, POOL_BASE)
    npg = w.pool_bytes // 8
    for L in synth.launches_uniform(w, 4, 20000, k0=200):
        rec = synth.records_host(hw, L)
        iv = oracle.spec_build(table, L.arg_values(POOL_BASE))
        d = np.zeros(npg, np.uint8)
        vv = np.zeros(npg, np.uint8)
        oracle.track(iv, rec, table, POOL_BASE, 8, npg, d, vv)
        bad = oracle.validate(iv, rec, table, L.k)
        flagged = set(bad["index"].tolist())
        words = {(int(r) - POOL_BASE) >> 3 for i, r in enumerate(rec)
                 if (int(r) & 1) and i not in flagged}
        assert set(np.flatnonzero(d).tolist()) == words
        vic = {(int(x["addr"]) - POOL_BASE) >> 3 for x in bad
               if x["is_write"] and x["victim"] >= 0}
        assert set(np.flatnonzero(vv).tolist()) == vic
        wp = np.zeros(npg, np.uint8)
        oracle.write_interval_pages(iv, POOL_BASE, 8, npg, wp)
        assert not (d & (1 - wp)).any()  # dirty words lie inside write intervals


# -------------------------------------------------------------------- images
def test_snapshot_hand_example():
    pool = np.arange(64, dtype=np.uint8)
    table = oracle.Table([1000 + 16, 1000 + 40], [8, 16])
    img = oracle.snapshot(pool, 1000, table)
    assert img.tolist() == list(range(16, 24)) + list(range(40, 56))
    pool2 = np.zeros(64, np.uint8)
    oracle.restore(pool2, 1000, table, img)
    assert pool2[16:24].tolist() == list(range(16, 24)) and pool2[40:56].tolist() == list(range(40, 56))
    assert pool2[:16].sum() == 0 and pool2[24:40].sum() == 0 and pool2[56:].sum() == 0


def test_gather_hand_example():
    src = np.arange(100, dtype=np.uint8)
    dst = np.zeros(20, np.uint8)
    oracle.gather(src, dst, [10, 50], [0, 5], [5, 3])
    assert dst[:8].tolist() == [10, 11, 12, 13, 14, 50, 51, 52]


def _stream_setup(n_launch=25, n_rec=20000):
    w = _small_world()
    hw = synth.HostWorld(w, POOL_BASE)
    pool = synth.content_host(w.seed, 0, w.pool_bytes)
    launches = synth.launches_uniform(w, n_launch, n_rec)
    rec_cache = {}

    def records_fn(L):
        if L.k not in rec_cache:
            rec_cache[L.k] = synth.records_host(hw, L)
        return rec_cache[L.k]

    def apply_fn(p, L, rec):
        synth.apply_writes_host(p, POOL_BASE, w.seed, L.k, rec)

    return w, pool, launches, records_fn, apply_fn


def test_cow_sets_copy_every_page_before_its_first_write():
    w, pool, launches, records_fn, apply_fn = _stream_setup()
    t1, t2 = 5, 20
    res = oracle.run_stream(w, launches, POOL_BASE, records_fn, apply_fn, pool,
                            snap_before=(t1, t2), cow_window=(t1, t2), window=(t1, t2))
    copied_by = {}
    for j, s in enumerate(res.cow_sets):
        for p in s.tolist():
            assert p not in copied_by  # each page is copied once
            copied_by[p] = t1 + j
    table = oracle.Table.from_world(w, POOL_BASE)
    inbuf = np.zeros(w.n_pages, np.uint8)
    for o, b in zip(w.alloc_off, w.alloc_bytes):
        inbuf[int(o) // w.page_bytes:(int(o) + int(b)) // w.page_bytes] = 1
    for j in range(t1, t2):
        L = launches[j]
        rec = records_fn(L)
        for r in rec.tolist():
            if not r & 1:
                continue
            p = ((r & ~7) - POOL_BASE) // w.page_bytes
            if inbuf[p]:
                assert copied_by.get(p, 1 << 30) <= j, (p, j)
    # the written image bytes of copied pages equal the t1 snapshot by construction
    assert set(copied_by) <= set(np.flatnonzero(inbuf).tolist())
    d = res.dirty | res.victim
    assert set(np.flatnonzero(d).tolist()) <= set(copied_by)
    assert not np.array_equal(res.snapshots[t1], res.snapshots[t2])
    del table


def test_restore_sets_disjoint_and_cover_touched_pages():
    w, pool, launches, records_fn, _ = _stream_setup(10, 5000)
    table = oracle.Table.from_world(w, POOL_BASE)
    present = np.zeros(w.n_pages, np.uint8)
    union = np.zeros(w.n_pages, np.uint8)
    for L in launches:
        t = np.zeros(w.n_pages, np.uint8)
        oracle.touched_pages(records_fn(L), table, POOL_BASE, w.page_bytes, w.n_pages, t)
        f = t & (1 - present)
        assert not (f & present).any()
        present |= f
        union |= t
    assert np.array_equal(present, union)


# ------------------------------------------- page sets: brute-force pins
# A tiny pool [0, 512) with buffers [64, 128), [192, 320), [384, 448) and gaps
# between them; page sizes from one word to the whole pool.
TINY_BUFS = [(64, 64), (192, 128), (384, 64)]
TINY_POOL = 512
TINY_PAGES = (8, 16, 32, 64, 128, 512)


def _allocated_bytes(bufs):
    s = set()
    for b, n in bufs:
        s |= set(range(b, b + n))
    return s


def test_touched_pages_brute_force_tiny_pool():
    """Section 6: a launch touches the pages holding its accesses that lie
    inside allocated buffers.  Every 8-aligned address (and a few outside the
    pool) x read/write x page size, alone and all together, against a set
    built by enumerating the buffers' bytes."""
    table = oracle.Table([b for b, _ in TINY_BUFS], [n for _, n in TINY_BUFS])
    alloc = _allocated_bytes(TINY_BUFS)
    addrs = list(range(0, TINY_POOL, 8)) + [TINY_POOL, TINY_POOL + 64]
    for page in TINY_PAGES:
        npg = TINY_POOL // page
        for a in addrs:
            for w in (0, 1):
                got = np.zeros(npg, np.uint8)
                oracle.touched_pages(np.array([a | w], np.uint64), table, 0, page, npg, got)
                want = {a // page} if a in alloc else set()
                assert set(np.flatnonzero(got).tolist()) == want, (page, a, w)
        rec = np.array([a | (i & 1) for i, a in enumerate(addrs)], np.uint64)
        got = np.zeros(npg, np.uint8)
        oracle.touched_pages(rec, table, 0, page, npg, got)
        want = {a // page for a in addrs if a in alloc}
        assert set(np.flatnonzero(got).tolist()) == want, page
    # a pool that starts above address 0: pages count from its base
    got = np.zeros(8, np.uint8)
    table2 = oracle.Table([1024 + 64], [64])
    oracle.touched_pages(np.array([1024 + 64, 1024 + 120, 1024 + 128, 8], np.uint64), table2,
                         1024, 64, 8, got)
    assert np.flatnonzero(got).tolist() == [1]


def test_write_interval_pages_brute_force():
    """The pages a launch may write (Section 4.2's copy-before-write set):
    the pages overlapping its intervals that hold the W mode, clipped to the
    pool.  Every interval of 8-aligned bounds in a 256-byte pool x mode
    {R, W, R|W} x page size, against an enumeration of the interval's
    bytes; then mixed sets of read and write intervals."""
    pool = 256
    for page in (8, 16, 64, 256):
        npg = pool // page
        for lo in range(0, pool, 8):
            for hi in range(lo + 8, pool + 16, 8):
                for mode in (1, 2, 3):
                    iv = np.zeros(1, dtype=oracle.INTERVAL_DTYPE)
                    iv[0] = (lo, hi, mode, 0)
                    got = np.zeros(npg, np.uint8)
                    oracle.write_interval_pages(iv, 0, page, npg, got)
                    want = {x // page for x in range(lo, min(hi, pool))} if mode & 2 else set()
                    assert set(np.flatnonzero(got).tolist()) == want, (page, lo, hi, mode)
    rng = np.random.default_rng(11)
    for _ in range(200):
        k = int(rng.integers(1, 6))
        parts = []
        for _ in range(k):
            lo = int(rng.integers(0, 60)) * 8
            hi = lo + 8 * int(rng.integers(1, 20))
            parts.append((lo, hi, int(rng.integers(1, 4))))
        iv = np.zeros(k, dtype=oracle.INTERVAL_DTYPE)
        for j, p in enumerate(parts):
            iv[j] = (*p, 0)
        for page in (8, 32, 128):
            npg = 512 // page
            got = np.zeros(npg, np.uint8)
            oracle.write_interval_pages(iv, 0, page, npg, got)
            want = set()
            for lo, hi, m in parts:
                if m & 2:
                    want |= {x // page for x in range(lo, min(hi, 512))}
            assert set(np.flatnonzero(got).tolist()) == want


def test_needed_pages_brute_force():
    """Section 6: touched pages inside buffers, plus with prefetch every page
    of the speculated intervals lying in a buffer; against enumeration."""
    table = oracle.Table([b for b, _ in TINY_BUFS], [n for _, n in TINY_BUFS])
    alloc = _allocated_bytes(TINY_BUFS)
    rec = np.array([8 | 1, 72, 136 | 1, 200, 400 | 1, 456], np.uint64)
    for page in TINY_PAGES:
        npg = TINY_POOL // page
        for args in ([], [(oracle.ARG_PTR_CONST, 0, 200, 0)], [(oracle.ARG_PTR_MUT, 0, 64, 0)],
                     [(oracle.ARG_RANGE, oracle.R, 120, 96)],
                     [(oracle.ARG_PTR_CONST, 0, 400, 0), (oracle.ARG_RANGE, oracle.W, 0, 512)]):
            touched = {int(a) // page for a in (rec & ~np.uint64(7)).tolist() if int(a) in alloc}
            spec_bytes = set()
            for x in oracle.spec_build(table, args):
                spec_bytes |= set(range(int(x["lo"]), int(x["hi"])))
            pre = {x // page for x in spec_bytes & alloc}
            for prefetch, want in ((False, touched), (True, touched | pre)):
                got = oracle.needed_pages(table, args, rec, 0, page, npg, prefetch)
                assert set(np.flatnonzero(got).tolist()) == want, (page, args, prefetch)


def test_buffer_pages_brute_force():
    table = oracle.Table([b for b, _ in TINY_BUFS], [n for _, n in TINY_BUFS])
    alloc = _allocated_bytes(TINY_BUFS)
    for page in TINY_PAGES:
        npg = TINY_POOL // page
        got = oracle.buffer_pages(table, 0, page, npg)
        want = {x // page for x in alloc}
        assert set(np.flatnonzero(got).tolist()) == want, page


# --------------------------------- copy-on-write sets: a hand-built stream
# Pool of 16 pages of 64 bytes at HAND_BASE: buffer A = pages 0-2, gap page 3,
# B = pages 4-7, gap pages 8-9, C = pages 10-11, free pages 12-15.
HAND_BASE = 0x10000
HAND_PAGE = 64


def _hand_world():
    return synth.World(seed=7, pool_bytes=16 * HAND_PAGE, page_bytes=HAND_PAGE,
                       alloc_off=np.array([0, 4 * HAND_PAGE, 10 * HAND_PAGE], np.uint64),
                       alloc_bytes=np.array([3 * HAND_PAGE, 4 * HAND_PAGE, 2 * HAND_PAGE],
                                            np.uint64), name="hand")


def _hand_stream():
    """Three launches (buffer index, mutable?) and their accesses (page, offset, write?)."""
    A, B, C = 0, 1, 2
    named = {0: [(A, 1), (B, 0)], 1: [(B, 1), (C, 0)], 2: [(A, 1), (C, 1)]}
    acc = {
        # valid write A/p1; write to read-only B/p5 (victim); write to gap p3;
        # read of unnamed C/p10 (a violation: its record names buffer C, but a
    # read marks no victim page)
        0: [(1, 8, 1), (5, 16, 1), (3, 0, 1), (10, 24, 0)],
        # valid write B/p6; write to read-only C/p11 (victim); write to
        # unnamed A/p0 (victim, copied already)
        1: [(6, 0, 1), (11, 8, 1), (0, 32, 1)],
        # valid write C/p10; write to the free p13; write to unnamed B/p7
        2: [(10, 40, 1), (13, 0, 1), (7, 56, 1)],
    }
    w = _hand_world()
    launches = [synth.launch_custom(w, k, named[k], len(acc[k])) for k in range(3)]
    recs = {k: np.array([(HAND_BASE + p * HAND_PAGE + o) | wr for p, o, wr in acc[k]], np.uint64)
            for k in range(3)}
    return w, launches, recs


def _hand_apply(pool, L, rec):
    """The hand stream's application: a write stores 8 bytes of value k + 1."""
    for r in rec.tolist():
        if r & 1:
            off = (r & ~7) - HAND_BASE
            pool[off:off + 8] = L.k + 1


def test_cow_sets_hand_built_three_launches():
    """Section 4.2 with the background copy paused: before launch k, copy the
    pages of its write intervals and the victim pages of its violating writes
    that no earlier launch of the window copied.  Sets worked out by hand:
    launch 0 writes A (pages 0-2) and hits read-only B on page 5; launch 1
    writes B (4-7) and hits C on 11 and A on 0; launch 2 writes A and C
    (10-11) and hits B on 7."""
    w, launches, recs = _hand_stream()
    pool = np.zeros(w.pool_bytes, np.uint8)
    res = oracle.run_stream(w, launches, HAND_BASE, lambda L: recs[L.k], _hand_apply, pool,
                            snap_before=(0, 3), window=(0, 3), cow_window=(0, 3))
    assert [s.tolist() for s in res.cow_sets] == [[0, 1, 2, 5], [4, 6, 7, 11], [10]]
    # Section 4.3 on the same window: dirty = valid-write pages, victim =
    # pages of failing writes inside buffers (gap and free pages excluded)
    assert np.flatnonzero(res.dirty).tolist() == [1, 6, 10]
    assert np.flatnonzero(res.victim).tolist() == [0, 5, 7, 11]
    # the violations, in order, with their reasons and victims
    v = [[(int(x["index"]), int(x["reason"]), int(x["victim"])) for x in vk]
         for vk in res.violations]
    assert v == [[(1, 2, 1), (2, 1, -1), (3, 1, 2)], [(1, 2, 2), (2, 1, 0)],
                 [(1, 1, -1), (2, 1, 1)]]
    # images: t1 all zero; t2 holds each write's value (gaps excluded)
    assert not res.snapshots[0].any()
    img = res.snapshots[3].reshape(-1, HAND_PAGE)  # image pages: A 0-2, B 4-7, C 10-11
    want = np.zeros_like(img)
    want[1, 8:16] = 1    # A p1 (image page 1) by launch 0
    want[0, 32:40] = 2   # A p0 (image page 0) by launch 1
    want[4, 16:24] = 1   # B p5 (image page 4) by launch 0
    want[5, 0:8] = 2     # B p6 (image page 5) by launch 1
    want[6, 56:64] = 3   # B p7 (image page 6) by launch 2
    want[7, 40:48] = 3   # C p10 (image page 7) by launch 2
    want[8, 8:16] = 2    # C p11 (image page 8) by launch 1
    assert np.array_equal(img, want)


def test_precopy_rounds_hand_built():
    """Plain pre-copy rounds (Sections 4.3 and 7): a round copies and unmarks
    everything marked so far.  Five launches' dirty pages by hand; rounds
    before launches 2 and 4; page 5 lies outside every buffer."""
    n = 6
    inbuf = np.array([1, 1, 1, 1, 1, 0], np.uint8)

    def d(*p):
        a = np.zeros(n, np.uint8)
        a[list(p)] = 1
        return a

    per = [d(0, 1), d(1, 5), d(2), d(0), d(3)]
    left, copied = oracle.precopy_rounds(per, [2, 4], inbuf)
    # round at 2 copies {0, 1} (5 is no image page); round at 4 copies {2, 0}
    assert copied == 4 and np.flatnonzero(left).tolist() == [3]
    left, copied = oracle.precopy_rounds(per, [], inbuf)
    assert copied == 0 and np.flatnonzero(left).tolist() == [0, 1, 2, 3, 5]
    left, copied = oracle.precopy_rounds(per, [0], inbuf)  # nothing marked yet
    assert copied == 0


def test_final_rounds_hand_built():
    """Final-page rounds: dirty {0, 1, 2, 6}, victim {3, 4, 5} with their last
    failing writes from launches 0, 3 and 1; launches 2 and 3 may write pages
    1 and 4; page 6 lies outside every buffer.  Worked out by hand: the round
    before launch 2 takes {0, 2, 3, 5, 6} (4 image pages) and leaves dirty {1}
    and victim {4}; the round before launch 4 takes both."""
    n = 8
    dirty = np.zeros(n, np.uint8)
    dirty[[0, 1, 2, 6]] = 1
    victim = np.zeros(n, np.uint8)
    victim[[3, 4, 5]] = 1
    last = np.full(n, -1, np.int64)
    last[3], last[4], last[5] = 0, 3, 1
    inbuf = np.array([1, 1, 1, 1, 1, 1, 0, 1], np.uint8)
    up = {2: [1, 4], 4: []}

    def upcoming(r):
        m = np.zeros(n, np.uint8)
        m[up[r]] = 1
        return m

    dl, vl, copied = oracle.final_rounds(dirty, victim, last, [2], upcoming, inbuf)
    assert (np.flatnonzero(dl).tolist(), np.flatnonzero(vl).tolist(), copied) == ([1], [4], 4)
    dl, vl, copied = oracle.final_rounds(dirty, victim, last, [2, 4], upcoming, inbuf)
    assert (dl.any(), vl.any(), copied) == (False, False, 6)
    assert oracle.recopy_pages(dirty, victim, inbuf) == 6


def test_final_rounds_give_the_snapshot_at_t2():
    """The invariant that makes a final-page round safe (Section 4.3): an image
    copied once at t1, overwritten by each round's pages as the pool stands
    at the round, and by the pages left marked at t2, equals the snapshot at
    t2.  Checked on seeded streams where later launches keep writing the
    pages of earlier ones, with rounds at several places."""
    w, pool0, launches, records_fn, apply_fn = _stream_setup(20, 4000)
    table = oracle.Table.from_world(w, POOL_BASE)
    npg, page = w.n_pages, w.page_bytes
    n = len(launches)
    dirty, victim, last = oracle.track_launches(
        table, n, lambda j: (launches[j].arg_values(POOL_BASE), records_fn(launches[j])),
        POOL_BASE, page, npg, threads=4)
    inbuf = oracle.buffer_pages(table, POOL_BASE, page, npg).astype(bool)

    def upcoming(r):
        return oracle.write_pages(table, [L.arg_values(POOL_BASE) for L in launches[r:]],
                                  POOL_BASE, page, npg)

    for rounds in ([5], [3, 9, 15], [1, 2, 19], [10, 20]):
        pool = pool0.copy()
        image = pool.copy()  # every page copied at t1 (the background copy)
        d, v = dirty.astype(bool), victim.astype(bool)
        copied = 0
        for j in range(n + 1):
            if j in rounds:
                fin_v = v & (last >= 0) & (last < j)
                listed = (d | fin_v) & ~upcoming(j).astype(bool)
                for p in np.flatnonzero(listed & inbuf).tolist():
                    image[p * page:(p + 1) * page] = pool[p * page:(p + 1) * page]
                copied += int((listed & inbuf).sum())
                d &= ~listed
                v &= ~(fin_v & ~upcoming(j).astype(bool))
            if j < n:
                apply_fn(pool, launches[j], records_fn(launches[j]))
        for p in np.flatnonzero((d | v) & inbuf).tolist():  # the recopy at t2
            image[p * page:(p + 1) * page] = pool[p * page:(p + 1) * page]
        assert np.array_equal(oracle.snapshot(image, POOL_BASE, table),
                              oracle.snapshot(pool, POOL_BASE, table)), rounds
        dl, vl, c = oracle.final_rounds(dirty, victim, last, rounds, upcoming, inbuf)
        assert np.array_equal(dl, d) and np.array_equal(vl, v) and c == copied
    # rounds that take nothing: every marked page is still to be written
    dl, vl, c = oracle.final_rounds(dirty, victim, last, [0], lambda r: np.ones(npg, np.uint8),
                                    inbuf)
    assert c == 0 and np.array_equal(dl, dirty.astype(bool))


# ------------------------------------------------------ page fingerprints
def test_page_hash_sees_every_byte_and_place():
    """The full-size comparisons rest on the fingerprint changing with any
    byte of the page, with the order of its words and with the page index."""
    rng = np.random.default_rng(3)
    page = rng.integers(0, 256, 256, dtype=np.uint8)
    h0 = oracle.page_hash(page, 5)
    seen = {h0}
    for i in range(page.size):
        for delta in (1, 128):
            q = page.copy()
            q[i] ^= delta
            h = oracle.page_hash(q, 5)
            assert h != h0
            seen.add(h)
    assert len(seen) == 2 * page.size + 1
    sw = page.copy().view(np.uint64)
    sw[[0, 1]] = sw[[1, 0]]
    assert oracle.page_hash(sw.view(np.uint8), 5) != h0
    assert oracle.page_hash(page, 6) != h0
    assert oracle.page_hash(np.zeros(64, np.uint8), 0) != oracle.page_hash(np.zeros(64, np.uint8), 1)


def test_image_hashes_match_the_snapshot():
    """Fingerprints taken straight from the pool equal those of the snapshot
    (whose layout is pinned by the hand example above), and chunked hashing
    equals hashing in one piece."""
    w = _small_world()
    pool = synth.content_host(w.seed, 0, w.pool_bytes)
    table = oracle.Table.from_world(w, POOL_BASE)
    img = oracle.snapshot(pool, POOL_BASE, table)
    want = oracle.hash_pages(img, w.page_bytes)
    for threads in (1, 3):
        got = oracle.image_hashes_from_pool(pool, POOL_BASE, table, w.page_bytes, threads)
        assert np.array_equal(got, want)
    for chunk in (w.page_bytes, 5 * w.page_bytes, img.nbytes):
        got = oracle.hash_chunks(lambda o, n: img[o:o + n], img.nbytes, w.page_bytes, chunk, 3)
        assert np.array_equal(got, want)
    for i in (0, 7, want.size - 1):
        assert int(want[i]) == oracle.page_hash(img[i * w.page_bytes:(i + 1) * w.page_bytes], i)


def test_apply_stream_and_validate_launches_match_run_stream():
    """The threaded full-size helpers compose the per-launch definitions as
    run_stream does."""
    w, pool0, launches, records_fn, apply_fn = _stream_setup(12, 3000)
    table = oracle.Table.from_world(w, POOL_BASE)
    res = oracle.run_stream(w, launches, POOL_BASE, records_fn, apply_fn, pool0.copy(),
                            snap_before=(len(launches),))
    pool = pool0.copy()
    oracle.apply_stream(pool, launches, records_fn, apply_fn, threads=3, ahead=4)
    assert np.array_equal(oracle.snapshot(pool, POOL_BASE, table), res.snapshots[len(launches)])
    vl = oracle.validate_launches(table, POOL_BASE, launches, records_fn, threads=3)
    assert all(np.array_equal(a, b) for a, b in zip(vl, res.violations))


def test_run_stream_hashed_matches_run_stream():
    """The full-size replay composes the same per-launch definitions as
    run_stream, its fingerprints are those of run_stream's snapshots, and its
    last-victim positions are those of launch-by-launch tracking."""
    w, pool0, launches, records_fn, apply_fn = _stream_setup(15, 3000)
    table = oracle.Table.from_world(w, POOL_BASE)
    res = oracle.run_stream(w, launches, POOL_BASE, records_fn, apply_fn, pool0.copy(),
                            snap_before=(0, 6, 15), window=(3, 12))
    h = oracle.run_stream_hashed(w, launches, POOL_BASE, records_fn, apply_fn, pool0.copy(),
                                 hash_before=(0, 6, 15), window=(3, 12), threads=3, ahead=4)
    assert all(np.array_equal(a, b) for a, b in zip(h.violations, res.violations))
    assert np.array_equal(h.dirty, res.dirty) and np.array_equal(h.victim, res.victim)
    for j in (0, 6, 15):
        assert np.array_equal(h.hashes[j], oracle.hash_pages(res.snapshots[j], w.page_bytes))
    _, _, last = oracle.track_launches(
        table, 9, lambda i: (launches[3 + i].arg_values(POOL_BASE), records_fn(launches[3 + i])),
        POOL_BASE, w.page_bytes, w.n_pages)
    assert np.array_equal(h.last, np.where(last >= 0, last + 3, -1))


def test_reader_and_gather_hashes_match_their_definitions():
    """Chunked fingerprints of a pool read piece by piece equal those of its
    snapshot; fingerprints of a gather equal those of orc_gather's output."""
    w = _small_world()
    pool = synth.content_host(w.seed, 0, w.pool_bytes)
    table = oracle.Table.from_world(w, POOL_BASE)
    want = oracle.hash_pages(oracle.snapshot(pool, POOL_BASE, table), w.page_bytes)
    for chunk in (w.page_bytes, 3 * w.page_bytes, 1 << 30):
        got = oracle.image_hashes_from_reader(lambda o, n: pool[o:o + n], POOL_BASE, table,
                                              w.page_bytes, chunk, threads=3)
        assert np.array_equal(got, want)
    page = 4096
    src_off = np.array([0, 5, 9, 20], np.uint64) * page
    dst_off = np.array([0, 2, 3, 6], np.uint64) * page
    ln = np.array([2, 1, 3, 1], np.uint64) * page
    dst = np.zeros(8 * page, np.uint8)
    oracle.gather(pool, dst, src_off, dst_off, ln)
    got = oracle.gather_hashes(lambda o, n: pool[o:o + n], src_off, dst_off, ln, page, 7,
                               threads=2, piece_bytes=page)
    assert np.array_equal(got, oracle.hash_pages(dst[:7 * page], page))
