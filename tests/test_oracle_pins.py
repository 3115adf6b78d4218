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
