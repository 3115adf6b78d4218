"""GPU parity: speculation (Section 4.1), validation (Section 4.1) and write-set
tracking (Section 4.3) through the C ABI, element by element against the
oracle on the same seeded inputs.  Integer work: the bar is bit-exact."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_harness import Env, bits_to_pages, u64

pytestmark = pytest.mark.gpu
FLAGS = 1 | 2  # reads and writes


@pytest.fixture(scope="module")
def env1():
    e = Env(synth.config1_world())
    yield e
    e.close()


def test_device_generator_matches_host(env1):
    w = env1.world
    launches = synth.config1_launches(w, 4, 300001)
    dev = u64(env1.records(launches, 300001))
    for j, L in enumerate(launches):
        assert np.array_equal(dev[j * 300001:(j + 1) * 300001], synth.records_host(env1.hw, L))
    assert np.array_equal(env1.pool_host(), synth.content_host(w.seed, 0, w.pool_bytes))


def test_spec_register_golden():
    from paper_2405_12079_amd import phos
    with open(os.path.join(os.path.dirname(__file__), "golden", "spec_cases.json")) as f:
        g = json.load(f)
    T = __import__("torch")
    back = T.empty(1 << 20, dtype=T.uint8, device="cuda")
    base = (back.data_ptr() + 4095) // 4096 * 4096
    # the golden table uses small absolute addresses: shift everything by `base`
    ctx = phos.phos_create(0, base, 64 << 10, 4096)
    try:
        phos.phos_buffers_register(ctx, [(base + b, n) for b, n in g["buffers"]])
        for case in g["cases"]:
            structs = {}
            for pos, vals in case.get("struct", {}).items():
                structs[int(pos)] = b"".join((base + int(v)).to_bytes(8, "little") if int(v) >= 4096
                                             else int(v).to_bytes(8, "little") for v in vals)
            for pos, hx in case.get("struct_raw", {}).items():
                raw = bytearray(bytes.fromhex(hx[2:]))
                raw[:8] = (int.from_bytes(raw[:8], "little") + base).to_bytes(8, "little")
                structs[int(pos)] = bytes(raw)
            args = []
            for kind, mode, value, nb in case["args"]:
                if kind in (1, 2, 4) and value >= 4096:
                    value += base
                args.append((kind, mode, value, nb))
            s = phos.phos_spec_register(ctx, 0, args, structs)
            iv = phos.phos_spec_intervals(ctx, s)
            got = [[int(x["lo"]) - base, int(x["hi"]) - base, int(x["mode"])] for x in iv]
            assert got == case["expect"], case["name"]
            phos.phos_spec_release(ctx, s)
    finally:
        phos.phos_destroy(ctx)


def test_spec_register_matches_oracle(env1):
    from paper_2405_12079_amd import phos
    for L in synth.config1_launches(env1.world, 100, 1):
        s = env1.spec(L)
        got = phos.phos_spec_intervals(env1.ctx, s)
        want = oracle.spec_build(env1.table, L.arg_values(env1.base))
        assert np.array_equal(got, want), L.k
        phos.phos_spec_release(env1.ctx, s)


def _validate_one(env, L, rec_t, n, flags=FLAGS, cap=None, stream=None):
    from paper_2405_12079_amd import phos
    cap = n if cap is None else cap
    out, cnt = env.violations_buffers(cap)
    s = env.spec(L)
    phos.phos_validate(env.ctx, s, rec_t, n, flags, out, cap, cnt, stream or env.app)
    (stream or env.app).synchronize()
    phos.phos_spec_release(env.ctx, s)
    return Env.read_violations(out, cnt, cap)


def test_validate_config1_all_launches(env1):
    """Full plain-tiny workload: 100 launches x 1M records, violations bit-exact."""
    w = env1.world
    launches = synth.config1_launches(w)
    total = 0
    for g in range(0, 100, 20):
        grp = launches[g:g + 20]
        recs = env1.records(grp, 1_000_000)
        for j, L in enumerate(grp):
            r = recs[j * 1_000_000:(j + 1) * 1_000_000]
            n, got = _validate_one(env1, L, r, 1_000_000)
            iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
            want = oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k)
            assert n == len(want), (L.k, n, len(want))
            assert np.array_equal(got, want), L.k
            total += n
        del recs
    assert 90_000 < total < 110_000  # 0.1 % of 1e8


@pytest.mark.parametrize("scan_path", [False, True])
def test_validate_batch_matches_per_launch(env1, scan_path, monkeypatch):
    """Batched validation, ordered by the one-workgroup finish or (forced) by the
    segment scan + scatter kernels."""
    from paper_2405_12079_amd import phos
    if scan_path:
        monkeypatch.setenv("PHOS_VFINISH_MAX_TILES", "0")
        env1 = Env(env1.world)
    w = env1.world
    launches = synth.config1_launches(w, 40, 250_000)
    recs = env1.records(launches, 250_000)
    specs = [env1.spec(L) for L in launches]
    cap = 40 * 250_000
    out, cnt = env1.violations_buffers(cap)
    ptrs = [recs.data_ptr() + j * 250_000 * 8 for j in range(40)]
    phos.phos_validate_batch(env1.ctx, specs, ptrs, [250_000] * 40, FLAGS, out, cap, cnt, env1.app)
    env1.app.synchronize()
    n, got = Env.read_violations(out, cnt, cap)
    want = []
    for L in launches:
        iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
        want.append(oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k))
    want = np.concatenate(want)
    assert n == len(want) and np.array_equal(got, want)
    # a second call with identical descriptors reuses the device copy
    out.zero_()
    phos.phos_validate_batch(env1.ctx, specs, ptrs, [250_000] * 40, FLAGS, out, cap, cnt, env1.app)
    env1.app.synchronize()
    n2, got2 = Env.read_violations(out, cnt, cap)
    assert n2 == n and np.array_equal(got2, want)
    for s in specs:
        phos.phos_spec_release(env1.ctx, s)
    if scan_path:
        env1.close()


@pytest.mark.parametrize("n", [0, 1, 2, 3, 127, 2047, 2048, 2049, 8193, 70001])
@pytest.mark.parametrize("shift", [0, 1])
def test_validate_ragged_and_misaligned(env1, n, shift):
    """Ragged tails and 8-byte (not 16-byte) aligned record arrays."""
    L = synth.config1_launches(env1.world, 1, n + 1)[0]
    recs = env1.records([L], n + 1)
    r = recs[shift:shift + n] if n else recs[:0]
    n_got, got = _validate_one(env1, L, r.data_ptr() if n else 0, n, cap=max(n, 1))
    host = synth.records_host(env1.hw, L)[shift:shift + n]
    iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
    want = oracle.validate(iv, host, env1.table, L.k)
    assert n_got == len(want) and np.array_equal(got, want)


def test_validate_many_intervals_struct_path(env1):
    """A struct argument naming 20 buffers -> more than 8 intervals (general path)."""
    w = env1.world
    idx = list(range(0, 200, 10))
    st = b"".join((env1.base + int(w.alloc_off[i]) + 8).to_bytes(8, "little") for i in idx)
    # the access stream touches 8 of the 20 named buffers (the generator's limit)
    L = synth.Launch(500, [(i, 1) for i in idx[::3]], [(synth.ARG_STRUCT, 0, 0, len(st))], 200_000)
    from paper_2405_12079_amd import phos
    recs = env1.records([L], 200_000)
    s = phos.phos_spec_register(env1.ctx, L.k, L.arg_values(env1.base), {0: st})
    out, cnt = env1.violations_buffers(200_000)
    phos.phos_validate(env1.ctx, s, recs, 200_000, FLAGS, out, 200_000, cnt, env1.app)
    env1.app.synchronize()
    n, got = Env.read_violations(out, cnt, 200_000)
    iv = oracle.spec_build(env1.table, L.arg_values(env1.base), {0: st})
    assert len(iv) == 20
    assert np.array_equal(phos.phos_spec_intervals(env1.ctx, s), iv)
    want = oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k)
    assert n == len(want) and np.array_equal(got, want)


def test_validate_naming_nothing_overflows_lds_lists(env1):
    """Every record violates: per-wave lists overflow and the ordered rescan runs."""
    L = synth.Launch(600, [], [(synth.ARG_SCALAR, 0, 5, 0)], 100_000)
    recs = env1.records([L], 100_000)
    n, got = _validate_one(env1, L, recs, 100_000)
    iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
    want = oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k)
    assert n == 100_000 and np.array_equal(got, want)


def test_validate_reports_true_count_beyond_cap(env1):
    """More violations than cap (Section 4.1 reports into a buffer of fixed
    size): the true count comes back, phos_stream_status reports
    PHOS_E_OVERFLOW once, and PHOS_V_SYNC reports it from the call itself;
    a call within its cap reports nothing."""
    from paper_2405_12079_amd import phos
    L = synth.config1_launches(env1.world, 1, 1_000_000)[0]
    recs = env1.records([L], 1_000_000)
    iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
    want = oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k)
    phos.phos_stream_status(env1.ctx, env1.app)  # nothing pending
    n, _ = _validate_one(env1, L, recs, 1_000_000, cap=10)
    assert n == len(want) > 10
    with pytest.raises(phos.PhosError) as e:
        phos.phos_stream_status(env1.ctx, env1.app)
    assert e.value.status == phos.E_OVERFLOW
    phos.phos_stream_status(env1.ctx, env1.app)  # reported once
    out, cnt = env1.violations_buffers(len(want))
    s = env1.spec(L)
    try:
        with pytest.raises(phos.PhosError) as e:
            phos.phos_validate(env1.ctx, s, recs, 1_000_000, FLAGS | phos.V_SYNC, out, 10, cnt,
                               env1.app)
        assert e.value.status == phos.E_OVERFLOW and int(cnt.item()) == len(want)
        phos.phos_validate(env1.ctx, s, recs, 1_000_000, FLAGS | phos.V_SYNC, out, len(want),
                           cnt, env1.app)
        n, got = Env.read_violations(out, cnt, len(want))
        assert n == len(want) and np.array_equal(got, want)
        with pytest.raises(phos.PhosError) as e:  # the V_SYNC overflow is also sticky
            phos.phos_stream_status(env1.ctx, env1.app)
        assert e.value.status == phos.E_OVERFLOW
        phos.phos_stream_status(env1.ctx, env1.app)
    finally:
        phos.phos_spec_release(env1.ctx, s)


@pytest.mark.parametrize("flags", [1, 2])
def test_validate_flag_selection(env1, flags):
    L = synth.config1_launches(env1.world, 1, 300_000)[0]
    recs = env1.records([L], 300_000)
    n, got = _validate_one(env1, L, recs, 300_000, flags=flags)
    iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
    want = oracle.validate(iv, synth.records_host(env1.hw, L), env1.table, L.k, flags=flags)
    assert n == len(want) and np.array_equal(got, want)


def test_track_bitmaps_config1_window(env1):
    """Dirty (validated writes) and victim (failing writes in buffers) page bitmaps
    over launches 20..79 of the plain-tiny stream, word for word."""
    from paper_2405_12079_amd import phos
    w = env1.world
    launches = synth.config1_launches(w)[20:80]
    phos.phos_track_reset(env1.ctx, env1.app)
    dirty = np.zeros(w.n_pages, np.uint8)
    vic = np.zeros(w.n_pages, np.uint8)
    for g in range(0, 60, 20):
        grp = launches[g:g + 20]
        recs = env1.records(grp, 1_000_000)
        for j, L in enumerate(grp):
            r = recs[j * 1_000_000:(j + 1) * 1_000_000]
            _validate_one(env1, L, r, 1_000_000, flags=FLAGS | phos.V_TRACK)
            iv = oracle.spec_build(env1.table, L.arg_values(env1.base))
            oracle.track(iv, synth.records_host(env1.hw, L), env1.table, env1.base, w.page_bytes,
                         w.n_pages, dirty, vic)
        del recs
    d = phos.phos_track_read(env1.ctx, 0, w.n_pages)
    v = phos.phos_track_read(env1.ctx, 1, w.n_pages)
    assert np.array_equal(d, oracle.pages_to_bitmap(dirty, w.n_pages))
    assert np.array_equal(v, oracle.pages_to_bitmap(vic, w.n_pages))
    assert dirty.sum() > 0 and vic.sum() > 0
    assert np.array_equal(bits_to_pages(d, w.n_pages), dirty)


def _edge_records(bounds, seed):
    """Records on and around every bound (8-byte slots from 24 bytes below to
    24 bytes above), as reads and as writes, plus random records over the
    same span, shuffled."""
    rng = np.random.default_rng(seed)
    addrs = []
    for b in bounds:
        for d in range(-24, 32, 8):
            addrs.append(((b + d) & ~7) & ((1 << 64) - 1))
    lo, hi = min(bounds) - 4096, max(bounds) + 4096
    addrs += list(rng.integers(lo // 8, hi // 8, 60_000, dtype=np.int64).astype(np.uint64) * 8)
    a = np.array(addrs, dtype=np.uint64)
    rec = np.concatenate([a, a | np.uint64(1)])
    rng.shuffle(rec)
    return rec


@pytest.mark.parametrize("case", ["inside", "past_end"])
def test_validate_range_bounds(env1, case):
    """Section 4.1 ranges with bounds off 8-byte slots.  "inside": every
    interval inside the pool and holding a slot (the 32-bit offset test);
    "past_end": adds ranges of 1, 7 and 8 bytes that hold no slot, one that
    reaches past the pool's end and one beyond it (the 64-bit test).  Violations bit-exact and dirty / victim pages
    equal to the oracle's, on records at and around every bound."""
    from paper_2405_12079_amd import phos
    T = env1.T
    w, base = env1.world, env1.base
    R, W_ = 1, 2
    b0, b1 = int(w.alloc_off[3]), int(w.alloc_off[40])
    # each holds at least one 8-byte slot (the 32-bit test needs that)
    ranges = [(base + b0 + 1003, 1008, R | W_), (base + b0 + 5 * 4096 + 5, 61, W_),
              (base + b1 + 3 * 4096 + 7, 9, R | W_)]
    if case == "past_end":
        # ranges shorter than a slot, or holding none, and two past the pool
        ranges += [(base + b1 + 13, 1, R), (base + b1 + 4096 + 1, 7, W_),
                   (base + b1 + 8192 + 3, 8, R | W_),
                   (base + w.pool_bytes - 100, 300, R | W_), (base + w.pool_bytes + 4096, 64, R | W_)]
    args = [(synth.ARG_RANGE, m, lo, n) for lo, n, m in ranges]
    bounds = [lo for lo, _, _ in ranges] + [lo + n for lo, n, _ in ranges]
    rec_h = _edge_records(bounds, 7 if case == "inside" else 8)
    n = len(rec_h)
    rec_d = T.from_numpy(rec_h.view(np.int64)).cuda()
    phos.phos_track_reset(env1.ctx, env1.app)
    s = phos.phos_spec_register(env1.ctx, 900, args)
    out, cnt = env1.violations_buffers(n)
    phos.phos_validate(env1.ctx, s, rec_d, n, FLAGS | phos.V_TRACK, out, n, cnt, env1.app)
    env1.app.synchronize()
    got_n, got = Env.read_violations(out, cnt, n)
    phos.phos_spec_release(env1.ctx, s)
    iv = oracle.spec_build(env1.table, args)
    want = oracle.validate(iv, rec_h, env1.table, 900)
    assert got_n == len(want) and np.array_equal(got, want)
    assert 0 < len(want) < n
    dirty = np.zeros(w.n_pages, np.uint8)
    vic = np.zeros(w.n_pages, np.uint8)
    oracle.track(iv, rec_h, env1.table, base, w.page_bytes, w.n_pages, dirty, vic)
    assert np.array_equal(phos.phos_track_read(env1.ctx, 0, w.n_pages),
                          oracle.pages_to_bitmap(dirty, w.n_pages))
    assert np.array_equal(phos.phos_track_read(env1.ctx, 1, w.n_pages),
                          oracle.pages_to_bitmap(vic, w.n_pages))
    assert dirty.sum() > 0
