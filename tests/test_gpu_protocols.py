"""GPU parity of the protocols on the plain-tiny workload (64 MiB pool, 256
buffers, 100 launches x 1M accesses, checkpoint opened before launch 20 and
re-quiesced after launch 79):

* Section 4.2 soft copy-on-write: the image equals the snapshot at t1; with
  the background copy deferred, the pages copied before each launch are
  exactly the oracle's copy sets;
* Section 4.3 soft recopy: the image equals the snapshot at t2 and the
  recopied pages are exactly the dirty and victim pages;
* Section 6 concurrent restore: restored pool + launches equals the oracle;
  with the background restore deferred, the present pages after each launch
  are exactly the pages touched so far;
* protocol-order and argument errors.
Byte copies: the bar is bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_harness import Env, bits_to_pages

pytestmark = pytest.mark.gpu
N = 1_000_000
T1, T2 = 20, 80  # begin before launch 20; re-quiesce after launch 79
V = 1 | 2 | 4    # reads, writes, track


@pytest.fixture()
def env():
    e = Env(synth.config1_world())
    yield e
    e.close()


def _buffer_pages(env):
    w = env.world
    return oracle.buffer_pages(env.table, env.base, w.page_bytes, w.n_pages)


class Stream:
    """The plain-tiny launches, generated on the device in groups of 20."""

    def __init__(self, env, launches):
        self.env, self.launches = env, launches
        self.cache = {}

    def records(self, j):
        g = j // 20
        if g not in self.cache:
            self.env.T.cuda.synchronize()  # earlier records may still be read by queued kernels
            self.cache.clear()
            self.cache[g] = self.env.records(self.launches[g * 20:(g + 1) * 20], N)
        return self.cache[g][(j % 20) * N:(j % 20 + 1) * N]


def _run_plain(env, st, host_pool, j0, j1):
    """Launches j0..j1-1 with no checkpoint open (device and host)."""
    for j in range(j0, j1):
        L = st.launches[j]
        r = st.records(j)
        env.mutate(L, r.data_ptr(), N)
        synth.apply_writes_host(host_pool, env.base, env.world.seed, L.k,
                                synth.records_host(env.hw, L))
    env.app.synchronize()


def _validate(env, spec, r, out, cnt, flags=V):
    env.phos.phos_validate(env.ctx, spec, r, N, flags, out, N, cnt, env.app)


@pytest.mark.parametrize("defer", [True, False, "start"])
def test_soft_cow_config1(env, defer):
    """defer: background copy at the end; "start": deferred, then started by
    phos_ckpt_start after the fifth launch of the window."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    res = oracle.run_stream(w, launches[T1:T2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(0,), cow_window=(0, T2 - T1), keep_violations=False)
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND if defer else 0,
                              image, None, env.copy)
    out, cnt = env.violations_buffers(N)
    cum = np.zeros(w.n_pages, np.uint8)
    for j in range(T1, T2):
        L = launches[j]
        s = env.spec(L)
        r = st.records(j)
        _validate(env, s, r, out, cnt)
        phos.phos_ckpt_cow(ck, s, env.app)
        env.mutate(L, r.data_ptr(), N)
        cum[res.cow_sets[j - T1].astype(np.int64)] = 1
        if defer == "start" and j == T1 + 4:
            phos.phos_ckpt_start(ck, env.app)
            with pytest.raises(phos.PhosError) as e:  # started once
                phos.phos_ckpt_start(ck, env.app)
            assert e.value.status == phos.E_STATE
        if defer is True and (j - T1) % 7 == 0:
            env.app.synchronize()
            got = bits_to_pages(phos.phos_ckpt_copied(ck, w.n_pages), w.n_pages)
            assert np.array_equal(got, cum), f"copy set after launch {j}"
        phos.phos_spec_release(env.ctx, s)
    stats = phos.phos_ckpt_end(ck, env.app)
    assert np.array_equal(image.cpu().numpy(), res.snapshots[0]), "CoW image != snapshot at t1"
    n_img_pages = env.image_bytes // w.page_bytes
    assert stats.bg_pages + stats.cow_pages == n_img_pages
    if defer is True:
        assert stats.cow_pages == int(cum.sum())
    assert stats.recopy_pages == 0
    # the application's own writes went to the pool, unaffected by the checkpoint
    assert np.array_equal(env.pool_host(), host)


@pytest.fixture()
def env_w3(monkeypatch):
    """The plain-tiny world with copy-on-write taking victim pages 3 launches
    at a time (read when the context is created)."""
    monkeypatch.setenv("PHOS_COW_VICTIM_WINDOW", "3")
    e = Env(synth.config1_world())
    monkeypatch.delenv("PHOS_COW_VICTIM_WINDOW")
    yield e
    e.close()


def test_soft_cow_chunked_validation_small_window(env_w3):
    """As below ("same"), with victim windows of 3 launches: several windows
    per validation call, the last one cut short at the call's end."""
    _chunked_validation(env_w3, "same", 3, 3)


@pytest.mark.parametrize("vstream", ["same", "other"])
def test_soft_cow_chunked_validation(env, vstream):
    _chunked_validation(env, vstream, 128, 16)


def _chunked_validation(env, vstream, window, first):
    """The training step's order on the plain-tiny workload: each chunk of 20
    launches is validated in one batched call ahead of its launches, on the
    application's stream ("same": a copy-on-write call whose write pages
    earlier calls already asked for, with no new victim pages, is skipped on
    the host) or on a stream of its own that the application waits for chunk
    by chunk, every chunk issued up front ("other": the host cannot order the
    victim pages, so every call looks at them).  With the background copy
    deferred, copy-on-write copies exactly the union of the oracle's copy
    sets ("same": each launch's set before that launch, and nothing beyond the
    sets of the launches its victim window reaches), and the image is the
    snapshot at t1."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    res = oracle.run_stream(w, launches[T1:T2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(0,), cow_window=(0, T2 - T1), keep_violations=False)
    union = np.zeros(w.n_pages, np.uint8)
    for cs in res.cow_sets:
        union[cs.astype(np.int64)] = 1
    T.cuda.synchronize()
    groups = {g: env.records(launches[g * 20:(g + 1) * 20], N) for g in range(T1 // 20, T2 // 20)}
    T.cuda.synchronize()
    specs = {j: env.spec(launches[j]) for j in range(T1, T2)}
    cap = 100_000
    bufs = {g: env.violations_buffers(cap) for g in groups}
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, image, None, env.copy)
    vs = T.cuda.Stream() if vstream == "other" else env.app

    def validate(g):
        js = range(g * 20, (g + 1) * 20)
        out, cnt = bufs[g]
        phos.phos_validate_batch(env.ctx, [specs[j] for j in js],
                                 [groups[g].data_ptr() + (j % 20) * N * 8 for j in js], [N] * 20,
                                 V, out, cap, cnt, vs)

    done = {}
    if vstream == "other":
        vs.wait_stream(env.app)
        for g in groups:
            validate(g)
            done[g] = T.cuda.Event()
            done[g].record(vs)
    so_far = np.zeros(w.n_pages, np.uint8)
    covered = 0
    for j in range(T1, T2):
        g = j // 20
        if j % 20 == 0:
            if vstream == "other":
                env.app.wait_event(done[g])
            else:
                validate(g)
        phos.phos_ckpt_cow(ck, specs[j], env.app)
        if vstream == "same":
            # before each launch its oracle copy set (the pages of its write
            # intervals and the victim pages it is the first to write) has
            # been copied, and nothing beyond the copy sets of the launches
            # its victim window reaches
            so_far[res.cow_sets[j - T1].astype(np.int64)] = 1
            # launch numbers count from 1 at the checkpoint's open; a call
            # takes the window from the first launch not yet taken, at least
            # through its own, `window` launches (`first` for the first call),
            # cut at its validation call's end
            q, last = j - T1 + 1, (g + 1) * 20 - T1
            if q > covered:
                covered = max(q, min(last, covered + (first if covered == 0 else window)))
            upto = np.zeros(w.n_pages, np.uint8)
            for cs in res.cow_sets[:covered]:
                upto[cs.astype(np.int64)] = 1
            env.app.synchronize()
            got = bits_to_pages(phos.phos_ckpt_copied(ck, w.n_pages), w.n_pages)
            assert not np.any(so_far & ~got), f"pages missing before launch {j}"
            assert not np.any(got & ~upto), f"pages copied ahead of validation before launch {j}"
        env.mutate(launches[j], groups[g].data_ptr() + (j % 20) * N * 8, N)
    stats = phos.phos_ckpt_end(ck, env.app)
    T.cuda.synchronize()
    for j in range(T1, T2):
        phos.phos_spec_release(env.ctx, specs[j])
    assert np.array_equal(image.cpu().numpy(), res.snapshots[0]), "CoW image != snapshot at t1"
    assert stats.cow_pages == int(union.sum())
    assert stats.bg_pages + stats.cow_pages == env.image_bytes // w.page_bytes
    assert np.array_equal(env.pool_host(), host)


@pytest.mark.parametrize("policy,defer,budget", [
    ("host_direct", True, 0), ("host_direct", True, 10), ("host_direct", True, None),
    ("host_direct", False, 64),
    ("block", True, 1), ("block", True, 7), ("block", False, 64), ("block", True, None)])
def test_cow_staging_host_image(env, policy, defer, budget):
    """Copy-on-write into a pinned host image through a device staging area of
    `budget` pages (None: room for every page).  host_direct: staged pages
    reach the image at the end, the overflow goes straight to the host.
    block: the area is a ring the host drains during the checkpoint, every
    copy-on-write page goes through it and waits for a free slot when it is
    full (1 and 7 slots: the ring wraps thousands of times).  The image is the
    t1 snapshot either way."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    res = oracle.run_stream(w, launches[T1:T2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(0,), cow_window=(0, T2 - T1), keep_violations=False)
    himg = T.zeros(env.image_bytes, dtype=T.uint8, pin_memory=True)
    pages = w.n_pages if budget is None else budget
    staging = T.empty(max(1, pages) * w.page_bytes, dtype=T.uint8, device="cuda")
    T.cuda.synchronize()
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND if defer else 0,
                              himg, None, env.copy)
    phos.phos_ckpt_staging_policy(ck, staging, pages * w.page_bytes,
                                  phos.STAGE_BLOCK if policy == "block" else phos.STAGE_HOST_DIRECT)
    out, cnt = env.violations_buffers(N)
    for j in range(T1, T2):
        L = launches[j]
        s = env.spec(L)
        r = st.records(j)
        _validate(env, s, r, out, cnt)
        phos.phos_ckpt_cow(ck, s, env.app)
        env.mutate(L, r.data_ptr(), N)
        phos.phos_spec_release(env.ctx, s)
    stats = phos.phos_ckpt_end(ck, env.app)
    assert np.array_equal(himg.numpy(), res.snapshots[0]), "CoW host image != snapshot at t1"
    n_img_pages = env.image_bytes // w.page_bytes
    assert stats.bg_pages + stats.cow_pages == n_img_pages
    if policy == "block":
        assert stats.staged_pages == stats.cow_pages
    else:
        assert stats.staged_pages == min(stats.cow_pages, pages)
    if defer:
        assert stats.cow_pages == sum(len(c) for c in res.cow_sets)
    assert np.array_equal(env.pool_host(), host)


def test_blocking_staging_wait_timeout():
    """Section 4.2 blocking policy, failure handling forced from the host: a
    one-slot ring under a device wait budget of one poll.  Copies that wait
    for a slot give up and go straight to the image, every kernel exits
    normally, the checkpoint reports PHOS_E_TIMEOUT within seconds (the drain
    stops at the first slot left unpublished), and the device keeps working."""
    import os
    import time
    from paper_2405_12079_amd import phos
    w = synth.config1_world()
    old = os.environ.get("PHOS_SPIN_LIMIT")
    os.environ["PHOS_SPIN_LIMIT"] = "1"  # read when the context is created
    try:
        env = Env(w)
    finally:
        if old is None:
            del os.environ["PHOS_SPIN_LIMIT"]
        else:
            os.environ["PHOS_SPIN_LIMIT"] = old
    T = env.T
    try:
        launches = synth.config1_launches(w)[:6]
        st = Stream(env, launches)
        himg = T.zeros(env.image_bytes, dtype=T.uint8, pin_memory=True)
        staging = T.empty(w.page_bytes, dtype=T.uint8, device="cuda")
        T.cuda.synchronize()
        t0 = time.perf_counter()
        ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, himg, None, env.copy)
        phos.phos_ckpt_staging_policy(ck, staging, w.page_bytes, phos.STAGE_BLOCK)
        out, cnt = env.violations_buffers(N)
        for j, L in enumerate(launches):
            s = env.spec(L)
            r = st.records(j)
            _validate(env, s, r, out, cnt)
            phos.phos_ckpt_cow(ck, s, env.app)
            env.mutate(L, r.data_ptr(), N)
            phos.phos_spec_release(env.ctx, s)
        with pytest.raises(phos.PhosError) as e:
            phos.phos_ckpt_end(ck, env.app)
        assert e.value.status == phos.E_TIMEOUT
        assert time.perf_counter() - t0 < 30
        T.cuda.synchronize()
        x = T.arange(1 << 20, device="cuda", dtype=T.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    finally:
        env.close()


def test_staging_rejects_bad_use(env):
    phos, T = env.phos, env.T
    dimg = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    staging = T.empty(1 << 20, dtype=T.uint8, device="cuda")
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, dimg, None, env.copy)
    with pytest.raises(phos.PhosError) as e:  # a device image needs no staging
        phos.phos_ckpt_staging(ck, staging, 1 << 20)
    assert e.value.status == phos.E_INVAL
    phos.phos_ckpt_end(ck, env.app)
    himg = T.empty(env.image_bytes, dtype=T.uint8, pin_memory=True)
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, himg, None, env.copy)
    with pytest.raises(phos.PhosError) as e:  # staging in host memory
        phos.phos_ckpt_staging(ck, himg, 1 << 20)
    assert e.value.status == phos.E_INVAL
    with pytest.raises(phos.PhosError) as e:  # no such policy
        phos.phos_ckpt_staging_policy(ck, staging, 1 << 20, 7)
    assert e.value.status == phos.E_INVAL
    phos.phos_ckpt_end(ck, env.app)
    pageable = T.empty(env.image_bytes, dtype=T.uint8)
    with pytest.raises(phos.PhosError) as e:  # no kernel may write pageable memory
        phos.phos_ckpt_begin(env.ctx, phos.COW, 0, pageable, None, env.copy)
    assert e.value.status == phos.E_INVAL


def _tracked(env, launches, j0, j1):
    """The oracle's dirty and victim pages of launches j0..j1-1, and per page
    the last launch j with a failing write inside a buffer there (-1: none)."""
    w = env.world
    d, v, last = oracle.track_launches(
        env.table, j1 - j0,
        lambda i: (launches[j0 + i].arg_values(env.base), synth.records_host(env.hw, launches[j0 + i])),
        env.base, w.page_bytes, w.n_pages, threads=4)
    return d, v, np.where(last >= 0, last + j0, -1)


@pytest.mark.parametrize("mode", ["plain", "drain", "deferred", "implicit", "precopy"])
def test_soft_recopy_config1(env, mode):
    """deferred: the background copy starts at the recopy, when every page the
    window wrote is already traced, so it copies exactly the untraced pages;
    implicit: no recopy call, phos_ckpt_end recopies; precopy: two pre-copy
    rounds inside the window (iterative recopy)."""
    phos, w, T = env.phos, env.world, env.T
    drain = mode == "drain"
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    res = oracle.run_stream(w, launches[T1:T2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(T2 - T1,), window=(0, T2 - T1), keep_violations=False)
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    himg = T.empty(env.image_bytes, dtype=T.uint8, pin_memory=True) if drain else None
    flags = phos.CKPT_DEFER_BACKGROUND if mode == "deferred" else 0
    ck = phos.phos_ckpt_begin(env.ctx, phos.RECOPY, flags, image, himg, env.copy)
    out, cnt = env.violations_buffers(N)
    rounds = [T1 + (T2 - T1) // 3, T1 + 2 * (T2 - T1) // 3] if mode == "precopy" else []
    for j in range(T1, T2):
        if j in rounds:
            phos.phos_ckpt_precopy(ck, env.app)
        L = launches[j]
        s = env.spec(L)
        r = st.records(j)
        _validate(env, s, r, out, cnt)
        env.mutate(L, r.data_ptr(), N)
        phos.phos_spec_release(env.ctx, s)
    if mode != "implicit":
        phos.phos_ckpt_recopy(ck, env.app)
    else:
        with pytest.raises(phos.PhosError) as e:  # its recopy list lives in the maps
            phos.phos_track_reset(env.ctx, env.app)
        assert e.value.status == phos.E_STATE
    d = phos.phos_track_read(env.ctx, 0, w.n_pages)
    v = phos.phos_track_read(env.ctx, 1, w.n_pages)
    # the final recopy sees only the marks made after the last round
    per_launch = [_tracked(env, launches, j, j + 1)[0] for j in range(T1, T2)] if rounds else []
    dirty_left, pre = (oracle.precopy_rounds(per_launch, [r - T1 for r in rounds], _buffer_pages(env))
                       if rounds else (res.dirty, 0))
    assert np.array_equal(d, oracle.pages_to_bitmap(dirty_left, w.n_pages))
    assert np.array_equal(v, oracle.pages_to_bitmap(res.victim, w.n_pages))
    stats = phos.phos_ckpt_end(ck, env.app)
    want = res.snapshots[T2 - T1]
    assert np.array_equal(image.cpu().numpy(), want), "recopy image != snapshot at t2"
    if drain:
        assert np.array_equal(himg.numpy(), want), "drained host image differs"
    assert stats.recopy_pages == oracle.recopy_pages(dirty_left, res.victim, _buffer_pages(env))
    assert stats.precopy_pages == pre
    n_img_pages = env.image_bytes // w.page_bytes
    if mode == "deferred":
        assert stats.bg_pages + stats.recopy_pages == n_img_pages
    else:
        assert n_img_pages - stats.recopy_pages - stats.precopy_pages <= stats.bg_pages <= n_img_pages
    # launches after t2 leave the image unchanged
    _run_plain(env, st, host, T2, T2 + 5)
    assert np.array_equal(image.cpu().numpy(), want)


@pytest.mark.parametrize("vstream", ["same", "other"])
def test_precopy_final_rounds(env, vstream):
    """Iterative recopy with the window's remaining launches known: every
    launch of the window is validated up front in one batched call (as the
    training step does), and two rounds copy the pages whose last write in
    the window has been issued: dirty pages outside the write intervals of
    the launches still to come, and victim pages (outside them too) whose
    last failing write came from a launch issued already.  With the
    validation on a stream of its own ("other", waited for with an event)
    the victim marks are not ordered before the rounds, which then leave
    every victim page to the recopy.  The maps left, the pages copied by the
    rounds and by the recopy follow the oracle, and the image is the
    snapshot at t2."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    res = oracle.run_stream(w, launches[T1:T2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(T2 - T1,), window=(0, T2 - T1), keep_violations=False)
    last = _tracked(env, launches, T1, T2)[2]
    T.cuda.synchronize()
    groups = {g: env.records(launches[g * 20:(g + 1) * 20], N) for g in range(T1 // 20, T2 // 20)}
    T.cuda.synchronize()
    specs = {j: env.spec(launches[j]) for j in range(T1, T2)}
    ptr = {j: groups[j // 20].data_ptr() + (j % 20) * N * 8 for j in range(T1, T2)}
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    ck = phos.phos_ckpt_begin(env.ctx, phos.RECOPY, 0, image, None, env.copy)
    cap = 200_000
    out, cnt = env.violations_buffers(cap)
    vs = T.cuda.Stream() if vstream == "other" else env.app
    vs.wait_stream(env.app)
    phos.phos_validate_batch(env.ctx, [specs[j] for j in range(T1, T2)],
                             [ptr[j] for j in range(T1, T2)], [N] * (T2 - T1), V, out, cap, cnt,
                             vs)
    env.app.wait_stream(vs)
    with pytest.raises(phos.PhosError) as e:  # more launches ahead than upcoming
        phos.phos_ckpt_precopy_final(ck, [specs[T2 - 1]], 2, env.app)
    assert e.value.status == phos.E_INVAL
    rounds = [T1 + (T2 - T1) // 2, T2 - 6]
    for j in range(T1, T2):
        if j in rounds:
            phos.phos_ckpt_precopy_final(ck, [specs[i] for i in range(j, T2)], T2 - j, env.app)
        env.mutate(launches[j], ptr[j], N)
    phos.phos_ckpt_recopy(ck, env.app)
    with pytest.raises(phos.PhosError) as e:  # no round after the recopy
        phos.phos_ckpt_precopy_final(ck, [], 0, env.app)
    assert e.value.status == phos.E_STATE
    d = phos.phos_track_read(env.ctx, 0, w.n_pages)
    v = phos.phos_track_read(env.ctx, 1, w.n_pages)
    stats = phos.phos_ckpt_end(ck, env.app)
    T.cuda.synchronize()
    for j in range(T1, T2):
        phos.phos_spec_release(env.ctx, specs[j])
    inbuf = _buffer_pages(env)
    if vstream == "other":
        last[:] = -1  # no victim page is known to be final
    dirty_left, victim_left, pre = oracle.final_rounds(
        res.dirty, res.victim, last, rounds,
        lambda r: oracle.write_pages(env.table, [L.arg_values(env.base) for L in launches[r:T2]],
                                     env.base, w.page_bytes, w.n_pages), inbuf)
    assert np.array_equal(d, oracle.pages_to_bitmap(dirty_left.astype(np.uint8), w.n_pages))
    assert np.array_equal(v, oracle.pages_to_bitmap(victim_left.astype(np.uint8), w.n_pages))
    if vstream == "same":  # victims went early too
        assert int(victim_left.sum()) < int(res.victim.astype(bool).sum())
    assert stats.precopy_pages == pre > 0
    assert stats.recopy_pages == oracle.recopy_pages(dirty_left, victim_left, inbuf)
    assert np.array_equal(image.cpu().numpy(), res.snapshots[T2 - T1]), "image != snapshot at t2"


@pytest.mark.parametrize("window", ["whole", "empty"])
def test_precopy_final_degenerate(env, window):
    """Degenerate final-page rounds.  "whole": one round after the window's
    last launch (nothing upcoming) takes every dirty and victim page, and the
    recopy at the re-quiesce then copies none.  "empty": a window with no
    launch; the round copies nothing.  The image is the snapshot at t2
    either way."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    _run_plain(env, st, host, 0, T1)
    t2 = T2 if window == "whole" else T1
    res = oracle.run_stream(w, launches[T1:t2], env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(t2 - T1,), window=(0, t2 - T1), keep_violations=False)
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    ck = phos.phos_ckpt_begin(env.ctx, phos.RECOPY, 0, image, None, env.copy)
    out, cnt = env.violations_buffers(N)
    for j in range(T1, t2):
        L = launches[j]
        sp = env.spec(L)
        r = st.records(j)
        _validate(env, sp, r, out, cnt)
        env.mutate(L, r.data_ptr(), N)
        phos.phos_spec_release(env.ctx, sp)
    phos.phos_ckpt_precopy_final(ck, [], 0, env.app)
    phos.phos_ckpt_recopy(ck, env.app)
    d = phos.phos_track_read(env.ctx, 0, w.n_pages)
    v = phos.phos_track_read(env.ctx, 1, w.n_pages)
    stats = phos.phos_ckpt_end(ck, env.app)
    assert not d.any() and not v.any()
    assert stats.recopy_pages == 0
    assert stats.precopy_pages == oracle.recopy_pages(res.dirty, res.victim, _buffer_pages(env))
    if window == "whole":
        assert stats.precopy_pages > 0
    assert np.array_equal(image.cpu().numpy(), res.snapshots[t2 - T1]), "image != snapshot at t2"


@pytest.mark.parametrize("mode", ["separate", "pair", "pair_precopy"])
def test_both_protocols_open_together(env, mode):
    """A CoW checkpoint (t1 image) and a recopy checkpoint (t2 image) over one
    window.  separate: each with its own background pass; pair: one shared
    pass (phos_ckpt_start_pair) that reads each page once for both images,
    with the recopy checkpoint on another copy stream; pair_precopy: the
    same, with two pre-copy rounds of the recopy image in the window.  Either
    way the copy-on-write image is the snapshot at t1 and the recopy image
    the snapshot at t2, and every image page is copied once per image by
    exactly one path of its checkpoint."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)[:40]
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    res = oracle.run_stream(w, launches, env.base, lambda L: synth.records_host(env.hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, env.base, w.seed, L.k, rec),
                            host, snap_before=(0, 40), keep_violations=False)
    img_a = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    img_b = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    copy2 = T.cuda.Stream()
    pair = mode != "separate"
    flags = phos.CKPT_DEFER_BACKGROUND if pair else 0
    ca = phos.phos_ckpt_begin(env.ctx, phos.COW, flags, img_a, None, env.copy)
    cb = phos.phos_ckpt_begin(env.ctx, phos.RECOPY, flags, img_b, None, copy2)
    with pytest.raises(phos.PhosError):
        phos.phos_ckpt_begin(env.ctx, phos.COW, 0, img_a, None, env.copy)
    if pair:
        with pytest.raises(phos.PhosError) as e:  # a copy-on-write, then a recopy checkpoint
            phos.phos_ckpt_start_pair(cb, ca, None)
        assert e.value.status == phos.E_INVAL
        phos.phos_ckpt_start_pair(ca, cb, env.app)
        with pytest.raises(phos.PhosError) as e:
            phos.phos_ckpt_start(cb, None)
        assert e.value.status == phos.E_STATE
    rounds = (13, 27) if mode == "pair_precopy" else ()
    out, cnt = env.violations_buffers(N)
    for j, L in enumerate(launches):
        if j in rounds:
            phos.phos_ckpt_precopy(cb, env.app)
        s = env.spec(L)
        r = st.records(j)
        _validate(env, s, r, out, cnt)
        phos.phos_ckpt_cow(ca, s, env.app)
        env.mutate(L, r.data_ptr(), N)
        phos.phos_spec_release(env.ctx, s)
    phos.phos_ckpt_recopy(cb, env.app)
    sa = phos.phos_ckpt_end(ca, env.app)
    sb = phos.phos_ckpt_end(cb, env.app)
    assert np.array_equal(img_a.cpu().numpy(), res.snapshots[0]), "copy-on-write image != t1"
    assert np.array_equal(img_b.cpu().numpy(), res.snapshots[40]), "recopy image != t2"
    n_img_pages = env.image_bytes // w.page_bytes
    assert sa.bg_pages + sa.cow_pages == n_img_pages
    assert n_img_pages - sb.recopy_pages - sb.precopy_pages <= sb.bg_pages <= n_img_pages
    if rounds:
        assert sb.precopy_pages > 0
    if pair:  # one read per page for both images
        assert max(sa.bg_pages, sb.bg_pages) <= sa.bg_read_pages <= sa.bg_pages + sb.bg_pages
        assert sb.bg_read_pages == 0
    else:
        assert (sa.bg_read_pages, sb.bg_read_pages) == (sa.bg_pages, sb.bg_pages)


def test_cow_straight_to_pinned_host(env):
    """No device staging: the image is pinned host memory written over PCIe."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)[:10]
    st = Stream(env, launches)
    want = oracle.snapshot(synth.content_host(w.seed, 0, w.pool_bytes), env.base, env.table)
    himg = T.empty(env.image_bytes, dtype=T.uint8, pin_memory=True)
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, 0, himg, None, env.copy)
    out, cnt = env.violations_buffers(N)
    for j, L in enumerate(launches):
        s = env.spec(L)
        r = st.records(j)
        _validate(env, s, r, out, cnt)
        phos.phos_ckpt_cow(ck, s, env.app)
        env.mutate(L, r.data_ptr(), N)
        phos.phos_spec_release(env.ctx, s)
    phos.phos_ckpt_end(ck, env.app)
    assert np.array_equal(himg.numpy(), want)


@pytest.mark.parametrize("mode", ["background", "deferred", "prefetch", "host_image", "chunked",
                                  "mixed", "pageable"])
def test_concurrent_restore_config1(env, mode):
    """chunked: pinned host pieces; mixed: every other piece pageable (moved by
    DMA, never read by a kernel); pageable: one pageable host image."""
    phos, w, T = env.phos, env.world, env.T
    launches = synth.config1_launches(w)[:20]
    st = Stream(env, launches)
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    image_h = oracle.snapshot(host, env.base, env.table)
    chunks = None
    dma_want = 0
    if mode == "host_image":
        image = T.from_numpy(image_h.copy()).pin_memory()
    elif mode == "pageable":
        image = T.from_numpy(image_h.copy())
        dma_want = env.image_bytes // w.page_bytes
    elif mode in ("chunked", "mixed"):
        # the image in host pieces of 3 MiB (the last one partly used)
        cb = 3 << 20
        chunks = []
        for k, o in enumerate(range(0, image_h.size, cb)):
            piece = T.zeros(cb, dtype=T.uint8)
            if mode == "chunked" or k % 2 == 0:
                piece = piece.pin_memory()
            else:
                dma_want += (min(cb, image_h.size - o)) // w.page_bytes
            piece[:min(cb, image_h.size - o)] = T.from_numpy(image_h[o:o + cb].copy())
            chunks.append(piece)
        image = None
    else:
        image = T.from_numpy(image_h.copy()).cuda()
    env.pool.fill_(0xAB)  # the pool before restore holds garbage
    T.cuda.synchronize()
    flags = {"background": 0, "deferred": phos.RST_DEFER_BACKGROUND,
             "prefetch": phos.RST_DEFER_BACKGROUND | phos.RST_PREFETCH_SPEC,
             "host_image": 0, "chunked": 0, "mixed": 0, "pageable": 0}[mode]
    if chunks is not None:
        rs = phos.phos_restore_begin_chunked(env.ctx, flags, chunks, 3 << 20, env.copy)
    else:
        rs = phos.phos_restore_begin(env.ctx, flags, image, env.copy)
    faulted = T.zeros(1, dtype=T.int64, device="cuda")
    present = np.zeros(w.n_pages, np.uint8)
    for j, L in enumerate(launches):
        s = env.spec(L)
        r = st.records(j)
        phos.phos_restore_on_demand(rs, s, r, N, env.app, faulted)
        env.mutate(L, r.data_ptr(), N)
        rec_h = synth.records_host(env.hw, L)
        present |= oracle.needed_pages(env.table, L.arg_values(env.base), rec_h, env.base,
                                       w.page_bytes, w.n_pages, prefetch=mode == "prefetch")
        if mode in ("deferred", "prefetch") and j % 5 == 0:
            env.app.synchronize()
            got = bits_to_pages(phos.phos_restore_present(rs, w.n_pages), w.n_pages)
            assert np.array_equal(got, present), f"present pages after launch {j}"
            if mode == "deferred":
                assert int(faulted.item()) == int(present.sum())
        synth.apply_writes_host(host, env.base, w.seed, L.k, rec_h)
        phos.phos_spec_release(env.ctx, s)
    stats = phos.phos_restore_end(rs, env.app)
    assert stats.dma_pages == dma_want
    assert stats.bg_pages + stats.demand_pages + stats.dma_pages == env.image_bytes // w.page_bytes
    inbuf = np.repeat(_buffer_pages(env).astype(bool), w.page_bytes)
    got = env.pool_host()
    assert np.array_equal(got[inbuf], host[inbuf]), "restored pool + launches != oracle"


def test_restore_wait_timeout_ends_every_wait():
    """Section 6, failure handling forced from the host: launches wait for
    pages of a pageable image that the host's DMA has not brought in yet,
    under a device wait budget of one poll.  Every wait gives up, every
    kernel exits normally, the restore reports PHOS_E_TIMEOUT within seconds,
    and the device and the context keep working afterwards."""
    import os
    import time
    from paper_2405_12079_amd import phos
    w = synth.config1_world()
    old = os.environ.get("PHOS_SPIN_LIMIT")
    os.environ["PHOS_SPIN_LIMIT"] = "1"  # read when the context is created
    try:
        env = Env(w)
    finally:
        if old is None:
            del os.environ["PHOS_SPIN_LIMIT"]
        else:
            os.environ["PHOS_SPIN_LIMIT"] = old
    T = env.T
    try:
        launches = synth.config1_launches(w)[:4]
        recs = env.records(launches, N)
        host = synth.content_host(w.seed, 0, w.pool_bytes)
        image = T.from_numpy(oracle.snapshot(host, env.base, env.table))  # pageable: DMA only
        T.cuda.synchronize()
        t0 = time.perf_counter()
        rs = phos.phos_restore_begin(env.ctx, 0, image, env.copy)
        for j, L in enumerate(launches):
            s = env.spec(L)
            phos.phos_restore_on_demand(rs, s, recs[j * N:(j + 1) * N], N, env.app, None)
            phos.phos_spec_release(env.ctx, s)
        with pytest.raises(phos.PhosError) as e:
            phos.phos_restore_end(rs, env.app)
        assert e.value.status == phos.E_TIMEOUT
        assert time.perf_counter() - t0 < 30
        # the error was consumed; the device and the context still work
        T.cuda.synchronize()
        x = T.arange(1 << 20, device="cuda", dtype=T.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
        image_d = image.cuda()
        rs = phos.phos_restore_begin(env.ctx, 0, image_d, env.copy)
        phos.phos_restore_end(rs, env.app)
        got = env.pool_host()
        inbuf = np.repeat(_buffer_pages(env).astype(bool), w.page_bytes)
        assert np.array_equal(got[inbuf], host[inbuf])
    finally:
        env.close()


def test_image_manifest_guards_the_restore(env):
    """Section 2.2: the image holds the buffers' bytes only; its manifest
    names them.  A restore through the manifest of the same buffers gives
    the image back; a damaged manifest, or one written for other buffers, is
    refused before anything is copied."""
    phos, w, T = env.phos, env.world, env.T
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    image = T.from_numpy(oracle.snapshot(host, env.base, env.table)).cuda()
    m = phos.phos_manifest_write(env.ctx, phos.COW)
    assert len(m) == 32 + 16 * w.n_alloc + 8 and m[:8] == b"PHOSIMG1"
    phos.phos_manifest_check(env.ctx, m)
    for bad in (m[:-1] + bytes([m[-1] ^ 1]), m[:40] + bytes([m[40] ^ 1]) + m[41:], m[:-8]):
        with pytest.raises(phos.PhosError) as e:
            phos.phos_manifest_check(env.ctx, bad)
        assert e.value.status == phos.E_INVAL
    # the same buffer sizes at other places in the pool: accepted (an image
    # maps buffer i to buffer i); one buffer of another size: refused
    other = Env(synth.config1_world())
    try:
        bufs = other.world.buffers(other.base)
        phos.phos_manifest_check(other.ctx, m)
        b0, n0 = bufs[0]
        phos.phos_buffers_register(other.ctx, [(b0, n0 + w.page_bytes)] + bufs[1:]
                                   if bufs[1][0] >= b0 + n0 + w.page_bytes else bufs[:-1])
        with pytest.raises(phos.PhosError) as e:
            phos.phos_manifest_check(other.ctx, m)
        assert e.value.status == phos.E_INVAL
        with pytest.raises(phos.PhosError) as e:
            phos.phos_restore_begin_manifest(other.ctx, 0, image, m, other.copy)
        assert e.value.status == phos.E_INVAL
    finally:
        other.close()
    env.pool.zero_()
    T.cuda.synchronize()
    rs = phos.phos_restore_begin_manifest(env.ctx, 0, image, m, env.copy)
    phos.phos_restore_end(rs, env.app)
    got = env.pool_host()
    assert np.array_equal(oracle.snapshot(got, env.base, env.table), image.cpu().numpy())


def test_restore_without_launches_is_the_image(env):
    phos, w, T = env.phos, env.world, env.T
    host = synth.content_host(w.seed, 0, w.pool_bytes)
    image_h = oracle.snapshot(host, env.base, env.table)
    image = T.from_numpy(image_h.copy()).cuda()
    env.pool.zero_()
    T.cuda.synchronize()
    rs = phos.phos_restore_begin(env.ctx, 0, image, env.copy)
    phos.phos_restore_end(rs, env.app)
    got = env.pool_host()
    assert np.array_equal(oracle.snapshot(got, env.base, env.table), image_h)


def test_protocol_errors(env):
    phos, T = env.phos, env.T
    image = T.empty(env.image_bytes + 16, dtype=T.uint8, device="cuda")
    L = synth.config1_launches(env.world, 1, 1)[0]
    s = env.spec(L)
    ck = phos.phos_ckpt_begin(env.ctx, phos.RECOPY, 0, image, None, env.copy)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_ckpt_cow(ck, s, env.app)
    assert e.value.status == phos.E_STATE
    with pytest.raises(phos.PhosError) as e:
        phos.phos_buffers_register(env.ctx, env.world.buffers(env.base))
    assert e.value.status == phos.E_STATE
    with pytest.raises(phos.PhosError) as e:
        phos.phos_restore_begin(env.ctx, 0, image, env.copy)
    assert e.value.status == phos.E_STATE
    phos.phos_ckpt_recopy(ck, env.app)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_ckpt_recopy(ck, env.app)
    assert e.value.status == phos.E_STATE
    phos.phos_ckpt_end(ck, env.app)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_ckpt_begin(env.ctx, phos.COW, 0, image[8:], None, env.copy)
    assert e.value.status == phos.E_INVAL
    ck = phos.phos_ckpt_begin(env.ctx, phos.COW, 0, image, None, env.copy)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_ckpt_recopy(ck, env.app)
    assert e.value.status == phos.E_STATE
    phos.phos_ckpt_end(ck, env.app)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_validate(env.ctx, 12345, 0, 0, 3, 0, 0, 0, env.app)
    assert e.value.status == phos.E_INVAL
    out, cnt = env.violations_buffers(16)
    s2 = env.spec(L)
    with pytest.raises(phos.PhosError) as e:  # violation output not 16-byte aligned
        phos.phos_validate(env.ctx, s2, 0, 0, 3, out.data_ptr() + 8, 8, cnt, env.app)
    assert e.value.status == phos.E_INVAL
    phos.phos_spec_release(env.ctx, s2)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_spec_register(env.ctx, 0, [(4, 0, env.base, 64)])  # range without mode
    assert e.value.status == phos.E_INVAL
    with pytest.raises(phos.PhosError) as e:
        phos.phos_buffers_register(env.ctx, [(env.base + 100, 4096)])  # misaligned
    assert e.value.status == phos.E_INVAL
    with pytest.raises(phos.PhosError) as e:
        phos.phos_create(0, env.base + 8, 1 << 20, 4096)
    assert e.value.status == phos.E_INVAL
    phos.phos_spec_release(env.ctx, s)
