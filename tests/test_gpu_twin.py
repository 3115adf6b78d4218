"""GPU parity of the twin kernel (Section 4.1): an application kernel with the
validator fused in.  Its violations, dirty and victim maps must equal the
oracle's validation and tracking of the record stream made of the kernel's own
accesses (per element i: read x[i], read idx[i], read y[j], write y[j]); its
memory effect must equal the uninstrumented kernel's.  Integer work: the bar is
bit-exact (violations compared as sets: the twin reports them unordered)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_harness import Env, bits_to_pages

pytestmark = pytest.mark.gpu
RW_T = 1 | 2 | 4
MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def env1():
    e = Env(synth.config1_world())
    yield e
    e.close()


def _pick(w):
    """x: the largest buffer, y and idx the next two (x longer than n, so
    writes can be aimed at its unread tail); other buffers are victims."""
    order = np.argsort(-w.alloc_bytes.astype(np.int64), kind="stable")
    bx, by, bi = (int(order[0]), int(order[1]), int(order[2]))
    others = [int(b) for b in order[3:]]
    return bx, by, bi, others


def _free_pages(w):
    """Pool pages covered by no buffer (gaps and the free tail)."""
    cov = np.zeros(w.n_pages, bool)
    for o, b in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
        cov[o // w.page_bytes:(o + b) // w.page_bytes] = True
    return np.flatnonzero(~cov)


def _case(env, n, n_inject, indirect, n_extra, seed):
    """Inputs of one launch: offsets (bytes from the pool base) of x, y, idx,
    the idx values, the spec arguments and the element count."""
    w = env.world
    bx, by, bi, others = _pick(w)
    off = w.alloc_off.astype(np.int64)
    nb = w.alloc_bytes.astype(np.int64)
    nmax = int(min(nb[by], nb[bi]) // 8)
    n = min(n, nmax, int(nb[bx] // 8) - 64)
    rng = np.random.default_rng(seed)
    j = rng.permutation(n).astype(np.int64) if indirect else np.arange(n, dtype=np.int64)
    # injected targets, all distinct and outside what the kernel reads or
    # writes otherwise: other buffers (not named: victims), x's unread tail
    # (named read-only) and free pages (no buffer)
    free = _free_pages(w)
    pos = rng.choice(n, size=min(n_inject, n), replace=False)
    targets = set()
    for k, p in enumerate(pos):
        kind = k % 3
        while True:
            if kind == 0:
                b = others[int(rng.integers(len(others)))]
                a = off[b] + 8 * int(rng.integers(nb[b] // 8))
            elif kind == 1:
                a = off[bx] + 8 * int(rng.integers(n + 1, nb[bx] // 8))
            else:
                pg = int(free[int(rng.integers(len(free)))])
                a = pg * w.page_bytes + 8 * int(rng.integers(w.page_bytes // 8))
            if a not in targets:
                targets.add(a)
                break
        j[p] = (a - off[by]) // 8
    base = env.base
    args = [(1, 0, base + int(off[bx]), 0), (2, 0, base + int(off[by]), 0),
            (1, 0, base + int(off[bi]), 0)]
    for b in others[:n_extra]:  # more named read-only buffers: more intervals
        args.append((1, 0, base + int(off[b]), 0))
    return int(off[bx]), int(off[by]), int(off[bi]), j, args, n


def _records(base, xo, yo, io, j, indirect):
    """The kernel's accesses as a record stream, in element order."""
    n = j.shape[0]
    i = np.arange(n, dtype=np.uint64)
    xa = np.uint64(base + xo) + 8 * i
    ya = (np.int64(base + yo) + 8 * j).astype(np.uint64)
    cols = [xa]
    if indirect:
        cols.append(np.uint64(base + io) + 8 * i)
    cols += [ya, ya | np.uint64(1)]
    return np.stack(cols, axis=1).reshape(-1), len(cols)


def _run(env, xo, yo, io, j, n, spec, flags, indirect, cap):
    phos, T = env.phos, env.T
    pool64 = env.pool.view(T.int64)
    if indirect:
        pool64[io // 8: io // 8 + n] = T.from_numpy(j).to("cuda")
    out, cnt = env.violations_buffers(cap)
    T.cuda.synchronize()  # inputs were made on the default stream; the kernel runs on app
    phos.phos_twin_scale_add(env.ctx, spec, env.base + xo, env.base + yo,
                             env.base + io if indirect else 0, n, flags, out.data_ptr(), cap,
                             cnt.data_ptr(), env.app)
    env.app.synchronize()
    return Env.read_violations(out, cnt, cap)


def _key(v, per):
    return sorted((int(x["index"]) // per if per else int(x["index"]), int(x["addr"]),
                   int(x["is_write"]), int(x["reason"]), int(x["victim"]), int(x["launch_id"]))
                  for x in v)


@pytest.mark.parametrize("n,inject,indirect,extra",
                         [(100_003, 300, True, 0), (65_536, 0, False, 0), (77_777, 120, True, 10),
                          (1, 1, True, 0), (0, 0, False, 0)])
def test_twin_matches_oracle(env1, n, inject, indirect, extra):
    env, w, phos = env1, env1.world, env1.phos
    xo, yo, io, j, args, n = _case(env, n, inject, indirect, extra, seed=n + inject)
    rec, per = _records(env.base, xo, yo, io, j, indirect)
    iv = oracle.spec_build(env.table, args)
    spec = phos.phos_spec_register(env.ctx, 7, args)
    try:
        assert len(phos.phos_spec_intervals(env.ctx, spec)) == len(iv)
        before = env.pool_host().copy()
        phos.phos_track_reset(env.ctx, env.app)
        cap = max(1, 4 * inject + 16)
        nv, got = _run(env, xo, yo, io, j, n, spec, RW_T, indirect, cap)
        want = oracle.validate(iv, rec, env.table, launch_id=7, flags=1 | 2)
        assert nv == want.shape[0]
        assert _key(got, 0) == _key(want, per)
        # tracking: the oracle's dirty / victim pages of the same stream
        dirty = np.zeros(w.n_pages, np.uint8)
        vic = np.zeros(w.n_pages, np.uint8)
        oracle.track(iv, rec, env.table, env.base, w.page_bytes, w.n_pages, dirty, vic)
        assert np.array_equal(bits_to_pages(phos.phos_track_read(env.ctx, 0, w.n_pages), w.n_pages),
                              dirty)
        assert np.array_equal(bits_to_pages(phos.phos_track_read(env.ctx, 1, w.n_pages), w.n_pages),
                              vic)
        # memory effect: every target t = y + 8 j gets 3 * old + x[i]
        after_twin = env.pool_host().copy()
        b64 = before.view(np.uint64).copy()
        if indirect:  # the idx array the kernel read was written into the pool first
            b64[io // 8: io // 8 + n] = j.view(np.uint64)
        exp = b64.copy()
        t = (yo // 8 + j).astype(np.int64)
        xs = b64[xo // 8: xo // 8 + n]
        exp[t] = (b64[t] * np.uint64(3) + xs) & np.uint64(MASK64)
        assert np.array_equal(after_twin.view(np.uint64), exp)
        # the uninstrumented kernel makes the same writes
        env.pool.copy_(env.T.from_numpy(before).to("cuda"))
        _run(env, xo, yo, io, j, n, spec, 0, indirect, 0)
        assert np.array_equal(env.pool_host(), after_twin)
    finally:
        env.pool.copy_(env.T.from_numpy(synth.content_host(w.seed, 0, w.pool_bytes)).to("cuda"))
        env.T.cuda.synchronize()
        phos.phos_spec_release(env.ctx, spec)


def test_twin_writes_only_and_overflow(env1):
    """Writes-only checking reports exactly the oracle's write violations; a
    cap below the count keeps the true count."""
    env, w, phos = env1, env1.world, env1.phos
    xo, yo, io, j, args, n = _case(env, 50_000, 90, True, 0, seed=5)
    rec, per = _records(env.base, xo, yo, io, j, True)
    iv = oracle.spec_build(env.table, args)
    spec = phos.phos_spec_register(env.ctx, 3, args)
    try:
        nv, got = _run(env, xo, yo, io, j, n, spec, 2, True, 1000)
        want = oracle.validate(iv, rec, env.table, launch_id=3, flags=2)
        assert nv == want.shape[0] == 90
        assert _key(got, 0) == _key(want, per)
        nv2, got2 = _run(env, xo, yo, io, j, n, spec, 2, True, 10)
        assert nv2 == 90 and got2.shape[0] == 10
    finally:
        env.pool.copy_(env.T.from_numpy(synth.content_host(w.seed, 0, w.pool_bytes)).to("cuda"))
        env.T.cuda.synchronize()
        phos.phos_spec_release(env.ctx, spec)


def test_twin_rejects_bad_arguments(env1):
    env, phos = env1, env1.phos
    out, cnt = env.violations_buffers(4)
    with pytest.raises(phos.PhosError) as e:  # instrumented without a count
        phos.phos_twin_scale_add(env.ctx, 0, env.base, env.base, 0, 8, 2, out.data_ptr(), 4, 0,
                                 env.app)
    assert e.value.status == phos.E_INVAL
    with pytest.raises(phos.PhosError) as e:  # misaligned y
        phos.phos_twin_scale_add(env.ctx, 0, env.base, env.base + 4, 0, 8, 0, 0, 0, 0, env.app)
    assert e.value.status == phos.E_INVAL
    with pytest.raises(phos.PhosError) as e:  # unknown spec
        phos.phos_twin_scale_add(env.ctx, 99999, env.base, env.base, 0, 8, 2, out.data_ptr(), 4,
                                 cnt.data_ptr(), env.app)
    assert e.value.status == phos.E_INVAL


@pytest.mark.parametrize("inject", [0, 3])
def test_twin_write_out_of_speculation_during_copy_on_write_is_a_misspeculation(env1, inject):
    """Section 4.2 with the validator inside the kernel: a copy-on-write
    checkpoint is open (background copy deferred, so only what copy-on-write
    takes is copied), copy-on-write takes the launch's write pages, then the
    twin runs.  Writes out of speculation into other buffers land on pages
    the checkpoint has not copied: phos_ckpt_end reports PHOS_E_MISSPEC.
    With none, the image is the snapshot at t1.  The next checkpoint starts
    clean either way."""
    env, w, phos, T = env1, env1.world, env1.phos, env1.T
    xo, yo, io, j, args, n = _case(env, 40_000, inject, True, 0, seed=11 + inject)
    spec = phos.phos_spec_register(env.ctx, 9, args)
    image = T.empty(env.image_bytes, dtype=T.uint8, device="cuda")
    try:
        # the index array the kernel reads is part of the state at t1
        env.pool.view(T.int64)[io // 8: io // 8 + n] = T.from_numpy(j).to("cuda")
        t1 = oracle.snapshot(env.pool_host(), env.base, env.table)
        ck = phos.phos_ckpt_begin(env.ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, image, None,
                                  env.copy)
        phos.phos_ckpt_cow(ck, spec, env.app)
        _run(env, xo, yo, io, j, n, spec, RW_T, True, 64)
        if inject:
            with pytest.raises(phos.PhosError) as e:
                phos.phos_ckpt_end(ck, env.app)
            assert e.value.status == phos.E_MISSPEC
        else:
            phos.phos_ckpt_end(ck, env.app)
            assert np.array_equal(image.cpu().numpy(), t1)
        # a later checkpoint with no instrumented launch in it ends cleanly
        ck = phos.phos_ckpt_begin(env.ctx, phos.COW, 0, image, None, env.copy)
        phos.phos_ckpt_end(ck, env.app)
        assert np.array_equal(image.cpu().numpy(),
                              oracle.snapshot(env.pool_host(), env.base, env.table))
    finally:
        env.pool.copy_(env.T.from_numpy(synth.content_host(w.seed, 0, w.pool_bytes)).to("cuda"))
        env.T.cuda.synchronize()
        phos.phos_spec_release(env.ctx, spec)
