"""phos_validate_noalloc, the validation entry point that allocates nothing
(its workspace is a fixed per-GPU array in device memory), through the C ABI
against phos_validate on the same seeded inputs: violation lists, counts and
the dirty / victim page maps of two calls in a row, the second smaller and
ragged, so the second runs over the workspace the first left behind.
Integer work: the bar is bit-exact.  Its limits are rejected on the host,
before any device work."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_harness import Env

pytestmark = pytest.mark.gpu
FLAGS = 1 | 2 | 4  # reads, writes, dirty / victim tracking


@pytest.fixture(scope="module")
def env():
    e = Env(synth.config1_world())
    yield e
    e.close()


def _call(env, fn, spec, rec, n, cap, stream):
    """One tracked validation from cleared maps: (count, violations, dirty, victim)."""
    phos = env.phos
    out, cnt = env.violations_buffers(cap)
    phos.phos_track_reset(env.ctx, stream)
    fn(env.ctx, spec, rec, n, FLAGS, out, cap, cnt, stream)
    stream.synchronize()
    nv, v = Env.read_violations(out, cnt, cap)
    dirty = phos.phos_track_read(env.ctx, 0, env.world.n_pages)
    victim = phos.phos_track_read(env.ctx, 1, env.world.n_pages)
    return nv, v, dirty, victim


def test_noalloc_matches_validate_twice(env):
    phos = env.phos
    sizes = (5_000_000, 123_457)  # hundreds of tiles, then a few dozen (ragged)
    launches = synth.config1_launches(env.world, 2, sizes[0])
    recs = [env.records([launches[j]], sizes[j]) for j in range(2)]
    specs = [env.spec(L) for L in launches]
    try:
        got = [_call(env, phos.phos_validate_noalloc, specs[j], recs[j], sizes[j], 20_000,
                     env.app) for j in range(2)]
        ref = [_call(env, phos.phos_validate, specs[j], recs[j], sizes[j], 20_000, env.app)
               for j in range(2)]
        for j in range(2):
            n, v, d, m = got[j]
            rn, rv, rd, rm = ref[j]
            assert n == rn > 0, (j, n, rn)
            assert np.array_equal(v, rv), f"call {j}: violations differ"
            assert np.array_equal(d, rd), f"call {j}: dirty maps differ"
            assert np.array_equal(m, rm), f"call {j}: victim maps differ"
        # and the small call against the oracle directly
        L = launches[1]
        iv = oracle.spec_build(env.table, L.arg_values(env.base))
        want = oracle.validate(iv, synth.records_host(env.hw, L, 0, sizes[1]), env.table, L.k)
        assert np.array_equal(got[1][1], want)
        phos.phos_stream_status(env.ctx, env.app)  # no overflow was raised
    finally:
        for s in specs:
            phos.phos_spec_release(env.ctx, s)


def test_noalloc_overflow_and_limits(env):
    phos = env.phos
    n = 1_000_000
    L = synth.config1_launches(env.world, 1, n)[0]
    rec = env.records([L], n)
    s = env.spec(L)
    out, cnt = env.violations_buffers(1000)
    try:
        # more violations than cap: the true count, and PHOS_E_OVERFLOW with V_SYNC
        with pytest.raises(phos.PhosError) as e:
            phos.phos_validate_noalloc(env.ctx, s, rec, n, 3 | phos.V_SYNC, out, 10, cnt, env.app)
        assert e.value.status == phos.E_OVERFLOW
        iv = oracle.spec_build(env.table, L.arg_values(env.base))
        want = oracle.validate(iv, synth.records_host(env.hw, L, 0, n), env.table, L.k)
        assert int(cnt.item()) == len(want) > 10
        with pytest.raises(phos.PhosError) as e:  # sticky until read
            phos.phos_stream_status(env.ctx, env.app)
        assert e.value.status == phos.E_OVERFLOW
        # limits, checked before any device work
        with pytest.raises(phos.PhosError) as e:
            phos.phos_validate_noalloc(env.ctx, s, rec, n, 3, out, (1 << 17) + 1, cnt, env.app)
        assert e.value.status == phos.E_INVAL
        # far more records than 4,096 tiles of any size hold (rejected on the
        # host; the kernel never sees the count, which the buffer could not
        # back)
        with pytest.raises(phos.PhosError) as e:
            phos.phos_validate_noalloc(env.ctx, s, rec, 1 << 40, 3, out, 10, cnt, env.app)
        assert e.value.status == phos.E_INVAL
        env.app.synchronize()
    finally:
        phos.phos_spec_release(env.ctx, s)
