"""GPU parity of the batched copy (no paper analog): many requests' dirty runs
copied into compact deltas by one persistent graph-captured launch, by the
plain per-request launches, and by the oracle's gather — byte for byte; the
graph is replayed several times with other work in between."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
PAGE = 64 * 1024


@pytest.fixture(scope="module")
def work():
    import torch
    reqs = synth.batch_requests(0xBA7C, 12, 4 << 20, 96 << 20, PAGE)
    src_bytes = sum(q.pages for q in reqs) * PAGE
    dst_bytes = sum(q.dirty_pages for q in reqs) * PAGE
    src = torch.empty(src_bytes, dtype=torch.uint8, device="cuda")
    synth.content_device(src, 0xBA7C)
    torch.cuda.synchronize()
    segs = synth.request_segments(reqs, src.data_ptr(), 0, PAGE)
    # expected deltas from the oracle's gather over the host copy of the sources
    src_h = synth.content_host(0xBA7C, 0, src_bytes)
    want = np.zeros(dst_bytes, np.uint8)
    oracle.gather(src_h, want, segs["src"] - np.uint64(src.data_ptr()), segs["dst"], segs["bytes"])
    return reqs, src, dst_bytes, want


def _segs_for(reqs, src, dst):
    return synth.request_segments(reqs, src.data_ptr(), dst.data_ptr(), PAGE)


@pytest.mark.parametrize("cfg", [(64 << 10, 1, 256), (1 << 20, 2, 512), (4 << 20, 8, 1024)])
def test_batched_graph_copy_matches_oracle(work, cfg):
    import torch
    from paper_2405_12079_amd import phos
    reqs, src, dst_bytes, want = work
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    segs = _segs_for(reqs, src, dst)
    c = phos.phos_batch_cfg(*cfg)
    b = phos.phos_batch_create(0, len(segs), len(reqs), c)
    s = torch.cuda.Stream()
    try:
        phos.phos_batch_load(b, segs, s)
        for rep in range(3):
            dst.zero_()
            torch.cuda.synchronize()
            phos.phos_batch_run(b, s)
            s.synchronize()
            assert np.array_equal(dst.cpu().numpy(), want), f"replay {rep}"
            ptr = phos.phos_batch_done_bytes(b)
            got = np.frombuffer(bytes(_read_device(ptr, 8 * len(reqs))), dtype=np.uint64)
            assert got.tolist() == [q.dirty_pages * PAGE for q in reqs]
            times = phos.phos_batch_times(b, len(reqs))
            assert (times > 0).all() and times.max() < 10_000.0
    finally:
        phos.phos_batch_destroy(b)


def _read_device(ptr, nbytes):
    import ctypes
    import torch
    out = torch.empty(nbytes, dtype=torch.uint8)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(out.data_ptr(), ptr, nbytes, 2) == 0  # device to host
    return out.numpy().tobytes()


def test_plain_per_request_matches_oracle(work):
    import torch
    from paper_2405_12079_amd import phos
    reqs, src, dst_bytes, want = work
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    lists = [phos.phos_seglist_create(0, _segs_for([q], src, dst)) for q in reqs]
    try:
        for l in lists:
            phos.phos_copy_plain(l, 1 << 20, 512, s)
        s.synchronize()
        assert np.array_equal(dst.cpu().numpy(), want)
    finally:
        for l in lists:
            phos.phos_seglist_destroy(l)


def test_alone_equals_in_the_mix(work):
    """Each request copied alone (its own batch) equals its bytes in the mix."""
    import torch
    from paper_2405_12079_amd import phos
    reqs, src, dst_bytes, want = work
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    b = phos.phos_batch_create(0, sum(q.dirty_start.size for q in reqs), len(reqs))
    s = torch.cuda.Stream()
    try:
        for q in reqs[:4]:
            dst.zero_()
            torch.cuda.synchronize()
            phos.phos_batch_copy(b, _segs_for([q], src, dst), s)
            s.synchronize()
            lo, hi = q.dst_off, q.dst_off + q.dirty_pages * PAGE
            got = dst.cpu().numpy()
            assert np.array_equal(got[lo:hi], want[lo:hi])
            assert not got[:lo].any() and not got[hi:].any()
    finally:
        phos.phos_batch_destroy(b)


def test_autotuner_picks_a_valid_config_and_caches(work, tmp_path):
    import torch
    from paper_2405_12079_amd import phos
    reqs, src, dst_bytes, _ = work
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    segs = _segs_for(reqs[:4], src, dst)
    cache = str(tmp_path / "tune.txt")
    best, ms = phos.phos_batch_tune(0, segs, cache)
    assert best.chunk_bytes in [64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20]
    assert best.wg_per_cu in (1, 2, 4, 8) and best.threads in (256, 512, 1024) and ms > 0
    assert os.path.exists(cache)
    best2, ms2 = phos.phos_batch_tune(0, segs, cache)
    assert (best2.chunk_bytes, best2.wg_per_cu, best2.threads) == \
        (best.chunk_bytes, best.wg_per_cu, best.threads) and ms2 == pytest.approx(ms, rel=1e-5)


def test_batch_rejects_misaligned_segments(work):
    from paper_2405_12079_amd import phos
    reqs, src, _, _ = work
    b = phos.phos_batch_create(0, 4, 2)
    try:
        bad = np.zeros(1, dtype=phos.SEG_DTYPE)
        bad[0] = (src.data_ptr() + 8, src.data_ptr(), 64, 0, 0)
        with pytest.raises(phos.PhosError) as e:
            phos.phos_batch_load(b, bad)
        assert e.value.status == phos.E_INVAL
        bad[0] = (src.data_ptr(), src.data_ptr() + 4096, 64, 5, 0)  # request id >= max_reqs
        with pytest.raises(phos.PhosError):
            phos.phos_batch_load(b, bad)
    finally:
        phos.phos_batch_destroy(b)


def _small_ctx(torch, phos):
    """A context for the device-segment batch calls (their pool is not used)."""
    back = torch.empty(2 * PAGE, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + PAGE - 1) // PAGE * PAGE
    return back, phos.phos_create(0, base, PAGE, PAGE)


@pytest.mark.parametrize("tuned", [False, True])
def test_copy_batch_device_segments_match_oracle(work, tuned):
    """phos_copy_batch / phos_copy_batch_tuned with the segments in device
    memory: the deltas equal the oracle's gather on three calls in a row (the
    tuned one replays its graph after the first); a malformed segment makes a
    call copy nothing and phos_stream_status report E_INVAL, once."""
    import torch
    from paper_2405_12079_amd import phos
    reqs, src, dst_bytes, want = work
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    segs = _segs_for(reqs, src, dst)
    d_segs = torch.from_numpy(segs.view(np.uint8).copy()).cuda()
    back, ctx = _small_ctx(torch, phos)
    s = torch.cuda.Stream()
    call = phos.phos_copy_batch_tuned if tuned else phos.phos_copy_batch
    try:
        for rep in range(3):
            dst.zero_()
            torch.cuda.synchronize()
            call(ctx, d_segs, len(segs), s)
            s.synchronize()
            assert np.array_equal(dst.cpu().numpy(), want), f"call {rep}"
            phos.phos_stream_status(ctx, s)
        bad = segs.copy()
        bad["bytes"][len(bad) // 2] += np.uint64(8)
        d_bad = torch.from_numpy(bad.view(np.uint8).copy()).cuda()
        dst.zero_()
        torch.cuda.synchronize()
        if tuned:  # the first call for these segments checks them on the host
            with pytest.raises(phos.PhosError) as e:
                call(ctx, d_bad, len(bad), s)
            assert e.value.status == phos.E_INVAL
        else:
            call(ctx, d_bad, len(bad), s)
            with pytest.raises(phos.PhosError) as e:
                phos.phos_stream_status(ctx, s)
            assert e.value.status == phos.E_INVAL
        phos.phos_stream_status(ctx, s)  # reported once
        assert int(dst.count_nonzero().item()) == 0
        call(ctx, d_segs, 0, s)  # nothing to copy
    finally:
        torch.cuda.synchronize()
        phos.phos_destroy(ctx)
