"""GPU parity of the serving loop (no paper analog): a short Poisson trace of
checkpoint, restore and fault-burst requests is served by the plain FIFO path
(each request alone) and by continuous batching (requests in the mix); every
request's destination bytes are equal in both runs and equal to what the
oracle says the request must produce.  Latency and throughput are measured by
bench.py, not checked here (parity unpinned for them)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
PAGE = 64 * 1024
SEED = 0x5E12E


def _expected(q, src_h, page):
    """What request q must leave in its destination (zeroed beforehand)."""
    want = np.zeros(q.size, np.uint8)
    img = src_h[q.src_off:q.src_off + q.size]
    if q.type == synth.REQ_RESTORE:
        want[:] = img
    elif q.type == synth.REQ_CKPT:
        st, ln = q.runs
        oracle.gather(img, want, st.astype(np.uint64) * page, st.astype(np.uint64) * page,
                      ln.astype(np.uint64) * page)
    else:
        w = synth.burst_world(q, page)
        L = synth.burst_launch(q, w)
        rec = synth.records_host(synth.HostWorld(w, 0), L)
        npg = q.size // page
        touched = np.zeros(npg, np.uint8)
        # the pages a burst touches inside its buffers, minus those already present
        oracle.touched_pages(rec, oracle.Table.from_world(w, 0), 0, page, npg, touched)
        need = touched & (1 - synth.present_host(SEED, q.r, npg))
        for p in np.flatnonzero(need):
            want[p * page:(p + 1) * page] = img[p * page:(p + 1) * page]
    return want


def test_serving_alone_equals_mix_equals_oracle():
    import torch
    import bench
    from paper_2405_12079_amd import phos

    arena = 256 << 20
    trace = synth.serving_trace(SEED, 2000.0, 0.06, 1 << 20, 16 << 20, PAGE, arena,
                                burst_records=8192)
    kinds = {q.type for q in trace}
    assert kinds == {0, 1, 2} and len(trace) > 60
    src = torch.empty(arena, dtype=torch.uint8, device="cuda")
    synth.content_device(src, SEED)
    budget = sum(q.size for q in trace)
    dst = torch.zeros(budget, dtype=torch.uint8, device="cuda")
    reqs, keep, bursts = bench.serving_inputs(torch, phos, synth, trace, PAGE, src.data_ptr(), SEED)
    src_h = src.cpu().numpy()
    results = {}
    # plain; batched shortest-remaining-first; batched small-first then arrival order
    runs = ((phos.SERVE_PLAIN, 0), (phos.SERVE_BATCHED, 2**64 - 1), (phos.SERVE_BATCHED, 8 << 20))
    for mode, small in runs:
        dst.zero_()
        bench.reseed_bursts(torch, synth, bursts, SEED)
        cfg = phos.phos_serve_cfg(mode, PAGE, budget, dst.data_ptr(), 4 << 20, 16 << 20,
                                  phos.phos_batch_cfg(256 << 10, 2, 512), 1, 0, small)
        outs, st = phos.phos_serve_run(0, cfg, reqs, len(trace))
        assert st.max_active >= 1 and all(o.latency_ms >= 0 for o in outs[:len(trace)])
        host = dst.cpu().numpy()
        results[(mode, small)] = [host[o.dst_off:o.dst_off + q.size].copy()
                                  for o, q in zip(outs[:len(trace)], trace)]
        if mode == phos.SERVE_BATCHED:
            assert st.iterations >= 1
    for j, q in enumerate(trace):
        want = _expected(q, src_h, PAGE)
        for key in runs:
            where = "alone" if key[0] == phos.SERVE_PLAIN else f"in the mix (small_bytes {key[1]})"
            assert np.array_equal(results[key][j], want), f"request {j} {where}"
    del keep


def test_serving_rejects_oversized_request():
    import torch
    from paper_2405_12079_amd import phos
    dst = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    arr = (phos.phos_serve_req * 1)()
    arr[0].arrival_s, arr[0].type, arr[0].bytes, arr[0].nseg = 0.0, 1, 4 << 20, 0
    cfg = phos.phos_serve_cfg(phos.SERVE_BATCHED, PAGE, 1 << 20, dst.data_ptr(), 1 << 20, 1 << 20,
                              phos.phos_batch_cfg(1 << 20, 2, 512), 0, 0)
    with pytest.raises(phos.PhosError) as e:
        phos.phos_serve_run(0, cfg, arr, 1)
    assert e.value.status == phos.E_INVAL
