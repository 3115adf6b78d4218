"""Full-size parity in the launch configuration bench.py times: the training
step (16 GiB pool of 2,000 buffers, 64 KiB pages, 1,000 launches x 10^6
accesses validated with tracking in one batched call, copy-on-write before
every launch, a copy-on-write and a recopy checkpoint open together on one
copy stream, pre-copy rounds of the pages whose last write has been issued
before launches 400, 650, 850, 950 and 990, recopy at the end).

Compared against what the oracle computes at this size: the dirty and victim
page maps of all 1,000 launches (Section 4.3), the violation lists of sampled
launches (Section 4.1), and both images against snapshots of the pool taken
at the step start (t1, Section 4.2) and after the last launch (t2,
Section 4.3)."""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_harness import final_rounds_expected

pytestmark = pytest.mark.gpu
N_LAUNCH, N_REC = 1000, 1_000_000
SAMPLED = (0, 1, 357, 998, 999)
# the final-page pre-copy rounds of the timed step (bench.py's default)
FINAL_AT = (400, 650, 850, 950, 990)


def _snapshot_device(torch, pool, w):
    """The image a stop-the-world checkpoint would write: the buffers back to
    back, copied on the device (the oracle's snapshot, at 16 GiB)."""
    img = torch.empty(int(w.alloc_bytes.sum()), dtype=torch.uint8, device="cuda")
    o = 0
    for off, nb in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
        img[o:o + nb].copy_(pool[off:off + nb])
        o += nb
    return img


def _oracle_maps(w, launches, base):
    """Dirty and victim pages of every launch, by the oracle, on host threads,
    and per page the last launch with a failing write inside a buffer there
    (-1: none)."""
    hw = synth.HostWorld(w, base)
    table = oracle.Table.from_world(w, base)
    npg = w.n_pages

    def part(js):
        d, v = np.zeros(npg, np.uint8), np.zeros(npg, np.uint8)
        last = np.full(npg, -1, np.int64)
        for j in js:
            L = launches[j]
            rec = synth.records_host(hw, L)
            vj = np.zeros(npg, np.uint8)
            oracle.track(oracle.spec_build(table, L.arg_values(base)), rec, table, base,
                         w.page_bytes, npg, d, vj)
            v |= vj
            last[vj != 0] = j
        return d, v, last

    parts = [list(range(len(launches)))[i::8] for i in range(8)]
    dirty, victim = np.zeros(npg, np.uint8), np.zeros(npg, np.uint8)
    last = np.full(npg, -1, np.int64)
    with cf.ThreadPoolExecutor(8) as ex:
        for d, v, lp in ex.map(part, parts):
            dirty |= d
            victim |= v
            last = np.maximum(last, lp)
    return dirty, victim, last


def test_training_step_full_size():
    import torch
    from paper_2405_12079_amd import phos

    w = synth.config2_world()
    launches = synth.config2_launches(w, N_LAUNCH, N_REC)
    page = w.page_bytes
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + w.pool_bytes]
    synth.content_device(pool, w.seed)
    recs = torch.empty(N_LAUNCH * N_REC, dtype=torch.int64, device="cuda")
    dw = synth.DeviceWorld(w, base)
    for g in range(0, N_LAUNCH, 100):
        synth.records_device(dw, launches[g:g + 100], N_REC,
                             out=recs[g * N_REC:(g + 100) * N_REC])
    torch.cuda.synchronize()
    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    try:
        phos.phos_buffers_register(ctx, w.buffers(base))
        nimg = phos.phos_image_bytes(ctx)
        specs = [phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches]
        ptrs = [recs.data_ptr() + j * N_REC * 8 for j in range(N_LAUNCH)]
        want_a = _snapshot_device(torch, pool, w)  # t1
        img_a = torch.empty(nimg, dtype=torch.uint8, device="cuda")
        img_b = torch.empty(nimg, dtype=torch.uint8, device="cuda")
        cap = 2_000_000
        vout = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
        vcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        app, cpy = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        ca = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_a, None, cpy)
        cb = phos.phos_ckpt_begin(ctx, phos.RECOPY, 0, img_b, None, cpy)
        phos.phos_validate_batch(ctx, specs, ptrs, [N_REC] * N_LAUNCH,
                                 phos.V_READS | phos.V_WRITES | phos.V_TRACK, vout, cap,
                                 vcnt.data_ptr(), app)
        for j, L in enumerate(launches):
            if j in FINAL_AT:  # every launch was validated up front
                phos.phos_ckpt_precopy_final(cb, specs[j:], N_LAUNCH - j, app)
            phos.phos_ckpt_cow(ca, specs[j], app)
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, ptrs[j], N_REC, app)
        phos.phos_ckpt_recopy(cb, app)
        dirty_gpu = phos.phos_track_read(ctx, 0, w.n_pages)
        victim_gpu = phos.phos_track_read(ctx, 1, w.n_pages)
        sa = phos.phos_ckpt_end(ca, app)
        sb = phos.phos_ckpt_end(cb, app)
        torch.cuda.synchronize()
        want_b = _snapshot_device(torch, pool, w)  # t2
        assert torch.equal(img_a, want_a), "copy-on-write image != pool at t1"
        assert torch.equal(img_b, want_b), "recopy image != pool at t2"
        n_img_pages = nimg // page
        assert sa.bg_pages + sa.cow_pages == n_img_pages
        assert n_img_pages - sb.recopy_pages - sb.precopy_pages <= sb.bg_pages <= n_img_pages
        del want_a, want_b, img_a, img_b

        # write-set tracking of all 1,000 launches against the oracle, and the
        # pages the pre-copy rounds took (their last write issued before the
        # round)
        dirty, victim, last = _oracle_maps(w, launches, base)
        table = oracle.Table.from_world(w, base)

        def upcoming(r):
            m = np.zeros(w.n_pages, np.uint8)
            for L in launches[r:]:
                for iv in oracle.spec_build(table, L.arg_values(base)):
                    lo = max(int(iv["lo"]), base) - base
                    hi = min(int(iv["hi"]), base + w.pool_bytes) - base
                    if int(iv["mode"]) & 2 and hi > lo:
                        m[lo // page:(hi - 1) // page + 1] = 1
            return m

        inbuf = np.zeros(w.n_pages, np.uint8)
        for off, nb in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
            inbuf[off // page:(off + nb) // page] = 1
        dirty_left, victim_left, pre = final_rounds_expected(dirty, victim, last, FINAL_AT,
                                                             upcoming, inbuf)
        assert np.array_equal(dirty_gpu, oracle.pages_to_bitmap(dirty_left.astype(np.uint8),
                                                                w.n_pages))
        assert np.array_equal(victim_gpu, oracle.pages_to_bitmap(victim_left.astype(np.uint8),
                                                                 w.n_pages))
        assert sb.recopy_pages == int(((dirty_left | victim_left) & inbuf.astype(bool)).sum())
        assert sb.precopy_pages == pre

        # violation lists of sampled launches against the oracle
        nv = int(vcnt.item())
        assert nv <= cap
        got = vout[:nv * 32].cpu().numpy().view(phos.VIOLATION_DTYPE)
        hw = synth.HostWorld(w, base)
        table = oracle.Table.from_world(w, base)
        for j in SAMPLED:
            L = launches[j]
            want = oracle.validate(oracle.spec_build(table, L.arg_values(base)),
                                   synth.records_host(hw, L), table, L.k)
            mine = got[got["launch_id"] == L.k]
            for f in ("index", "addr", "is_write", "reason", "victim"):
                assert np.array_equal(mine[f], want[f]), f"launch {j}: field {f}"
        # the list is ordered by (position in the call, record index)
        pos = np.searchsorted(np.array([L.k for L in launches]), got["launch_id"])
        key = pos.astype(np.uint64) * np.uint64(1 << 32) + got["index"].astype(np.uint64)
        assert np.all(np.diff(key.astype(np.int64)) > 0)
    finally:
        phos.phos_destroy(ctx)
