"""Benchmark of the validated-speculation checkpoint hot path on one MI355X.

Default workload — the training-step configuration: a 16 GiB pool of 2,000
buffers (12 layers of bf16 4096x4096 / 4096x14336 weights with fp32 Adam
moments, 80 activations, 1,848 small buffers), 64 KiB pages, and a step of
1,000 launches x 1,000,000 accesses (1e9 validated addresses).  One step:

  * open a soft copy-on-write checkpoint (image A, frozen at the step start)
    and a soft recopy checkpoint (image B, taken at the step end), both with
    their background copies on one copy stream;
  * validate the launches' access streams (with dirty / victim tracking) in
    batched calls, then for every launch: copy-on-write of the pages it may
    write, then the application's launch itself (its writes);
  * re-quiesce, recopy the dirty and victim pages into B, close both.

The JSON line's value is the step's snapshot rate: bytes of the two finished
checkpoint images per second of step time (inputs resident in HBM); the bytes
actually copied into them (a page may be copied twice) are reported beside.
The roofline object covers the dominant kernel (the background copy);
`cpu_baseline` times the CPU oracle on a bounded sample of the same step.

Other workloads: --config 3 batched uneven checkpoints, 4 serving loop,
5 cold-start restore, 6 twin-kernel validator overhead, 7 preemptible drain,
8 copy-on-write staging budget.

  python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--config 2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, GB/s


def host_cpu_share():
    """CPUs this process may use: (threads, detail).  The scheduler affinity
    bounds it, and a cgroup CPU quota (cpu.max: quota per period) bounds it
    further: threads beyond the quota would share the same CPU time, so the
    oracle would be timed on cores the job is not given."""
    affinity = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) // int(period)))
    except (OSError, ValueError):
        pass
    threads = max(1, min(affinity, quota) if quota else affinity)
    return threads, {"host_cpus": os.cpu_count(), "affinity_cpus": affinity,
                     "cgroup_cpu_quota": quota}


# Host threads for the oracle's parity replays and the CPU baseline.
HOST_THREADS, HOST_CPU_DETAIL = host_cpu_share()
# the device code's sources: a counter summary is valid for these bytes only
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2405_12079_amd", "csrc", f)
                  for f in ("kernels.hip", "internal.h")]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload, key="traffic_bytes_per_launch", cast=int):
    """HBM bytes per launch (or the summary's `key`) of `kernel` on `workload`
    from the committed rocprofv3 counter summary
    (profiles/<kernel>_<workload>_pmc.txt), or None when there is none or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256() or key not in fields:
        return None
    return cast(float(fields[key]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Timer:
    """HIP event pair on a given stream; elapsed ms after synchronization."""

    def __init__(self, torch, stream):
        self.s = stream
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.e0.record(self.s)

    def stop(self):
        self.e1.record(self.s)

    def ms(self):
        return self.e0.elapsed_time(self.e1)


class HipGraph:
    """Stream capture of a launch-bound loop into a HIP graph (ctypes on the HIP
    runtime): captured once, replayed every step."""

    def __init__(self):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.graph = ctypes.c_void_p()
        self.exec = ctypes.c_void_p()

    def _ok(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what}: hipError {rc}")

    def capture(self, stream, fn):
        h = self.hip
        sp = self.ct.c_void_p(stream.cuda_stream)
        # relaxed capture mode (2): other streams keep running their copies
        self._ok(h.hipStreamBeginCapture(sp, 2), "hipStreamBeginCapture")
        try:
            fn()
        finally:
            self._ok(h.hipStreamEndCapture(sp, self.ct.byref(self.graph)), "hipStreamEndCapture")
        self._ok(h.hipGraphInstantiate(self.ct.byref(self.exec), self.graph, None, None, 0),
                 "hipGraphInstantiate")

    def launch(self, stream):
        self._ok(self.hip.hipGraphLaunch(self.exec, self.ct.c_void_p(stream.cuda_stream)),
                 "hipGraphLaunch")

    def close(self):
        if self.exec:
            self.hip.hipGraphExecDestroy(self.exec)
        if self.graph:
            self.hip.hipGraphDestroy(self.graph)


def copy_samples(torch, phos, nbytes=4 << 30, reps=5):
    """Sample HBM copy rates on this GPU, for context (not ceilings: a tuned
    kernel can beat them): the runtime's device-to-device copy and one
    contiguous segment through the persistent batch kernel (GB/s of HBM
    traffic = 2 x bytes copied / time)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(7)
    s = torch.cuda.Stream()
    t = Timer(torch, s)
    out = {}
    with torch.cuda.stream(s):
        ts = []
        for _ in range(reps):
            t.start()
            dst.copy_(src)
            t.stop()
            s.synchronize()
            ts.append(t.ms())
    out["runtime_d2d_GBps"] = round(2 * nbytes / (np.median(ts[1:]) / 1e3) / 1e9, 1)
    seg = np.zeros(1, dtype=phos.SEG_DTYPE)
    seg[0] = (src.data_ptr(), dst.data_ptr(), nbytes, 0, 0)
    b = phos.phos_batch_create(0, 1, 1)
    phos.phos_batch_load(b, seg, s)
    ts = []
    for _ in range(reps):
        t.start()
        phos.phos_batch_run(b, s)
        t.stop()
        s.synchronize()
        ts.append(t.ms())
    phos.phos_batch_destroy(b)
    out["batch_kernel_contiguous_GBps"] = round(2 * nbytes / (np.median(ts[1:]) / 1e3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


_pinned_keep = []


def pinned_tensor(torch, nbytes):
    """Exactly nbytes of pinned host memory (hipHostMalloc), as a CPU uint8 tensor
    (torch's pinned allocator rounds sizes up to a power of two)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    p = ctypes.c_void_p()
    rc = hip.hipHostMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes), 0)
    if rc != 0:
        hip.hipGetLastError()  # do not leave the error for the next HIP call to report
        raise RuntimeError(f"hipHostMalloc({nbytes}) failed: {rc}")
    arr = np.ctypeslib.as_array((ctypes.c_uint8 * nbytes).from_address(p.value))
    _pinned_keep.append(p)
    return torch.from_numpy(arr)


def release_pinned(torch):
    """Free every pinned_tensor allocation (the caller holds none of them any
    more, and no GPU work on them is pending)."""
    import ctypes
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    while _pinned_keep:
        hip.hipHostFree(_pinned_keep.pop())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- config 2
def run_training_step(args):
    import torch

    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    w = synth.config2_world()
    n_launch, n_rec = args.launches, 1_000_000
    launches = synth.config2_launches(w, n_launch, n_rec)
    page = w.page_bytes
    log(f"[bench] training-step: {w.n_alloc} buffers, {w.image_bytes / 2**30:.2f} GiB image, "
        f"{n_launch} launches x {n_rec} accesses")
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + w.pool_bytes]
    synth.content_device(pool, w.seed)
    dw = synth.DeviceWorld(w, base)
    recs = torch.empty(n_launch * n_rec, dtype=torch.int64, device="cuda")
    for g in range(0, n_launch, 100):
        synth.records_device(dw, launches[g:g + 100], n_rec, out=recs[g * n_rec:(g + 100) * n_rec])
    torch.cuda.synchronize()
    log("[bench] inputs resident")

    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    phos.phos_buffers_register(ctx, w.buffers(base))
    nimg = phos.phos_image_bytes(ctx)
    img_a = torch.empty(nimg, dtype=torch.uint8, device="cuda")
    img_b = torch.empty(nimg, dtype=torch.uint8, device="cuda")
    specs = np.array([phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches],
                     np.uint32)
    rec_list = [recs.data_ptr() + j * n_rec * 8 for j in range(n_launch)]
    rec_ptrs = np.array(rec_list, np.uint64)
    n_recs = np.full(n_launch, n_rec, np.uint64)
    cap = 4_000_000
    vout = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    vcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    chunk = max(1, args.val_chunk)
    nchunk = (n_launch + chunk - 1) // chunk
    lcap = 2_000_000  # per-call violation capacity (the list is reused call to call)
    lcnt = torch.zeros(nchunk, dtype=torch.int64, device="cuda")
    app, cpy = torch.cuda.Stream(), torch.cuda.Stream()
    VFLAGS = phos.V_READS | phos.V_WRITES | phos.V_TRACK

    # the background passes run on the library's own stream: their GPU time
    # comes back in the checkpoints' stats (bg_ms, HIP events on that stream)
    t_val, t_app = Timer(torch, app), Timer(torch, app)
    t_rec = Timer(torch, cpy)
    graph = None

    pair = not args.separate_passes

    def start_copies(ca, cb):
        # the background copies start once the first validation pass is done:
        # they then share HBM with the latency-bound launches, not with it
        cpy.wait_stream(app)
        if pair:  # one pass reads each page once for both images
            phos.phos_ckpt_start_pair(ca, cb, None)
            return
        phos.phos_ckpt_start(ca, None)
        phos.phos_ckpt_start(cb, None)

    final_at = {int(x) for x in args.final_at.split(",") if x.strip()}
    vstream = torch.cuda.Stream() if args.pipelined_validation else None
    vdone = [torch.cuda.Event() for _ in range(nchunk)] if vstream is not None else []

    def app_loop_pipelined(ca, cb):
        # every chunk's validation is issued on its own stream up front; the
        # launches of chunk c wait only for chunk c's pass, so the passes run
        # beside the (latency-bound) launches of earlier chunks
        vstream.wait_stream(app)
        for c in range(nchunk):
            sl = slice(c * chunk, min((c + 1) * chunk, n_launch))
            phos.phos_validate_batch(ctx, specs[sl], rec_ptrs[sl], n_recs[sl],
                                     VFLAGS, vout, lcap, lcnt.data_ptr() + 8 * c, vstream)
            vdone[c].record(vstream)
        for j, L in enumerate(launches):
            if j % chunk == 0:
                app.wait_event(vdone[j // chunk])
            phos.phos_ckpt_cow(ca, specs[j], app)
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_list[j], n_rec, app)

    e_first = torch.cuda.Event(enable_timing=True)  # launch 0 may start
    e_val = torch.cuda.Event(enable_timing=True)  # the step's first validation call has ended

    def app_loop(ca, cb):
        if vstream is not None:
            return app_loop_pipelined(ca, cb)
        for j, L in enumerate(launches):
            if j % chunk == 0:  # validate the next `chunk` launches' access streams
                c = j // chunk
                if args.precopy and j:  # every launch validated so far has been enqueued
                    phos.phos_ckpt_precopy(cb, app)
                sl = slice(j, min(j + chunk, n_launch))
                phos.phos_validate_batch(ctx, specs[sl], rec_ptrs[sl], n_recs[sl],
                                         VFLAGS, vout, lcap, lcnt.data_ptr() + 8 * c, app)
                if j == 0:
                    e_val.record(app)
                if j == 0 and args.copy_start == "validation":
                    start_copies(ca, cb)
            if j in final_at:  # pages no remaining launch may write
                ahead = min((j // chunk + 1) * chunk, n_launch) - j  # validated, still to come
                phos.phos_ckpt_precopy_final(cb, specs[j:], ahead, app)
            phos.phos_ckpt_cow(ca, specs[j], app)
            if j == 0:
                e_first.record(app)
                if args.copy_start == "cow":
                    start_copies(ca, cb)
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_list[j], n_rec, app)

    warm = False

    def step():
        nonlocal graph, warm
        if args.copy_start != "begin":
            ca = phos.phos_ckpt_begin(ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, img_a, None, cpy)
            cb = phos.phos_ckpt_begin(ctx, phos.RECOPY, phos.CKPT_DEFER_BACKGROUND, img_b, None, cpy)
        elif pair:
            ca = phos.phos_ckpt_begin(ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, img_a, None, cpy)
            cb = phos.phos_ckpt_begin(ctx, phos.RECOPY, phos.CKPT_DEFER_BACKGROUND, img_b, None, cpy)
            phos.phos_ckpt_start_pair(ca, cb, None)
        else:
            ca = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_a, None, cpy)
            cb = phos.phos_ckpt_begin(ctx, phos.RECOPY, 0, img_b, None, cpy)
        t_app.start()
        if args.app_graph and warm:
            if graph is None:
                graph = HipGraph()
                graph.capture(app, lambda: app_loop(ca, cb))
            graph.launch(app)
        else:
            app_loop(ca, cb)
        t_app.stop()
        t_rec.e0.record(app)  # from the application's last launch to the recopy's end
        phos.phos_ckpt_recopy(cb, app)
        t_rec.stop()
        sa = phos.phos_ckpt_end(ca, app)
        sb = phos.phos_ckpt_end(cb, app)
        warm = True  # later steps replay the captured loop
        return sa, sb

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i} done")
    torch.cuda.synchronize()
    rows = []
    step_s = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts0 = time.perf_counter()
        sa, sb = step()  # ends with both checkpoints finished (synchronous)
        step_s.append(time.perf_counter() - ts0)
        stall = t_app.e0.elapsed_time(e_first) if not (args.app_graph or vstream) else float("nan")
        val = t_app.e0.elapsed_time(e_val) if not (args.app_graph or vstream) else float("nan")
        rows.append(dict(bg_a=sa.bg_ms, bg_b=sb.bg_ms if not pair else 0.0, app=t_app.ms(),
                         rec=t_rec.ms(), stall_t1=stall, val_in_step=val, bg_a_pages=sa.bg_pages,
                         cow_pages=sa.cow_pages,
                         bg_b_pages=sb.bg_pages, bg_read_pages=sa.bg_read_pages + sb.bg_read_pages,
                         recopy_pages=sb.recopy_pages,
                         precopy_pages=sb.precopy_pages))
        log(f"[bench] step {i}: " + ", ".join(f"{k}={v:.3f}" if isinstance(v, float) else f"{k}={v}"
                                             for k, v in rows[-1].items()))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1000.0 / args.steps
    nviol = int(lcnt.sum().item())

    # Validation alone (no concurrent copies), with and without dirty
    # tracking: four calls back to back between two events on the stream, so
    # each call's host preparation overlaps the previous pass on the GPU
    # (what a pass costs in a pipeline); and one call timed alone, host
    # preparation included (its latency).
    alone, alone_call = {}, {}
    for name, fl in (("track", VFLAGS), ("plain", phos.V_READS | phos.V_WRITES)):
        tv = Timer(torch, app)
        phos.phos_validate_batch(ctx, specs, rec_ptrs, n_recs, fl, vout, cap, vcnt, app)
        app.synchronize()
        ts, tc = [], []
        for _ in range(3):
            tv.start()
            for _ in range(4):
                phos.phos_validate_batch(ctx, specs, rec_ptrs, n_recs, fl, vout, cap, vcnt, app)
            tv.stop()
            app.synchronize()
            ts.append(tv.ms() / 4)
            tv.start()
            phos.phos_validate_batch(ctx, specs, rec_ptrs, n_recs, fl, vout, cap, vcnt, app)
            tv.stop()
            app.synchronize()
            tc.append(tv.ms())
        alone[name] = float(np.median(ts))
        alone_call[name] = float(np.median(tc))
    log(f"[bench] validation alone: track {alone['track']:.3f} ms, plain {alone['plain']:.3f} ms")
    # the background copy with nothing beside it, and the application's own
    # launches with no checkpoint open (what the step would cost without C/R)
    ts = []
    for _ in range(3):
        ca = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_a, None, cpy)
        ts.append(phos.phos_ckpt_end(ca, cpy).bg_ms)
    bg_alone_ms = float(np.median(ts))
    # the shared pass with nothing beside it (both images, every page)
    ts, hbm = [], []
    for _ in range(3):
        ca = phos.phos_ckpt_begin(ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, img_a, None, cpy)
        cb = phos.phos_ckpt_begin(ctx, phos.RECOPY, phos.CKPT_DEFER_BACKGROUND, img_b, None, cpy)
        phos.phos_ckpt_start_pair(ca, cb, None)
        sa = phos.phos_ckpt_end(ca, cpy)
        sb = phos.phos_ckpt_end(cb, cpy)
        ts.append(sa.bg_ms)
        hbm.append((sa.bg_read_pages + sa.bg_pages + sb.bg_pages) * page)
    pair_ms = float(np.median(ts))
    pair_alone = {"bound": "hbm", "kernel": "background_pair_kernel, nothing beside it",
                  "achieved": round(float(np.median(hbm)) / pair_ms / 1e6, 1),
                  "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                  "frac": round(float(np.median(hbm)) / pair_ms / 1e6 / HBM_PEAK_GBPS, 4),
                  "avg_launch_ms": round(pair_ms, 4)}
    log(f"[bench] shared background pass alone {pair_ms:.3f} ms ({pair_alone['achieved']} GB/s)")
    ts = []
    for _ in range(2):
        t_app.start()
        for j, L in enumerate(launches):
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_list[j], n_rec, app)
        t_app.stop()
        app.synchronize()
        ts.append(t_app.ms())
    app_alone_ms = float(np.median(ts))
    log(f"[bench] background copy alone {bg_alone_ms:.3f} ms; application launches alone "
        f"{app_alone_ms:.3f} ms")
    # The stop-the-world step the method replaces, in the same run: the
    # application stops while image A is copied (the library's background
    # copy with nothing beside it, its fastest whole-image copy), runs its
    # launches (no checkpoint open, so no validation), and stops again while
    # image B is copied.  Each part is timed with HIP events (the copies on
    # the library's stream, the launches on the application's); the sum
    # leaves out the host's gaps between them.
    stw = []
    t_launch = Timer(torch, app)
    for _ in range(3):
        torch.cuda.synchronize()
        ck = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_a, None, cpy)
        copy_a = phos.phos_ckpt_end(ck, cpy).bg_ms
        app.wait_stream(cpy)
        t_launch.start()
        for j, L in enumerate(launches):
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_list[j], n_rec, app)
        t_launch.stop()
        cpy.wait_stream(app)
        ck = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_b, None, cpy)
        copy_b = phos.phos_ckpt_end(ck, cpy).bg_ms
        torch.cuda.synchronize()
        stw.append([copy_a, t_launch.ms(), copy_b])
    stw_parts = np.median(np.array(stw), axis=0)
    stw_ms = float(np.median([sum(x) for x in stw]))
    log(f"[bench] stop-the-world step {stw_ms:.3f} ms (copy A {stw_parts[0]:.3f}, launches "
        f"{stw_parts[1]:.3f}, copy B {stw_parts[2]:.3f})")
    # the Section 5 drain of a finished image to pinned host memory (PCIe)
    host_img = pinned_tensor(torch, nimg)
    ca = phos.phos_ckpt_begin(ctx, phos.COW, 0, img_a, host_img.data_ptr(), cpy)
    torch.cuda.synchronize()  # the background copy (on the library's stream) has finished
    t0d = time.perf_counter()
    phos.phos_ckpt_end(ca, cpy)
    d2h_s = time.perf_counter() - t0d
    log(f"[bench] D2H drain of the image: {nimg / d2h_s / 1e9:.1f} GB/s")
    roofs = copy_samples(torch, phos)
    log(f"[bench] contiguous copy samples: {roofs}")

    # checkpoint image bytes finished per step (two images), and the bytes
    # actually copied into them
    img_bytes = 2 * nimg
    rec_ms = float(np.mean([r["rec"] for r in rows]))
    rec_bytes = float(np.mean([r["recopy_pages"] for r in rows])) * page
    copied_bytes = np.mean([(r["bg_a_pages"] + r["cow_pages"] + r["bg_b_pages"] + r["recopy_pages"]
                             + r["precopy_pages"]) * page for r in rows])
    snap_gbps = img_bytes / (ms_step / 1e3) / 1e9
    # dominant kernel: the background copy of the copy-on-write image (every
    # page not taken by copy-on-write; 2 bytes of HBM traffic per byte), timed
    # with HIP events on the copy stream while the application runs beside it.
    # The recopy image's background copy is reported apart: how many pages it
    # skips depends on how far validation got, so its work varies by run.
    # With the shared pass (default) the dominant kernel is that one pass: one
    # read of each page it copies and one write per image it copies it into.
    bg_ms = float(np.mean([r["bg_a"] for r in rows]))
    if pair:
        bg_kernel = "background_pair_kernel"
        bg_hbm = float(np.mean([r["bg_read_pages"] + r["bg_a_pages"] + r["bg_b_pages"]
                                for r in rows])) * page
    else:
        bg_kernel = "background_kernel"
        bg_hbm = 2 * float(np.mean([r["bg_a_pages"] for r in rows])) * page
    bg_gbps = bg_hbm / (bg_ms / 1e3) / 1e9
    bgb_ms = float(np.mean([r["bg_b"] for r in rows]))
    bgb_bytes = float(np.mean([r["bg_b_pages"] for r in rows])) * page
    n_addr = n_launch * n_rec
    log(f"[bench] step {ms_step:.2f} ms; snapshot {snap_gbps:.1f} GB/s; background copy "
        f"{bg_ms:.2f} ms = {bg_gbps:.0f} GB/s HBM; validated addr/s (batched pass alone) "
        f"{n_addr / (alone['track'] / 1e3):.3e}")

    result = {
        "metric": "snapshot GB/s (CoW + recopy images per step time) vs HBM peak; validated addr/s",
        "value": round(snap_gbps, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "step_ms": {q: round(float(np.percentile(step_s, p)) * 1e3, 3)
                    for q, p in (("p10", 10), ("median", 50), ("p90", 90))},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded layout, access streams and contents)",
        "config": {"workload": "training-step: 16 GiB pool, 2000 buffers, 64 KiB pages, "
                               f"{n_launch} launches x {n_rec} accesses, soft-CoW + recopy",
                   "image_bytes": int(nimg), "accesses_per_step": n_addr},
        "validated_addr_per_s": round(n_addr / (alone["track"] / 1e3), 1),
        "validation_ms_alone": {k: round(v, 4) for k, v in alone.items()},
        "validation_call_ms_alone": {k: round(v, 4) for k, v in alone_call.items()},
        # the step's own tracked validation call, from the step's start on the
        # application stream to the call's end (median over the timed steps)
        "validation_ms_in_step": round(float(np.nanmedian([r["val_in_step"] for r in rows])), 4)
        if rows and not np.isnan(rows[0]["val_in_step"]) else None,
        "app_loop_ms": round(float(np.mean([r["app"] for r in rows])), 3),
        "stop_the_world_step_ms": round(stw_ms, 3),
        "stop_the_world_parts_ms": {"copy_A": round(float(stw_parts[0]), 3),
                                    "launches": round(float(stw_parts[1]), 3),
                                    "copy_B": round(float(stw_parts[2]), 3)},
        # the application's stall where the checkpoint opens (t1): from the
        # step's start on the application stream to the moment launch 0 may
        # run (its accesses validated, its copy-on-write done); stop-the-world
        # stalls for the whole copy of image A
        "stall_t1_ms": {"concurrent": round(float(np.nanmedian([r["stall_t1"] for r in rows])), 3)
                        if rows and not np.isnan(rows[0]["stall_t1"]) else None,
                        "stop_the_world": round(float(stw_parts[0]), 3)},
        # downtime at the re-quiesce (t2): from the application's last launch
        # to the recopy's end; stop-the-world copies the whole image B there
        "downtime_t2_ms": {"concurrent": round(rec_ms, 3),
                           "stop_the_world": round(float(stw_parts[2]), 3)},
        "recopy_ms": round(rec_ms, 3),
        "recopy_pages": int(np.mean([r["recopy_pages"] for r in rows])),
        "precopy": {"rounds": ((nchunk - 1) if args.precopy else 0) + len(final_at),
                    "final_at": sorted(final_at),
                    "pages": int(np.mean([r["precopy_pages"] for r in rows]))},
        "app_loop_graph": bool(args.app_graph),
        "launches_per_validation_call": chunk,
        "copy_samples": dict(roofs, note="contiguous 4 GiB copies for context; not ceilings"),
        "violations_per_step": nviol,
        "image_bytes_per_step": int(img_bytes),
        "bytes_copied_into_images_per_step": int(copied_bytes),
        "background_passes": "shared (one pass, both images)" if pair else "one per image",
        "background_pages": {"copy_on_write_image": int(np.mean([r["bg_a_pages"] for r in rows])),
                             "recopy_image": int(np.mean([r["bg_b_pages"] for r in rows])),
                             "pool_pages_read": int(np.mean([r["bg_read_pages"] for r in rows]))},
        "roofline": {"bound": "hbm",
                     "kernel": (f"{bg_kernel} (both images)" if pair
                                else f"{bg_kernel} (copy-on-write image)"),
                     "achieved": round(bg_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(bg_gbps / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(bg_kernel, "training_step"),
                     # the counted launch copies a few hundred pages more or
                     # fewer than the mean here (the copy-on-write race)
                     "traffic_over_algorithmic": measured_traffic(
                         bg_kernel, "training_step", "traffic_over_algorithmic", float),
                     "algorithmic_bytes_per_launch": int(bg_hbm),
                     "avg_launch_ms": round(bg_ms, 4)},
        "roofline_background_alone": {"bound": "hbm", "kernel": "background_kernel, nothing beside it",
                                       "achieved": round(2 * nimg / bg_alone_ms / 1e6, 1),
                                       "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                       "frac": round(2 * nimg / bg_alone_ms / 1e6 / HBM_PEAK_GBPS, 4),
                                       "avg_launch_ms": round(bg_alone_ms, 4)},
        "application_alone_ms": round(app_alone_ms, 3),
        "roofline_background_pair_alone": pair_alone,
        "d2h_drain_GBps": round(nimg / d2h_s / 1e9, 2),
        "roofline_validate": {"bound": "hbm", "kernel": "validate_kernel (+scan, scatter), alone",
                              "achieved": round((8 * n_addr + 32 * nviol) / alone["track"] / 1e6, 1),
                              "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                              "frac": round((8 * n_addr + 32 * nviol) / alone["track"] / 1e6
                                            / HBM_PEAK_GBPS, 4),
                              "traffic": measured_traffic("validate_kernel", "training_step")},
        # the recopy at the re-quiesce: page list + gather, from the
        # application's last launch to the recopy's end
        # (no fraction of the roofline: a working set under 1 GiB partly sits
        # in the 256 MB last-level cache)
        "recopy_rate": {"kernel": "gather_pages_kernel (+ page list), recopy",
                        "achieved": round(2 * rec_bytes / rec_ms / 1e6, 1), "unit": "GB/s",
                        "working_set_bytes": int(2 * rec_bytes),
                        "traffic": measured_traffic("gather_pages_kernel", "training_step")},
    }
    if not pair:
        result["background_recopy_image"] = {"avg_launch_ms": round(bgb_ms, 4),
                                             "pages": int(bgb_bytes // page),
                                             "GBps_hbm": round(2 * bgb_bytes / bgb_ms / 1e6, 1)}
    if graph is not None:
        graph.close()
    phos.phos_destroy(ctx)
    del recs, img_a, img_b, back
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_training_step(w, launches, base, img_bytes, n_addr)
    return result


def config1_validation_rate(reps=5):
    """Validated addresses per second on the plain tiny workload (64 MiB pool
    of 256 buffers, 4 KiB pages, 100 launches x 10^6 accesses, tracked), one
    batched call over all launches, median of `reps` after one warm-up.  Its
    800 MB of records is under the 1 GiB floor for roofline claims."""
    import torch

    import synth
    from paper_2405_12079_amd import phos
    w = synth.config1_world()
    n_launch, n_rec = 100, 1_000_000
    launches = synth.config1_launches(w, n_launch, n_rec)
    page = w.page_bytes
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    recs = synth.records_device(synth.DeviceWorld(w, base), launches, n_rec)
    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    try:
        phos.phos_buffers_register(ctx, w.buffers(base))
        specs = [phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches]
        ptrs = [recs.data_ptr() + j * n_rec * 8 for j in range(n_launch)]
        cap = 400_000
        out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        s = torch.cuda.Stream()
        t = Timer(torch, s)
        ts = []
        for _ in range(reps + 1):
            t.start()
            phos.phos_validate_batch(ctx, specs, ptrs, [n_rec] * n_launch,
                                     phos.V_READS | phos.V_WRITES | phos.V_TRACK, out, cap,
                                     cnt.data_ptr(), s)
            t.stop()
            s.synchronize()
            ts.append(t.ms())
        ms = float(np.median(ts[1:]))
        nv = int(cnt.item())
    finally:
        torch.cuda.synchronize()
        phos.phos_destroy(ctx)
    del recs, back
    torch.cuda.empty_cache()
    return {"workload": "plain tiny: 64 MiB pool, 256 buffers, 4 KiB pages, "
                        f"{n_launch} launches x {n_rec} accesses, reads+writes checked, tracked",
            "validated_addr_per_s": round(n_launch * n_rec / (ms / 1e3), 1),
            "ms": round(ms, 4), "violations": nv}


# ---------------------------------------------------------------- config 3
def run_batched(args):
    """64 simultaneous checkpoint requests (images 100 MiB .. 8 GiB, 50..5000
    buffers, 5..60 % dirty at 64 KiB pages): every dirty run copied into
    compact per-request deltas by one persistent graph-captured launch with the
    autotuned chunk and grid, against 64 plain per-request launches."""
    import torch

    import oracle
    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    page = 64 << 10
    reqs = synth.config3_requests()
    src_bytes = sum(q.pages for q in reqs) * page
    dst_bytes = sum(q.dirty_pages for q in reqs) * page
    seed = synth.CFG_SEED + 3
    log(f"[bench] batched: {len(reqs)} requests, sources {src_bytes / 2**30:.1f} GiB, "
        f"deltas {dst_bytes / 2**30:.1f} GiB")
    src = torch.empty(src_bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(dst_bytes, dtype=torch.uint8, device="cuda")
    synth.content_device(src, seed)
    torch.cuda.synchronize()
    segs = synth.request_segments(reqs, src.data_ptr(), dst.data_ptr(), page)
    s = torch.cuda.Stream()
    # autotune on another seed's requests (a quarter of the count), same arenas
    treqs = [q for q in synth.batch_requests(seed + 100, 16, 100 << 20, 8 << 30, page)]
    acc_s = acc_d = 0
    fit = []
    for q in treqs:
        if acc_s + q.pages * page <= src_bytes and acc_d + q.dirty_pages * page <= dst_bytes:
            q.src_off, q.dst_off = acc_s, acc_d
            acc_s += q.pages * page
            acc_d += q.dirty_pages * page
            fit.append(q)
    tsegs = synth.request_segments(fit, src.data_ptr(), dst.data_ptr(), page)
    cache = os.path.join(ROOT, "paper_2405_12079_amd", "tune_cache.txt")
    t0 = time.perf_counter()
    cfg, tune_ms = phos.phos_batch_tune(0, tsegs, cache)
    log(f"[bench] tuned in {time.perf_counter() - t0:.1f} s: chunk {cfg.chunk_bytes >> 10} KiB, "
        f"{cfg.wg_per_cu} WG/CU, {cfg.threads} threads ({tune_ms:.2f} ms on the tuning set)")
    b = phos.phos_batch_create(0, len(segs), len(reqs), cfg)
    phos.phos_batch_load(b, segs, s)
    lists = [phos.phos_seglist_create(0, synth.request_segments([q], src.data_ptr(), dst.data_ptr(),
                                                               page)) for q in reqs]
    tb = Timer(torch, s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(reqs) + 1)]
    batched, plain, plain_done, bdone = [], [], [], []
    for i in range(args.warmup + args.steps):
        tb.start()
        phos.phos_batch_run(b, s)
        tb.stop()
        s.synchronize()
        ev[0].record(s)
        for j, l in enumerate(lists):
            phos.phos_copy_plain(l, cfg.chunk_bytes, cfg.threads, s)
            ev[j + 1].record(s)
        s.synchronize()
        if i >= args.warmup:
            batched.append(tb.ms())
            bdone.append(phos.phos_batch_times(b, len(reqs)))
            fin = [ev[0].elapsed_time(ev[j + 1]) for j in range(len(reqs))]
            plain.append(fin[-1])
            plain_done.append(fin)
        log(f"[bench] step {i}: batched {tb.ms():.2f} ms, plain {ev[0].elapsed_time(ev[-1]):.2f} ms")
    # parity: every delta page of every request against the oracle's gather
    # of the request's segments (source pages from the input generator),
    # compared as page fingerprints (37 GiB do not fit the host twice)
    parity = None
    if args.parity:
        torch.cuda.synchronize()
        with torch.cuda.stream(s):  # the clear and the copy in stream order
            dst.fill_(0)
        phos.phos_batch_run(b, s)
        s.synchronize()
        t0 = time.perf_counter()
        qs = synth.request_segments(reqs, 0, 0, page)  # offsets in the source / delta arenas
        n_dst = dst_bytes // page
        want = oracle.gather_hashes(lambda o, n: synth.content_host(seed, o, n), qs["src"],
                                    qs["dst"], qs["bytes"], page, n_dst, HOST_THREADS)
        got = oracle.hash_chunks(lambda o, n: dst[o:o + n].cpu().numpy(), dst_bytes, page,
                                 1 << 30, HOST_THREADS)
        bad = np.flatnonzero(got != want)
        log(f"[bench] parity: {n_dst} delta pages hashed in {time.perf_counter() - t0:.1f} s, "
            f"{bad.size} differ")
        assert bad.size == 0, f"batched copy: {bad.size} delta pages differ (first {bad[:5]})"
        parity = (f"hash-equal: all {n_dst} delta pages of the {len(reqs)} requests equal the "
                  "oracle's gather of their segments")
    bt = float(np.median(batched))
    pt = float(np.median(plain))
    fin = np.median(np.array(plain_done), axis=0)
    bfin = np.median(np.array(bdone), axis=0)  # GPU wall-clock completion stamps
    res = {
        "metric": "snapshot GB/s vs HBM peak (batched persistent copy); p99 request latency "
                  "batched vs plain",
        "value": round(dst_bytes / (bt / 1e3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(bt, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded request sizes, buffer shares, dirty sets, contents)",
        "config": {"workload": "batched-uneven: 64 checkpoint requests, images 100 MiB-8 GiB, "
                               "50-5000 buffers, 5-60 % dirty, 64 KiB pages",
                   "copied_bytes": int(dst_bytes), "segments": int(len(segs))},
        "batched_ms": round(bt, 3), "plain_ms": round(pt, 3),
        "plain_GBps": round(dst_bytes / (pt / 1e3) / 1e9, 2),
        "latency_ms": {"batched_p50": round(float(np.percentile(bfin, 50)), 3),
                       "batched_p99": round(float(np.percentile(bfin, 99)), 3),
                       "plain_p50": round(float(np.percentile(fin, 50)), 3),
                       "plain_p99": round(float(np.percentile(fin, 99)), 3)},
        "tuned": {"chunk_bytes": cfg.chunk_bytes, "wg_per_cu": cfg.wg_per_cu,
                  "threads": cfg.threads},
        "roofline": {"bound": "hbm", "kernel": "batch_copy_kernel",
                     "achieved": round(2 * dst_bytes / (bt / 1e3) / 1e9, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(2 * dst_bytes / (bt / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic("batch_copy_kernel", "batched_uneven"),
                     "algorithmic_bytes_per_launch": int(2 * dst_bytes),
                     "avg_launch_ms": round(bt, 4)},
        "parity": parity,
    }
    for l in lists:
        phos.phos_seglist_destroy(l)
    phos.phos_batch_destroy(b)
    if not args.no_cpu_baseline:
        # oracle gather on a bounded sample: 2 GiB of one request's dirty runs
        q = max(reqs, key=lambda x: x.dirty_pages)
        nb = min(q.dirty_pages, (2 << 30) // page)
        runs_s, runs_l, acc = [], [], 0
        for st, ln in zip(q.dirty_start, q.dirty_len):
            take = min(int(ln), nb - acc)
            if take <= 0:
                break
            runs_s.append(int(st))
            runs_l.append(take)
            acc += take
        span = (runs_s[-1] + runs_l[-1]) * page
        srch = synth.content_host(seed, q.src_off, span)
        out = np.empty(acc * page, np.uint8)
        so = np.array(runs_s, np.uint64) * np.uint64(page)
        ln = np.array(runs_l, np.uint64) * np.uint64(page)
        do = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
        t0 = time.perf_counter()
        oracle.gather(srch, out, so, do, ln)
        tg = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(acc * page / tg / 1e9, 3), "unit": "GB/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"gather of {acc * page / 2**30:.2f} GiB of request "
                                         f"{q.r}'s dirty runs", "cpu": cpu_model()}
    return res


# ---------------------------------------------------------------- config 5
def run_cold_start(args):
    """Cold-start restore at scale: a 70 GiB image of 500 buffers (16..512 MiB)
    in pinned host memory is restored into a fresh 70 GiB pool while a
    decode-like stream of 40,000 launches (2..6 buffers, 262,144 accesses
    each) runs; each launch first brings in the pages its accesses touch
    (validation in restore mode), the rest arrives in the background."""
    import torch

    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    w = synth.config5_world()
    n_launch, n_rec = args.launches5, 262_144
    page = w.page_bytes
    launches = synth.config5_launches(w, n_launch, n_rec)
    log(f"[bench] cold-start: {w.n_alloc} buffers, image {w.image_bytes / 2**30:.1f} GiB, "
        f"{n_launch} launches x {n_rec} accesses")
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + w.pool_bytes]
    dw = synth.DeviceWorld(w, base)
    recs = torch.empty(n_launch * n_rec, dtype=torch.int64, device="cuda")
    for g in range(0, n_launch, 2000):
        grp = launches[g:g + 2000]
        synth.records_device(dw, grp, n_rec, out=recs[g * n_rec:(g + len(grp)) * n_rec])
    # the library's context first: its own small pinned buffers must not find
    # the host's pinning limit already used up by the image
    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    phos.phos_buffers_register(ctx, w.buffers(base))
    # the image: the pool's initial contents, buffer by buffer, in host memory,
    # in pieces of 32 GiB; pinned as far as the system grants it (on the
    # MI355X host used here one process can pin 64 GiB), the rest pageable,
    # which the library moves by DMA instead of from its kernels
    t0 = time.perf_counter()
    cb = 32 << 30
    pieces, pinned_bytes = [], 0
    for o in range(0, w.image_bytes, cb):
        n = min(cb, w.image_bytes - o)
        try:
            pieces.append(pinned_tensor(torch, n))
            pinned_bytes += n
        except RuntimeError:
            pieces.append(torch.empty(n, dtype=torch.uint8))
    log(f"[bench] image in {len(pieces)} pieces: {pinned_bytes / 2**30:.1f} GiB pinned, "
        f"{(w.image_bytes - pinned_bytes) / 2**30:.1f} GiB pageable "
        f"({time.perf_counter() - t0:.1f} s)")

    def image_spans(o, b, off):
        """(pool offset, piece, offset in piece, bytes) covering image bytes [off, off+b)."""
        while b:
            k, r = divmod(off, cb)
            n = min(b, cb - r)
            yield o, pieces[k], r, n
            o, off, b = o + n, off + n, b - n

    synth.content_device(pool, w.seed)
    torch.cuda.synchronize()
    off = 0
    for o, b in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
        for po, piece, r, n in image_spans(o, b, off):
            piece[r:r + n].copy_(pool[po:po + n])
        off += b
    torch.cuda.synchronize()
    specs = [phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches]
    app, cpy = torch.cuda.Stream(), torch.cuda.Stream()

    # stop-the-world reference: the whole image copied in before launch 0
    pool.zero_()
    torch.cuda.synchronize()
    t_stw = Timer(torch, app)
    t_stw.start()
    with torch.cuda.stream(app):
        off = 0
        for o, b in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
            for po, piece, r, n in image_spans(o, b, off):
                pool[po:po + n].copy_(piece[r:r + n], non_blocking=True)
            off += b
    t_stw.stop()
    app.synchronize()
    stw_ms = t_stw.ms()
    log(f"[bench] stop-the-world restore: {stw_ms:.1f} ms ({w.image_bytes / stw_ms / 1e6:.1f} GB/s)")

    # concurrent restore
    pool.zero_()
    torch.cuda.synchronize()
    e_begin = torch.cuda.Event(enable_timing=True)
    e_end = torch.cuda.Event(enable_timing=True)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(n_launch)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(n_launch)]
    faulted = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e_begin.record(app)
    cpy.wait_event(e_begin)
    h0 = time.perf_counter()
    rs = phos.phos_restore_begin_chunked(ctx, 0, pieces, cb, cpy)
    h_begin = time.perf_counter() - h0
    h_first = 0.0
    for j, L in enumerate(launches):
        r = recs.data_ptr() + j * n_rec * 8
        ev0[j].record(app)
        h1 = time.perf_counter()
        phos.phos_restore_on_demand(rs, specs[j], r, n_rec, app, faulted)
        if j == 0:
            h_first = time.perf_counter() - h1
        ev1[j].record(app)
        synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, r, n_rec, app)
    e_end.record(app)
    st = phos.phos_restore_end(rs, app)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ttfk = e_begin.elapsed_time(ev1[0])
    # the background restore's GPU time (HIP events on the library's stream,
    # which starts right after the begin call), or the pageable pieces' DMA
    full = max(st.bg_ms, st.dma_ms)
    stream_ms = e_begin.elapsed_time(e_end)
    stalls = np.array([ev0[j].elapsed_time(ev1[j]) for j in range(n_launch)])
    h2d = w.image_bytes / (max(full, stream_ms) / 1e3) / 1e9
    log(f"[bench] host: begin call {h_begin * 1e3:.2f} ms, first on-demand call {h_first * 1e3:.2f} ms; "
        f"GPU: app stream reaches launch 0 after {e_begin.elapsed_time(ev0[0]):.2f} ms, "
        f"its fault-in takes {ev0[0].elapsed_time(ev1[0]):.2f} ms")
    log(f"[bench] time to first kernel {ttfk:.2f} ms; fully present {full:.1f} ms; stream "
        f"{stream_ms:.1f} ms; demand pages {st.demand_pages}, background {st.bg_pages}, "
        f"DMA {st.dma_pages} ({st.asked_pages} asked for, first queued after "
        f"{st.dma_first_issue_ms:.1f} ms, landed after {st.dma_first_copy_ms:.1f} ms, "
        f"published after {st.dma_first_ms:.1f} ms, "
        f"done after {st.dma_ms:.1f} ms); "
        f"stall p50 {np.percentile(stalls, 50) * 1e3:.1f} us p99 {np.percentile(stalls, 99) * 1e3:.1f} us")
    res = {
        "metric": "cold-start restore: time-to-first-kernel; PCIe GB/s of the concurrent restore",
        "value": round(ttfk, 3), "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(stream_ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded layout, decode-like access streams, contents)",
        "config": {"workload": "cold-start: 70 GiB image of 500 buffers in host memory, "
                               f"{n_launch} launches x {n_rec} accesses, 64 KiB pages",
                   "image_bytes": int(w.image_bytes), "pinned_bytes": int(pinned_bytes),
                   "pageable_bytes": int(w.image_bytes - pinned_bytes)},
        "time_to_first_kernel_ms": round(ttfk, 3),
        "stop_the_world_restore_ms": round(stw_ms, 3),
        "fully_present_ms": round(full, 3),
        "stream_ms": round(stream_ms, 3), "wall_s": round(wall, 3),
        "restore_h2d_GBps": round(h2d, 2),
        "stop_the_world_h2d_GBps": round(w.image_bytes / stw_ms / 1e6, 2),
        "demand_pages": int(st.demand_pages), "background_pages": int(st.bg_pages),
        "dma_pages": int(st.dma_pages), "dma_asked_pages": int(st.asked_pages),
        "dma_ms": round(st.dma_ms, 1),
        "stall_ms": {"p50": round(float(np.percentile(stalls, 50)), 4),
                     "p99": round(float(np.percentile(stalls, 99)), 4),
                     "max": round(float(stalls.max()), 3)},
    }
    if args.parity:
        # Section 6: the restored pool plus the launches equals the oracle's
        # stop-the-world restore of the image (the buffers' initial contents)
        # plus the same launches' writes in order, replayed on a host pool
        # from the seeded inputs; every buffer page compared as a fingerprint
        import oracle
        t0 = time.perf_counter()
        table = oracle.Table.from_world(w, base)
        got = oracle.image_hashes_from_reader(lambda o, n: pool[o:o + n].cpu().numpy(), base,
                                              table, page, 1 << 30, HOST_THREADS)
        del pieces  # the image's host memory, before the oracle's pool takes as much
        release_pinned(torch)
        hw = synth.HostWorld(w, base)
        host = synth.content_host_parallel(w.seed, 0, w.pool_bytes, HOST_THREADS)
        oracle.apply_stream(host, launches, lambda L: synth.records_host(hw, L),
                            lambda p, L, rec: synth.apply_writes_host(p, base, w.seed, L.k, rec),
                            threads=HOST_THREADS,
                            log=lambda j: log(f"[bench] parity: oracle replay at launch {j}"))
        want = oracle.image_hashes_from_pool(host, base, table, page, HOST_THREADS)
        del host
        bad = np.flatnonzero(got != want)
        log(f"[bench] parity: {want.size} pool pages against the oracle's replay in "
            f"{time.perf_counter() - t0:.1f} s, {bad.size} differ")
        res["parity"] = (f"hash-equal: all {want.size} buffer pages of the restored pool + "
                         f"{n_launch} launches equal the oracle's restore + the same launches: "
                         f"{bad.size == 0}")
        assert bad.size == 0, f"cold-start restore: {bad.size} pages differ (first {bad[:5]})"
    phos.phos_destroy(ctx)
    if not args.no_cpu_baseline:
        # the oracle's restore: each buffer's image bytes to its place in the
        # pool, for the buffers in the image's first 2 GiB
        cap = 2 << 30
        img_off = np.concatenate([[0], np.cumsum(w.alloc_bytes.astype(np.int64))])
        so, do, ln = [], [], []
        for b in range(w.n_alloc):
            if img_off[b] >= cap:
                break
            so.append(int(img_off[b]))
            do.append(int(w.alloc_off[b]))
            ln.append(int(min(w.alloc_bytes[b], cap - img_off[b])))
        res["cpu_baseline"] = cpu_gather_baseline(w.seed, cap, so, do, ln,
                                                  "image to pool of the image's first 2 GiB")
    return res


# ---------------------------------------------------------------- config 4
def serving_inputs(torch, phos, synth, trace, page, src_base, seed):
    """Marshal a serving trace: segment arrays for checkpoints / restores, device
    access records and seeded present-page claim words for bursts."""
    keep, bursts = [], []
    arr = (phos.phos_serve_req * max(1, len(trace)))()
    for j, q in enumerate(trace):
        R = arr[j]
        R.arrival_s, R.type, R.bytes = q.arrival_s, q.type, q.size
        if q.type == synth.REQ_BURST:
            w = synth.burst_world(q, page)
            L = synth.burst_launch(q, w)
            rec = synth.records_device(synth.DeviceWorld(w, 0), [L], q.n_rec)
            state = torch.empty(q.size // page, dtype=torch.int32, device="cuda")
            synth.present_device(state, seed, q.r)
            R.d_records, R.nrec = rec.data_ptr(), q.n_rec
            R.d_state, R.image = state.data_ptr(), src_base + q.src_off
            keep += [rec, state]
            bursts.append((q, state))
            continue
        if q.type == synth.REQ_CKPT:
            st, ln = q.runs
        else:
            st, ln = np.zeros(1, np.int64), np.array([q.size // page], np.int64)
        segs = np.zeros(len(st), dtype=phos.SEG_DTYPE)
        segs["src"] = np.uint64(src_base + q.src_off) + st.astype(np.uint64) * np.uint64(page)
        segs["dst"] = st.astype(np.uint64) * np.uint64(page)
        segs["bytes"] = ln.astype(np.uint64) * np.uint64(page)
        keep.append(segs)
        R.segs, R.nseg = segs.ctypes.data, len(segs)
    torch.cuda.synchronize()
    return arr, keep, bursts


def reseed_bursts(torch, synth, bursts, seed):
    for q, state in bursts:
        synth.present_device(state, seed, q.r)
    torch.cuda.synchronize()


def latency_stats(trace, outs, t_from, synth):
    res = {}
    names = {synth.REQ_CKPT: "checkpoint", synth.REQ_RESTORE: "restore", synth.REQ_BURST: "burst"}
    sel = [j for j, q in enumerate(trace) if q.arrival_s >= t_from]
    for ty, name in list(names.items()) + [(None, "all")]:
        lat = np.array([outs[j].latency_ms for j in sel if ty is None or trace[j].type == ty])
        if lat.size:
            res[name] = {"n": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "max_ms": round(float(lat.max()), 3)}
    return res


def run_serving(args):
    """Poisson arrivals (200 req/s, 30 s after a 2 s warm-up) of checkpoint
    (70 %), restore (20 %) and on-demand fault-burst (10 %) requests of
    64 MiB..16 GiB, admitted against a 2e11-byte HBM budget; the same trace is
    served by the plain FIFO path and by continuous batching."""
    import torch

    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    page, seed = 64 << 10, synth.CFG_SEED + 4
    arena = 16 << 30
    warm, dur = 2.0, args.serve_seconds
    trace = synth.serving_trace(seed, 200.0, warm + dur, 64 << 20, 16 << 30, page, arena)
    src = torch.empty(arena, dtype=torch.uint8, device="cuda")
    synth.content_device(src, seed)
    budget = 200_000_000_000 // page * page
    dst = torch.empty(budget, dtype=torch.uint8, device="cuda")
    reqs, keep, bursts = serving_inputs(torch, phos, synth, trace, page, src.data_ptr(), seed)
    cache = os.path.join(ROOT, "paper_2405_12079_amd", "tune_cache.txt")
    bcfg = phos.phos_batch_cfg(64 << 10, 1, 512)  # the contiguous-copy optimum measured here
    log(f"[bench] serving: {len(trace)} requests over {warm + dur:.0f} s, "
        f"{sum(q.size for q in trace) / (warm + dur) / 2**30:.0f} GiB/s offered (request sizes)")
    out = {}
    for mode, name in ((phos.SERVE_PLAIN, "plain"), (phos.SERVE_BATCHED, "batched")):
        reseed_bursts(torch, synth, bursts, seed)
        cfg = phos.phos_serve_cfg(mode, page, budget, dst.data_ptr(), args.quantum << 20,
                                  args.iter_mib << 20, bcfg, 0, 0, args.small_mib << 20)
        outs, st = phos.phos_serve_run(0, cfg, reqs, len(trace))
        lat = latency_stats(trace, outs, warm, synth)
        out[name] = {"latency": lat, "wall_ms": round(st.wall_ms, 1),
                     "GBps": round(st.bytes / (st.wall_ms / 1e3) / 1e9, 2),
                     "copied_bytes": int(st.bytes), "iterations": int(st.iterations),
                     "max_active": int(st.max_active)}
        log(f"[bench] {name}: p50 {lat['all']['p50_ms']} ms, p99 {lat['all']['p99_ms']} ms, "
            f"{out[name]['GBps']} GB/s, max active {st.max_active}, iterations {st.iterations}")
    del keep
    bp99, pp99 = out["batched"]["latency"]["all"]["p99_ms"], out["plain"]["latency"]["all"]["p99_ms"]
    return {
        "metric": "p99 C/R request latency, batched vs plain per-request path (same trace)",
        "value": bp99, "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": out["batched"]["wall_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded Poisson trace, sizes, dirty runs, burst accesses, contents)",
        "config": {"workload": f"serving: Poisson 200 req/s for {dur:.0f} s after {warm:.0f} s, "
                               "70 % checkpoint / 20 % restore / 10 % fault burst, 64 MiB-16 GiB, "
                               "2e11-byte HBM budget", "requests": len(trace),
                   "quantum_bytes": args.quantum << 20, "iteration_bytes": args.iter_mib << 20},
        "plain_p99_ms": pp99, "batched_p99_ms": bp99,
        "batched": out["batched"], "plain": out["plain"],
    }


def cpu_gather_baseline(seed, span, src_off, dst_off, lens, label):
    """The oracle's gather (plain C, one thread) of runs of a seeded host
    span: a bounded sample of the copies a workload makes (a snapshot of
    pages into an image, or an image back into the pool)."""
    import oracle
    import synth
    so, do, ln = (np.asarray(x, dtype=np.uint64) for x in (src_off, dst_off, lens))
    src = synth.content_host(seed, 0, int(span))
    dst = np.empty(int((do + ln).max()), np.uint8)
    t0 = time.perf_counter()
    oracle.gather(src, dst, so, do, ln)
    t = time.perf_counter() - t0
    n = int(ln.sum())
    return {"value": round(n / t / 1e9, 3), "unit": "GB/s (bytes copied)", "cores": 1,
            "kind": "oracle", "sample": f"{label}: {n / 2**30:.2f} GiB gathered in {t:.2f} s",
            "cpu": cpu_model()}


def cpu_baseline_training_step(w, launches, base, img_bytes, n_addr):
    """The oracle on a bounded sample of the step: validation + tracking of the
    step's launches (up to 1000) and snapshots of 4 GiB of buffers, on one
    thread and on the host's cores (T threads: the oracle's C calls release
    the GIL; launches and buffers split across them); scaled to the step's
    work (about 10 s of CPU time in all)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth
    hw = synth.HostWorld(w, base)
    table = oracle.Table.from_world(w, base)
    sample = launches[: min(1000, len(launches))]
    recs = [synth.records_host(hw, L) for L in sample]  # inputs: not timed
    npg = w.n_pages
    n_val = sum(r.shape[0] for r in recs)

    def validate_some(idx):
        dirty = np.zeros(npg, np.uint8)
        vic = np.zeros(npg, np.uint8)
        for i in idx:
            L = sample[i]
            iv = oracle.spec_build(table, L.arg_values(base))
            oracle.validate(iv, recs[i], table, L.k)
            oracle.track(iv, recs[i], table, base, w.page_bytes, npg, dirty, vic)

    t0 = time.perf_counter()
    validate_some(range(len(sample)))
    t_val = time.perf_counter() - t0
    T = HOST_THREADS
    t0 = time.perf_counter()
    with ThreadPoolExecutor(T) as ex:
        list(ex.map(validate_some, [range(t, len(sample), T) for t in range(T)]))
    t_val_T = time.perf_counter() - t0
    # snapshot sample: the first buffers up to 4 GiB, contents from the generator
    acc, nb = 0, 0
    while nb < w.n_alloc and acc + int(w.alloc_bytes[nb]) <= (4 << 30):
        acc += int(w.alloc_bytes[nb])
        nb += 1
    span = int(w.alloc_off[nb - 1] + w.alloc_bytes[nb - 1])
    pool = synth.content_host(w.seed, 0, span)
    sub = oracle.Table(table.base[:nb], table.bytes[:nb])
    t0 = time.perf_counter()
    img = oracle.snapshot(pool, base, sub)
    t_snap = time.perf_counter() - t0
    del img
    cuts = np.linspace(0, nb, T + 1).astype(int)
    parts = [oracle.Table(table.base[a:b], table.bytes[a:b]) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(T) as ex:
        list(ex.map(lambda t: oracle.snapshot(pool, base, t).shape, parts))
    t_snap_T = time.perf_counter() - t0
    del pool

    def rate(tv, ts):
        a, s = n_val / tv, acc / ts
        return img_bytes / (n_addr / a + img_bytes / s) / 1e9, a, s

    gb1, a1, s1 = rate(t_val, t_snap)
    gbT, aT, sT = rate(t_val_T, t_snap_T)
    return {"value": round(gbT, 3), "unit": "GB/s", "cores": T, "kind": "oracle",
            "sample": f"{len(sample)} launches x {sample[0].n_records} accesses validated+tracked "
                      f"and a {acc / 2**30:.1f} GiB snapshot, on {T} threads ({t_val_T:.2f} s + "
                      f"{t_snap_T:.2f} s) and on one ({t_val:.1f} s + {t_snap:.2f} s); step time = "
                      "all accesses / rate + image bytes / memcpy rate",
            "validated_addr_per_s": round(aT, 1), "snapshot_GBps": round(sT / 1e9, 3),
            "single_thread": {"value": round(gb1, 3), "validated_addr_per_s": round(a1, 1),
                              "snapshot_GBps": round(s1 / 1e9, 3)},
            "cpu": cpu_model(), **HOST_CPU_DETAIL}


def run_twin(args):
    """Section 4.1 twin kernel: the validator fused into an application kernel
    (y[j] = 3 y[j] + x[i], uint64, 2^28 elements of 8 bytes per array),
    timed against the same kernel uninstrumented; contiguous (j = i) and
    indirect (j = idx[i], a fixed permutation inside each 64-element block)."""
    import torch

    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    n = args.twin_n
    page = 64 << 10
    nb = (n * 8 + page - 1) // page * page
    back = torch.empty(3 * nb + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + 3 * nb]
    xo, yo, io = 0, nb, 2 * nb
    p64 = pool.view(torch.int64)
    x, y, idx = p64[:n], p64[nb // 8: nb // 8 + n], p64[2 * nb // 8: 2 * nb // 8 + n]
    g = torch.Generator(device="cuda").manual_seed(0x5457494E)
    x.random_(generator=g)
    y.random_(generator=g)
    perm = torch.randperm(64, generator=torch.Generator().manual_seed(7)).to("cuda")
    ar = torch.arange(n, device="cuda", dtype=torch.int64)
    idx.copy_((ar & ~63) + perm[ar & 63])
    del ar
    torch.cuda.synchronize()
    ctx = phos.phos_create(0, base, 3 * nb, page)
    phos.phos_buffers_register(ctx, [(base + xo, nb), (base + yo, nb), (base + io, nb)])
    spec = phos.phos_spec_register(ctx, 1, [(phos.ARG_PTR_CONST, 0, base + xo, 0),
                                            (phos.ARG_PTR_MUT, 0, base + yo, 0),
                                            (phos.ARG_PTR_CONST, 0, base + io, 0)])
    s = torch.cuda.Stream()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.zeros(1024 * 32, dtype=torch.uint8, device="cuda")
    log(f"[bench] twin kernel: 3 x {n * 8 / 2**30:.1f} GiB arrays, spec of 3 intervals")

    def launch(flags, indirect):
        phos.phos_twin_scale_add(ctx, spec, base + xo, base + yo, base + io if indirect else 0, n,
                                 flags, out.data_ptr(), 1024, cnt.data_ptr(), s)

    # parity on sampled elements: one instrumented then one plain launch
    samp = torch.randint(0, n, (4096,), generator=g, device="cuda")
    parity = []
    for indirect in (False, True):
        t = idx[samp] if indirect else samp
        y0, xs = y[t].clone(), x[samp].clone()
        torch.cuda.synchronize()
        phos.phos_track_reset(ctx, s)
        launch(phos.V_READS | phos.V_WRITES | phos.V_TRACK, indirect)
        s.synchronize()
        y1 = y[t].clone()
        nviol = int(cnt.item())
        dirty = phos.phos_track_read(ctx, 0, 3 * nb // page)
        pages = np.unpackbits(dirty.view(np.uint8), bitorder="little")[:3 * nb // page]
        launch(0, indirect)
        s.synchronize()
        y2 = y[t].clone()
        e1 = y0 * 3 + xs  # int64 arithmetic wraps like uint64
        ok = (bool(torch.equal(y1, e1)) and bool(torch.equal(y2, e1 * 3 + xs)) and nviol == 0
              and pages.sum() == (n * 8 + page - 1) // page and pages[nb // page] == 1
              and pages[:nb // page].sum() == 0)
        parity.append(ok)
        assert ok, f"twin kernel parity failed (indirect={indirect})"
    variants = [("plain", 0), ("writes", phos.V_WRITES), ("reads_writes", phos.V_READS | phos.V_WRITES),
                ("reads_writes_track", phos.V_READS | phos.V_WRITES | phos.V_TRACK)]
    res_ms = {}
    for indirect in (False, True):
        for name, fl in variants:
            e0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + args.warmup)]
            e1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + args.warmup)]
            for r in range(args.steps + args.warmup):
                e0[r].record(s)
                launch(fl, indirect)
                e1[r].record(s)
            s.synchronize()
            ts = np.array([e0[r].elapsed_time(e1[r]) for r in range(args.warmup, args.steps + args.warmup)])
            key = ("indirect_" if indirect else "contiguous_") + name
            res_ms[key] = {"median": round(float(np.median(ts)), 4),
                           "p10": round(float(np.percentile(ts, 10)), 4),
                           "p90": round(float(np.percentile(ts, 90)), 4)}
            log(f"[bench] {key}: {res_ms[key]['median']:.3f} ms")
    ov = {k: round(100.0 * (res_ms[k]["median"] / res_ms[("indirect_" if k.startswith("indirect")
                                                          else "contiguous_") + "plain"]["median"] - 1), 2)
          for k in res_ms if not k.endswith("plain")}
    plain_ms = res_ms["contiguous_plain"]["median"]
    twin_ms = res_ms["contiguous_reads_writes_track"]["median"]
    alg = 24 * n  # read x[i], read y[i], write y[i]
    log(f"[bench] twin overhead (%): {ov}")
    phos.phos_spec_release(ctx, spec)
    phos.phos_destroy(ctx)
    return {
        "metric": "twin-kernel validator overhead vs the uninstrumented kernel (reads + writes "
                  "checked, dirty pages tracked)",
        "value": ov["contiguous_reads_writes_track"], "unit": "%", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": twin_ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (seeded array contents, fixed in-block permutation)",
        "config": {"workload": f"twin kernel: y[j] = 3 y[j] + x[i] over {n} uint64 elements, "
                               "spec of 3 intervals (x R, y RW, idx R)", "elements": n},
        "ms": res_ms, "overhead_pct": ov,
        "roofline": {"bound": "hbm", "kernel": "twin_kernel (uninstrumented, contiguous)",
                     "achieved": round(alg / (plain_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(alg / (plain_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "traffic": None, "algorithmic_bytes_per_launch": alg},
        "roofline_twin": {"bound": "hbm", "kernel": "twin_kernel (reads + writes + tracking)",
                          "achieved": round(alg / (twin_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                          "unit": "GB/s", "frac": round(alg / (twin_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "parity": f"sampled elements equal 3 y + x after the twin and again after the plain kernel; "
                  f"no violations; dirty pages exactly y's: {parity}",
    }


def run_drain(args):
    """Section 5 preemptible drain: a 16 GiB image drained to pinned host
    memory by phos_ckpt_end, once as one copy and once in chunks (the
    default), while the application issues 64 MiB device-to-host copies;
    reports the application copies' latency and the drain rate."""
    import threading

    import torch

    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    page, pool_bytes = 64 << 10, 16 << 30
    back = torch.empty(pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    img = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    host_img = pinned_tensor(torch, pool_bytes)
    app_dev = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    app_host = pinned_tensor(torch, 64 << 20)
    app, cpy = torch.cuda.Stream(), torch.cuda.Stream()
    back.random_(0, 256)
    torch.cuda.synchronize()

    def app_copies(k):
        ts = []
        for _ in range(k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(app)
            with torch.cuda.stream(app):
                app_host.copy_(app_dev, non_blocking=True)
            e1.record(app)
            app.synchronize()
            ts.append(e0.elapsed_time(e1))
        return ts

    out = {"app_copy_alone_ms": round(float(np.median(app_copies(20))), 3)}
    for label, chunk_kb in (("one_copy", "0"), ("chunked", None)):
        saved = os.environ.get("PHOS_DRAIN_CHUNK_KB")
        if chunk_kb is not None:
            os.environ["PHOS_DRAIN_CHUNK_KB"] = chunk_kb
        try:
            ctx = phos.phos_create(0, base, pool_bytes, page)
        finally:
            if chunk_kb is not None:
                if saved is None:
                    del os.environ["PHOS_DRAIN_CHUNK_KB"]
                else:
                    os.environ["PHOS_DRAIN_CHUNK_KB"] = saved
        phos.phos_buffers_register(ctx, [(base, pool_bytes)])
        rates, lat = [], []
        for rep in range(max(2, args.steps)):
            ck = phos.phos_ckpt_begin(ctx, phos.COW, 0, img.data_ptr(), host_img.data_ptr(), cpy)
            torch.cuda.synchronize()  # the background copy has finished: time the drain alone
            box = {}

            def end():
                t0 = time.perf_counter()
                phos.phos_ckpt_end(ck, cpy)
                box["s"] = time.perf_counter() - t0

            th = threading.Thread(target=end)
            th.start()
            time.sleep(0.02)
            lat += app_copies(8)
            th.join()
            rates.append(pool_bytes / box["s"] / 1e9)
        same = bool(torch.equal(host_img[:1 << 20], img[:1 << 20].cpu()))
        phos.phos_destroy(ctx)
        out[label] = {"drain_GBps": round(float(np.median(rates)), 2),
                      "app_copy_ms_during_drain": {"median": round(float(np.median(lat)), 3),
                                                   "p90": round(float(np.percentile(lat, 90)), 3),
                                                   "max": round(float(np.max(lat)), 3)},
                      "image_prefix_equal": same}
        log(f"[bench] drain {label}: {out[label]}")
    return {
        "metric": "app device-to-host copy latency during the image drain (p90, ms); drain GB/s",
        "value": out["chunked"]["app_copy_ms_during_drain"]["p90"], "unit": "ms", "n_gpus": 1,
        "steps": max(2, args.steps), "warmup": 0, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (random image bytes)",
        "config": {"workload": "preemptible drain: 16 GiB image to pinned host memory, "
                               "64 MiB application copies to host meanwhile"},
        **out,
    }


def run_staging(args):
    """Section 4.2 copy-on-write staging budget: the training-step layout and
    launches with one copy-on-write checkpoint into a 16 GiB pinned host
    image.  The background copy crosses PCIe (~0.3 s), so the pages the
    launches write first are copied on demand; with a device staging area of
    B bytes the first B bytes of them are copied at HBM speed, the rest over
    PCIe.  Reports the launches' stall (loop time minus the same loop without
    a checkpoint) against B."""
    import torch

    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    w = synth.config2_world()
    n_launch, n_rec = args.launches, 1_000_000
    launches = synth.config2_launches(w, n_launch, n_rec)
    page = w.page_bytes
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + w.pool_bytes]
    dw = synth.DeviceWorld(w, base)
    recs = torch.empty(n_launch * n_rec, dtype=torch.int64, device="cuda")
    for g in range(0, n_launch, 100):
        synth.records_device(dw, launches[g:g + 100], n_rec, out=recs[g * n_rec:(g + 100) * n_rec])
    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    phos.phos_buffers_register(ctx, w.buffers(base))
    nimg = phos.phos_image_bytes(ctx)
    himg = pinned_tensor(torch, nimg)
    staging = torch.empty(nimg, dtype=torch.uint8, device="cuda")
    snap = torch.empty(w.pool_bytes, dtype=torch.uint8, device="cuda")
    specs = [phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches]
    rec_ptrs = [recs.data_ptr() + j * n_rec * 8 for j in range(n_launch)]
    lcap = 2_000_000
    vout = torch.empty(lcap * 32, dtype=torch.uint8, device="cuda")
    vcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    app, cpy = torch.cuda.Stream(), torch.cuda.Stream()
    flags = phos.V_READS | phos.V_WRITES | phos.V_TRACK
    log(f"[bench] CoW staging: {w.n_alloc} buffers, {nimg / 2**30:.2f} GiB host image, "
        f"{n_launch} launches x {n_rec} accesses")

    def loop(ck):
        phos.phos_validate_batch(ctx, specs, rec_ptrs, [n_rec] * n_launch, flags, vout, lcap,
                                 vcnt.data_ptr(), app)
        for j, L in enumerate(launches):
            if ck is not None:
                phos.phos_ckpt_cow(ck, specs[j], app)
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_ptrs[j], n_rec, app)

    def fresh():
        synth.content_device(pool, w.seed)
        torch.cuda.synchronize()

    t = Timer(torch, app)
    alone = []
    for _ in range(2):
        fresh()
        t.start()
        loop(None)
        t.stop()
        app.synchronize()
        alone.append(t.ms())
    alone_ms = float(np.median(alone))
    log(f"[bench] launches without a checkpoint: {alone_ms:.2f} ms")
    # sampled image pages checked against the pool at t1
    rng = np.random.default_rng(8)
    img_off = np.concatenate([[0], np.cumsum(w.alloc_bytes.astype(np.int64))])
    samples = rng.integers(0, nimg // page, 2048)
    rows, rows_block = {}, {}
    policies = [x for x in args.stage_policies.split(",") if x]
    cases = [(pol, int(mib)) for mib in args.budgets.split(",") for pol in policies
             if pol == "host_direct" or int(mib) > 0]
    for pol, mib in cases:
        fresh()
        snap.copy_(pool)
        torch.cuda.synchronize()
        ck = phos.phos_ckpt_begin(ctx, phos.COW, 0, himg.data_ptr(), None, cpy)
        phos.phos_ckpt_staging_policy(ck, staging, min(mib << 20, nimg),
                                      phos.STAGE_BLOCK if pol == "block" else phos.STAGE_HOST_DIRECT)
        t.start()
        loop(ck)
        t.stop()
        t0 = time.perf_counter()
        st = phos.phos_ckpt_end(ck, app)
        end_s = time.perf_counter() - t0
        loop_ms = t.ms()
        ok = True
        for p in samples.tolist():
            b = int(np.searchsorted(img_off, p * page, side="right") - 1)
            src = int(w.alloc_off[b]) + p * page - int(img_off[b])
            ok &= bool(torch.equal(himg[p * page:(p + 1) * page],
                                   snap[src:src + page].cpu()))
        assert ok, f"host image differs from the pool at t1 ({pol}, budget {mib} MiB)"
        row = {"loop_ms": round(loop_ms, 2), "stall_ms": round(loop_ms - alone_ms, 2),
               "cow_pages": int(st.cow_pages), "staged_pages": int(st.staged_pages),
               "background_pages": int(st.bg_pages), "end_s": round(end_s, 3)}
        if pol == "block":
            row["drain_batches"] = int(st.stage_batches)
        (rows_block if pol == "block" else rows)[mib] = row
        log(f"[bench] {pol}, budget {mib} MiB: {row}")
    phos.phos_destroy(ctx)
    if not rows:
        rows = rows_block
    first = rows[min(rows)]
    return {
        "metric": "copy-on-write stall of the launches (ms per step) vs the device staging budget",
        "value": rows[max(rows)]["stall_ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": rows[max(rows)]["loop_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded layout, access streams and contents)",
        "config": {"workload": "CoW staging: training-step layout, 1000 launches x 1e6 accesses, "
                               "16 GiB pinned host image, budgets " + args.budgets + " MiB"},
        "launches_without_checkpoint_ms": round(alone_ms, 2),
        # a full area: copies go straight to the host image (host_direct), or
        # wait for a slot the host's copy-engine drain frees (block)
        "by_budget_mib": rows, "by_budget_mib_block": rows_block,
        "stall_ms_without_staging": first["stall_ms"],
        "parity": "2048 sampled image pages equal the pool at t1 for every budget and policy",
    }


def run_cow(args):
    """Section 4.2 soft copy-on-write into a device image, on the training-step
    layout and launches.  Before each launch the pages of its write intervals,
    and the pages its violating writes hit inside buffers, are copied into the
    image unless already copied.  The access streams are validated once the
    checkpoint is open, before the timed launches.  Two orders: the background
    copy deferred until the launches are done (every page they write goes
    through copy-on-write: the worst case for the stall), and the background
    copy started with the launches, running beside them.
    Reports each launch's copy-on-write time (HIP events around the call on
    the application stream), the pages copied, their rate against HBM peak,
    and the launches' loop time against the same loop with no checkpoint.
    Parity: the image equals the pool at t1, copied buffer by buffer with
    torch (a stop-the-world snapshot)."""
    import torch

    import synth
    from paper_2405_12079_amd import phos

    torch.cuda.set_device(0)
    w = synth.config2_world()
    n_launch, n_rec = args.launches, 1_000_000
    launches = synth.config2_launches(w, n_launch, n_rec)
    page = w.page_bytes
    back = torch.empty(w.pool_bytes + page, dtype=torch.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    pool = back[base - back.data_ptr(): base - back.data_ptr() + w.pool_bytes]
    synth.content_device(pool, w.seed)
    dw = synth.DeviceWorld(w, base)
    recs = torch.empty(n_launch * n_rec, dtype=torch.int64, device="cuda")
    for g in range(0, n_launch, 100):
        synth.records_device(dw, launches[g:g + 100], n_rec, out=recs[g * n_rec:(g + 100) * n_rec])
    ctx = phos.phos_create(0, base, w.pool_bytes, page)
    phos.phos_buffers_register(ctx, w.buffers(base))
    nimg = phos.phos_image_bytes(ctx)
    img = torch.empty(nimg, dtype=torch.uint8, device="cuda")
    snap = torch.empty(nimg, dtype=torch.uint8, device="cuda")
    specs = [phos.phos_spec_register(ctx, L.k, L.arg_values(base)) for L in launches]
    rec_ptrs = [recs.data_ptr() + j * n_rec * 8 for j in range(n_launch)]
    lcap = 2_000_000
    vout = torch.empty(lcap * 32, dtype=torch.uint8, device="cuda")
    vcnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    app, cpy = torch.cuda.Stream(), torch.cuda.Stream()
    log(f"[bench] copy-on-write: {w.n_alloc} buffers, {nimg / 2**30:.2f} GiB device image, "
        f"{n_launch} launches x {n_rec} accesses")
    # pages of the launches' write intervals inside buffers (the deferred
    # order copies these and the victim pages of violating writes)
    inbuf = np.zeros(w.n_pages, bool)
    for off, nb in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
        inbuf[off // page:(off + nb) // page] = True
    wpages = np.zeros(w.n_pages, bool)
    for sp in specs:
        for iv in phos.phos_spec_intervals(ctx, sp):
            lo, hi = max(int(iv["lo"]), base), min(int(iv["hi"]), base + w.pool_bytes)
            if int(iv["mode"]) & phos.W and hi > lo:
                wpages[(lo - base) // page:(hi - base + page - 1) // page] = True
    n_wpages = int((wpages & inbuf).sum())
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_launch)]

    def loop(ck):
        for j, L in enumerate(launches):
            if ck is not None:
                ev[j][0].record(app)
                phos.phos_ckpt_cow(ck, specs[j], app)
                ev[j][1].record(app)
            synth.apply_writes_device(base, base, w.pool_bytes, w.seed, L.k, rec_ptrs[j], n_rec, app)

    def snapshot():
        o = 0
        for off, nb in zip(w.alloc_off.tolist(), w.alloc_bytes.tolist()):
            snap[o:o + nb].copy_(pool[off:off + nb])
            o += nb
        torch.cuda.synchronize()

    t = Timer(torch, app)
    alone = []
    for _ in range(3):
        t.start()
        loop(None)
        t.stop()
        app.synchronize()
        alone.append(t.ms())
    alone_ms = float(np.median(alone[1:]))
    log(f"[bench] launches without a checkpoint: {alone_ms:.2f} ms")
    rows = {}
    for mode in ("deferred", "concurrent"):
        runs = []
        for rep in range(max(1, args.warmup) + max(1, args.steps)):
            snapshot()
            # opening resets the victim list, so the streams are validated
            # after it; the background copy starts once they are
            ck = phos.phos_ckpt_begin(ctx, phos.COW, phos.CKPT_DEFER_BACKGROUND, img, None, cpy)
            phos.phos_validate_batch(ctx, specs, rec_ptrs, [n_rec] * n_launch,
                                     phos.V_READS | phos.V_WRITES | phos.V_TRACK, vout, lcap,
                                     vcnt.data_ptr(), app)
            if mode == "concurrent":
                phos.phos_ckpt_start(ck, app)
            t.start()
            loop(ck)
            t.stop()
            if mode == "deferred":
                phos.phos_ckpt_start(ck, app)
            st = phos.phos_ckpt_end(ck, app)
            torch.cuda.synchronize()
            assert torch.equal(img, snap), f"image != pool at t1 ({mode})"
            cow_ms = np.array([a.elapsed_time(b) for a, b in ev])
            if rep >= max(1, args.warmup):
                runs.append((t.ms(), cow_ms, int(st.cow_pages), int(st.bg_pages)))
        loop_ms = float(np.median([r[0] for r in runs]))
        cow_ms = np.concatenate([r[1] for r in runs])
        cow_pages = int(np.median([r[2] for r in runs]))
        total_cow_ms = float(np.median([r[1].sum() for r in runs]))
        gbps = 2 * cow_pages * page / (total_cow_ms / 1e3) / 1e9 if total_cow_ms else 0.0
        rows[mode] = {
            "loop_ms": round(loop_ms, 3), "stall_ms": round(loop_ms - alone_ms, 3),
            "cow_pages": cow_pages, "background_pages": int(np.median([r[3] for r in runs])),
            "cow_call_ms": {"p50": round(float(np.percentile(cow_ms, 50)), 4),
                            "p99": round(float(np.percentile(cow_ms, 99)), 4),
                            "max": round(float(cow_ms.max()), 4),
                            "sum": round(total_cow_ms, 3)},
            "cow_GBps_hbm": round(gbps, 1),
        }
        log(f"[bench] {mode}: {rows[mode]}")
    phos.phos_destroy(ctx)
    d = rows["deferred"]
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's copy-on-write snapshot of the write-interval pages in the
        # pool's first 2 GiB, each to its place in the image
        cap = 2 << 30
        img_off = np.concatenate([[0], np.cumsum(w.alloc_bytes.astype(np.int64))])
        sel = np.flatnonzero((wpages & inbuf)[:cap // page])
        so, do, ln = [], [], []
        for pg in sel.tolist():
            b = int(np.searchsorted(w.alloc_off, pg * page, side="right") - 1)
            dst = int(img_off[b]) + pg * page - int(w.alloc_off[b])
            if so and so[-1] + ln[-1] == pg * page and do[-1] + ln[-1] == dst:
                ln[-1] += page
            else:
                so.append(pg * page)
                do.append(dst)
                ln.append(page)
        if so:
            cpu = cpu_gather_baseline(w.seed, cap, so, do, ln,
                                      "write-interval pages of the pool's first 2 GiB to the image")
    return {
        "metric": "copy-on-write copy rate (HBM GB/s over the copy-on-write calls) and the "
                  "launches' stall",
        "value": d["cow_GBps_hbm"], "unit": "GB/s", "n_gpus": 1, "steps": max(1, args.steps),
        "warmup": max(1, args.warmup), "ms_per_step": d["loop_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded layout, access streams and contents)",
        "config": {"workload": "copy-on-write: training-step layout, 1000 launches x 1e6 accesses, "
                               "16 GiB device image, background deferred / beside"},
        # traffic: HBM bytes of the copy-on-write kernels of one deferred loop
        "roofline": {"bound": "hbm", "kernel": "cow_kernel (background deferred)",
                     "achieved": d["cow_GBps_hbm"], "peak": 8000.0, "unit": "GB/s",
                     "frac": round(d["cow_GBps_hbm"] / 8000.0, 4),
                     "traffic": measured_traffic("cow_kernel", "copy_on_write",
                                                 "traffic_bytes_per_loop"),
                     "algorithmic_bytes": 2 * d["cow_pages"] * page},
        "launches_without_checkpoint_ms": round(alone_ms, 3),
        "write_interval_pages": n_wpages,
        "by_order": rows,
        "parity": "the image equals the pool at t1 (whole image, every run)",
        "cpu_baseline": cpu,
    }


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--launches", type=int, default=1000)
    ap.add_argument("--val-chunk", type=int, default=1000,
                    help="launches validated per batched validation call inside the step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launches5", type=int, default=40_000)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--quantum", type=int, default=2048, help="MiB per request per iteration")
    ap.add_argument("--iter-mib", type=int, default=2048, help="MiB per batched iteration")
    ap.add_argument("--small-mib", type=int, default=1024,
                    help="batched order: requests with at most this many MiB left go first")
    ap.add_argument("--twin-n", type=int, default=1 << 28, help="elements per array (config 6)")
    ap.add_argument("--copy-start", dest="copy_start", default="cow",
                    choices=("begin", "validation", "cow"),
                    help="config 2: when the background copies start: with the checkpoints "
                         "(begin), after the first validation pass (validation), or after launch "
                         "0's copy-on-write, which takes the pages the first launches hit with "
                         "failing writes (cow)")
    ap.add_argument("--pipelined-validation", dest="pipelined_validation", action="store_true",
                    help="config 2: validate the launch chunks on their own stream ahead of the "
                         "launches (use with --val-chunk)")
    ap.add_argument("--precopy", action="store_true",
                    help="config 2: a pre-copy round of the recopy image before each validation "
                         "chunk after the first (iterative recopy; use with --val-chunk)")
    ap.add_argument("--final-at", dest="final_at", default="300,600,800,900,970,995",
                    help="config 2: launch positions before which a pre-copy round copies the "
                         "dirty pages no remaining launch may write ('' for none)")
    ap.add_argument("--budgets", default="0,256,1024,2048,8192,16384",
                    help="config 8: staging budgets in MiB")
    ap.add_argument("--stage-policies", default="host_direct,block",
                    help="config 8: policies for a full staging area (host_direct, block)")
    ap.add_argument("--no-parity", dest="parity", action="store_false")
    ap.add_argument("--shared-pass", dest="separate_passes", action="store_false",
                    help="config 2: one shared background pass for both images (one read per "
                         "page) instead of one pass per image")
    ap.add_argument("--step-only", dest="step_only", action="store_true",
                    help="config 2: only the training step (no plain-tiny validation rate and "
                         "no batched-uneven latency beside it)")
    ap.add_argument("--app-graph", action="store_true",
                    help="replay the per-launch copy-on-write + application loop as one HIP "
                         "graph (eager is faster: it skips copy-on-write once the background "
                         "copy is known done)")
    return ap.parse_args(argv)


def main():
    args = parse_args()
    if args.pipelined_validation:
        if args.app_graph or args.precopy:
            sys.exit("--pipelined-validation runs alone (no --app-graph, --precopy)")
        args.copy_start = "begin"
    if args.final_at and (args.app_graph or args.pipelined_validation):
        # a round builds its page mask on the host at the call
        log("[bench] final-page pre-copy rounds are off with --app-graph / --pipelined-validation")
        args.final_at = ""
    if args.app_graph and args.copy_start != "begin":
        log("[bench] --app-graph starts the background copies with the checkpoints")
        args.copy_start = "begin"
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the hot path is per GPU and shards by process "
              f"(one pool per GPU), so --gpus {args.gpus} is not run.", file=sys.stderr)
        sys.exit(2)
    if args.config == 2:
        res = run_training_step(args)
        if not args.step_only:
            # the metric's other two parts, on their own workloads
            res["plain_tiny_validation"] = config1_validation_rate()
            log(f"[bench] plain tiny validation: {res['plain_tiny_validation']}")
            b = run_batched(parse_args(["--config", "3", "--steps", "5", "--warmup", "1",
                                        "--no-parity", "--no-cpu-baseline"]))
            res["batched_uneven"] = {k: b[k] for k in ("config", "batched_ms", "plain_ms",
                                                       "latency_ms", "tuned", "roofline")}
            res["batched_uneven"]["steps"] = 5
            log(f"[bench] batched uneven: {res['batched_uneven']['latency_ms']}")
    elif args.config == 3:
        res = run_batched(args)
    elif args.config == 4:
        res = run_serving(args)
    elif args.config == 5:
        res = run_cold_start(args)
    elif args.config == 6:
        res = run_twin(args)
    elif args.config == 7:
        res = run_drain(args)
    elif args.config == 8:
        res = run_staging(args)
    elif args.config == 9:
        res = run_cow(args)
    else:
        sys.exit(f"unknown config {args.config}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
