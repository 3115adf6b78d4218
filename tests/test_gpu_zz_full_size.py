"""Parity at the full sizes of the batched-uneven and cold-start workloads, in
the configuration bench.py times (its own runs, whose checks against the
oracle's host replays raise on a mismatch).  Collected last: they take most of the GPU's
memory (the batched workload ~152 GiB of HBM, the cold start 64 GiB of pinned
host memory), which they hand back before the next test."""
import gc

import pytest

import bench

pytestmark = pytest.mark.gpu


def _release():
    import torch
    gc.collect()
    bench.release_pinned(torch)
    torch.cuda.empty_cache()


def test_batched_uneven_full_size():
    """64 requests, 115 GiB of source images, 37 GiB of deltas: every delta
    page of every request equals the oracle's gather of its segments
    (compared as page fingerprints)."""
    args = bench.parse_args(["--config", "3", "--steps", "1", "--warmup", "0"])
    _release()  # memory the earlier tests left cached
    try:
        res = bench.run_batched(args)
    finally:
        _release()
    assert res["parity"].startswith("hash-equal")
    assert res["batched_ms"] > 0 and res["plain_ms"] > 0


def test_cold_start_full_size():
    """70 GiB image (64 GiB pinned, 6 GiB pageable), 40,000 launches: the
    restored pool plus the launches equals the oracle's restore of the image
    plus the same launches replayed on a host pool, over every buffer page
    (compared as page fingerprints)."""
    args = bench.parse_args(["--config", "5"])
    _release()
    try:
        res = bench.run_cold_start(args)
    finally:
        _release()
    assert res["parity"].endswith("True")
    assert res["time_to_first_kernel_ms"] < res["stop_the_world_restore_ms"]
