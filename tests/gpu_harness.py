"""Helpers for the GPU parity tests: device pools, contexts and readbacks.
Inputs come from synth (both sides); expected values from oracle (CPU)."""
import numpy as np

import oracle
import synth


def torch():
    import torch as t
    return t


def alloc_pool(pool_bytes: int, page: int):
    """Device pool whose base is page aligned; returns (backing tensor, view, base)."""
    T = torch()
    back = T.empty(pool_bytes + page, dtype=T.uint8, device="cuda")
    base = (back.data_ptr() + page - 1) // page * page
    off = base - back.data_ptr()
    return back, back[off:off + pool_bytes], base


def u64(t) -> np.ndarray:
    """int64 tensor (uint64 bit patterns) -> numpy uint64."""
    return t.cpu().numpy().view(np.uint64)


class Env:
    """A world on the GPU: pool filled with its initial contents, a libphos
    context with the buffers registered, an app stream and a copy stream."""

    def __init__(self, world, device: int = 0):
        from paper_2405_12079_amd import phos
        T = torch()
        self.T, self.phos, self.world = T, phos, world
        self.back, self.pool, self.base = alloc_pool(world.pool_bytes, world.page_bytes)
        synth.content_device(self.pool, world.seed)
        T.cuda.synchronize()
        self.dw = synth.DeviceWorld(world, self.base)
        self.hw = synth.HostWorld(world, self.base)
        self.table = oracle.Table.from_world(world, self.base)
        self.ctx = phos.phos_create(device, self.base, world.pool_bytes, world.page_bytes)
        phos.phos_buffers_register(self.ctx, world.buffers(self.base))
        self.app = T.cuda.Stream()
        self.copy = T.cuda.Stream()
        self.image_bytes = phos.phos_image_bytes(self.ctx)

    def close(self):
        self.T.cuda.synchronize()
        self.phos.phos_destroy(self.ctx)

    def spec(self, L):
        return self.phos.phos_spec_register(self.ctx, L.k, L.arg_values(self.base))

    def records(self, launches, n_per):
        return synth.records_device(self.dw, launches, n_per)

    def mutate(self, L, rec_ptr, n, stream=None):
        synth.apply_writes_device(self.base, self.base, self.world.pool_bytes, self.world.seed,
                                  L.k, rec_ptr, n, stream if stream is not None else self.app)

    def pool_host(self) -> np.ndarray:
        self.T.cuda.synchronize()
        return self.pool.cpu().numpy()

    def violations_buffers(self, cap):
        T = self.T
        out = T.zeros(max(cap, 1) * 32, dtype=T.uint8, device="cuda")
        cnt = T.zeros(1, dtype=T.int64, device="cuda")
        return out, cnt

    @staticmethod
    def read_violations(out, cnt, cap):
        n = int(cnt.item())
        raw = out.cpu().numpy()[: min(n, cap) * 32]
        from paper_2405_12079_amd import phos
        return n, raw.view(phos.VIOLATION_DTYPE).copy()


def bits_to_pages(words: np.ndarray, n_pages: int) -> np.ndarray:
    b = np.unpackbits(words.view(np.uint8), bitorder="little")[:n_pages]
    return b.astype(np.uint8)
