/*
 * synth_dev.hip — device (gfx950) side of the seeded synthetic workload
 * generator: access records, initial pool contents and the synthetic
 * application's writes, bit-identical to synth_host.c (same synth_gen.h).
 * Inputs only; nothing here belongs to the checkpoint/restore method.
 */
#include <hip/hip_runtime.h>
#include "synth_gen.h"

extern "C" {

__global__ void synth_records_kernel(synth_world W, const synth_launch *__restrict__ L,
                                     uint32_t k0, uint64_t n_per, uint64_t *__restrict__ out) {
  const uint32_t l = blockIdx.y;
  const synth_launch Ll = L[l];
  const uint32_t k = k0 + l;
  const uint64_t ki = synth_key(W.seed, SYNTH_T_INJ, k), kk = synth_key(W.seed, SYNTH_T_KIND, k);
  const uint64_t kp = synth_key(W.seed, SYNTH_T_POS, k), kr = synth_key(W.seed, SYNTH_T_RW, k);
  const uint64_t k2 = synth_key(W.seed, SYNTH_T_POS2, k);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_per;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[(uint64_t)l * n_per + i] = synth_record(&W, &Ll, ki, kk, kp, kr, k2, i);
}

__global__ void synth_content_kernel(uint32_t *__restrict__ pool, uint64_t nwords, uint64_t key) {
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
       w += (uint64_t)gridDim.x * blockDim.x)
    pool[w] = synth_content_word(key, w);
}

__global__ void synth_apply_writes_kernel(uint8_t *__restrict__ pool, uint64_t pool_base,
                                          uint64_t pool_bytes, uint64_t key,
                                          const uint64_t *__restrict__ rec, uint64_t n) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = rec[j];
    if (!(r & 1u)) continue;
    const uint64_t a = r & ~7ull;
    if (a < pool_base || a - pool_base + 8 > pool_bytes) continue;
    const uint64_t off = a - pool_base;
    *reinterpret_cast<uint64_t *>(pool + off) = synth_write_value(key, off);
  }
}

// Claim words of a burst's pages: page p already present (2) with p = 1/2.
__global__ void synth_present_kernel(uint32_t *state, uint64_t n, uint64_t key) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * blockDim.x)
    state[p] = (synth_at(key, p) & 1u) ? 2u : 0u;
}

static unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

/* Records of launches k0 .. k0+nlaunch-1, n_per each, out[l * n_per + i].
 * W's pointers and L are device pointers.  Returns a hipError_t value. */
int synth_dev_records(const synth_world *W, const synth_launch *d_launches, uint32_t nlaunch,
                      uint32_t k0, uint64_t n_per, uint64_t *d_out, hipStream_t stream) {
  if (nlaunch == 0 || n_per == 0) return 0;
  dim3 grid(grid_for(n_per, 256, 4096), nlaunch);
  hipLaunchKernelGGL(synth_records_kernel, grid, dim3(256), 0, stream, *W, d_launches, k0, n_per,
                     d_out);
  return (int)hipGetLastError();
}

int synth_dev_content(void *d_pool, uint64_t nbytes, uint64_t seed, hipStream_t stream) {
  uint64_t nw = nbytes >> 2;
  if (nw == 0) return 0;
  hipLaunchKernelGGL(synth_content_kernel, dim3(grid_for(nw, 256, 65536)), dim3(256), 0, stream,
                     (uint32_t *)d_pool, nw, synth_key(seed, SYNTH_T_CONTENT, 0));
  return (int)hipGetLastError();
}

int synth_dev_apply_writes(void *d_pool, uint64_t pool_base, uint64_t pool_bytes, uint64_t seed,
                           uint32_t k, const uint64_t *d_rec, uint64_t n, hipStream_t stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(synth_apply_writes_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, stream,
                     (uint8_t *)d_pool, pool_base, pool_bytes, synth_key(seed, SYNTH_T_WVAL, k),
                     d_rec, n);
  return (int)hipGetLastError();
}

int synth_dev_present(uint32_t *d_state, uint64_t n, uint64_t seed, uint32_t r,
                      hipStream_t stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(synth_present_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, stream,
                     d_state, n, synth_key(seed, SYNTH_T_PRESENT, r));
  return (int)hipGetLastError();
}

} /* extern "C" */
