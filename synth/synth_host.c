/*
 * synth_host.c — host (CPU) side of the seeded synthetic workload generator.
 * Inputs only: access records, initial pool contents and the values the
 * synthetic application stores.  See synth_gen.h for the definitions.
 */
#include <string.h>
#include "synth_gen.h"

/* Records i0 .. i0+n-1 of launch k (out[j] = record i0+j). */
void synth_records_host(const synth_world *W, const synth_launch *L, uint32_t k, uint64_t i0,
                        uint64_t n, uint64_t *out) {
  uint64_t ki = synth_key(W->seed, SYNTH_T_INJ, k), kk = synth_key(W->seed, SYNTH_T_KIND, k);
  uint64_t kp = synth_key(W->seed, SYNTH_T_POS, k), kr = synth_key(W->seed, SYNTH_T_RW, k);
  uint64_t k2 = synth_key(W->seed, SYNTH_T_POS2, k);
  uint64_t j;
  for (j = 0; j < n; ++j) out[j] = synth_record(W, L, ki, kk, kp, kr, k2, i0 + j);
}

/* Initial contents of pool bytes [byte0, byte0 + nbytes), both multiples of 4. */
void synth_content_host(uint64_t seed, uint64_t byte0, uint64_t nbytes, uint8_t *out) {
  uint64_t key = synth_key(seed, SYNTH_T_CONTENT, 0);
  uint64_t w0 = byte0 >> 2, nw = nbytes >> 2, j;
  for (j = 0; j < nw; ++j) {
    uint32_t v = synth_content_word(key, w0 + j);
    memcpy(out + 4 * j, &v, 4);
  }
}

/* The synthetic application's launch k: every write record stores its value.
 * Records outside [pool_base, pool_base + pool_bytes) are ignored. */
void synth_apply_writes_host(uint8_t *pool, uint64_t pool_base, uint64_t pool_bytes,
                             uint64_t seed, uint32_t k, const uint64_t *rec, uint64_t n) {
  uint64_t key = synth_key(seed, SYNTH_T_WVAL, k), j;
  for (j = 0; j < n; ++j) {
    uint64_t r = rec[j];
    if (!(r & 1u)) continue;
    uint64_t a = r & ~7ull;
    if (a < pool_base || a - pool_base + 8 > pool_bytes) continue;
    uint64_t off = a - pool_base, v = synth_write_value(key, off);
    memcpy(pool + off, &v, 8);
  }
}

/* Raw generator access for tests. */
uint64_t synth_mix_host(uint64_t z) { return synth_mix(z); }
uint64_t synth_draw_host(uint64_t seed, uint32_t tag, uint64_t a, uint64_t b) {
  return synth_draw(seed, tag, a, b);
}
uint64_t synth_below_host(uint64_t r, uint64_t n) { return synth_below(r, n); }

/* Pages already present (1) before burst r: page p with probability 1/2. */
void synth_present_host(uint64_t seed, uint32_t r, uint64_t n, uint8_t *out) {
  uint64_t key = synth_key(seed, SYNTH_T_PRESENT, r), p;
  for (p = 0; p < n; ++p) out[p] = (uint8_t)(synth_at(key, p) & 1u);
}
