/*
 * synth_gen.h — seeded synthetic workload generator (inputs only).
 *
 * This header holds NO checkpoint/restore arithmetic: it only describes the
 * synthetic application whose memory is checkpointed — its buffer layout, its
 * per-launch access streams (8-byte records "address | is_write"), the initial
 * pool contents and the values its kernels write.  The same inline functions
 * compile for the host (C, gcc) and for the device (HIP, gfx950), so the CPU
 * oracle and the GPU harness draw bit-identical inputs without moving them.
 *
 * Generator: the splitmix64 output function (Steele, Lea, Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) applied to a
 * Weyl-sequence counter, with the 64-bit golden-ratio increment.  Bounded
 * integers use Lemire's multiply-high reduction ("Fast random integer
 * generation in an interval", ACM TOMACS 2019): floor(r * n / 2^64).
 *
 * All addresses inside the structures below are offsets relative to the pool
 * base; the pool base is added only when a record is emitted, so every stored
 * value and every written word depends on pool-relative offsets alone.
 */
#ifndef SYNTH_GEN_H
#define SYNTH_GEN_H

#include <stdint.h>

#if defined(__HIPCC__)
#define SYNTH_FN __host__ __device__ static inline
#else
#define SYNTH_FN static inline
#endif

#define SYNTH_GOLDEN 0x9E3779B97F4A7C15ull
#define SYNTH_MAX_NAMED 8

/* Stream tags (one independent stream per purpose). */
enum {
  SYNTH_T_INJ = 1,     /* is access i of launch k injected out of spec?  */
  SYNTH_T_KIND = 2,    /* which kind of injected access                  */
  SYNTH_T_POS = 3,     /* position draw                                  */
  SYNTH_T_RW = 4,      /* read / write draw                              */
  SYNTH_T_POS2 = 5,    /* secondary position draw (offset inside buffer) */
  SYNTH_T_CONTENT = 6, /* initial pool contents                          */
  SYNTH_T_WVAL = 7,    /* value stored by the application's writes       */
  SYNTH_T_PRESENT = 8  /* pages already present before a restore burst   */
};

/* splitmix64 output function. */
SYNTH_FN uint64_t synth_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Key of the sub-stream (seed, tag, a); draws are synth_at(key, b). */
SYNTH_FN uint64_t synth_key(uint64_t seed, uint32_t tag, uint64_t a) {
  uint64_t s = synth_mix(seed + SYNTH_GOLDEN * ((uint64_t)tag + 1u));
  return synth_mix(s + SYNTH_GOLDEN * (a + 1u));
}
SYNTH_FN uint64_t synth_at(uint64_t key, uint64_t b) {
  return synth_mix(key + SYNTH_GOLDEN * (b + 1u));
}
SYNTH_FN uint64_t synth_draw(uint64_t seed, uint32_t tag, uint64_t a, uint64_t b) {
  return synth_at(synth_key(seed, tag, a), b);
}

/* floor(r * n / 2^64) — Lemire's reduction to [0, n). */
SYNTH_FN uint64_t synth_below(uint64_t r, uint64_t n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(r, n);
#else
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
#endif
}

/* The application's world: buffers and free space, pool-relative. */
typedef struct {
  uint64_t seed;
  uint64_t pool_base;      /* absolute address added to every record   */
  uint64_t inj_threshold;  /* access injected iff draw < inj_threshold */
  uint32_t n_alloc;
  uint32_t n_free;
  const uint64_t *alloc_off;   /* [n_alloc] ascending buffer offsets     */
  const uint64_t *alloc_bytes; /* [n_alloc] buffer sizes (multiples of 8) */
  const uint64_t *free_off;    /* [n_free] free intervals (gaps + tail)  */
  const uint64_t *free_cum;    /* [n_free] exclusive prefix of free bytes */
  uint64_t free_total;         /* total free bytes                        */
} synth_world;

/* One launch's named buffers, in the order the launch names them. */
typedef struct {
  uint32_t n_named;
  uint32_t n_const;                       /* named read-only buffers        */
  uint64_t named_bytes_total;
  uint64_t const_bytes_total;
  uint64_t named_off[SYNTH_MAX_NAMED];
  uint64_t named_bytes[SYNTH_MAX_NAMED];
  uint32_t named_mut[SYNTH_MAX_NAMED];    /* 1 = named through a mutable pointer */
  uint32_t named_idx_sorted[SYNTH_MAX_NAMED]; /* allocation indices, ascending */
} synth_launch;

/* Offset of the byte at position `pos` of the concatenation of the named
 * buffers selected by `want_const` (0 = all named, 1 = only read-only). */
SYNTH_FN uint64_t synth_named_pos(const synth_launch *L, uint64_t pos, int want_const,
                                  uint32_t *which) {
  uint32_t j;
  for (j = 0; j < L->n_named; ++j) {
    if (want_const && L->named_mut[j]) continue;
    if (pos < L->named_bytes[j]) { *which = j; return L->named_off[j] + pos; }
    pos -= L->named_bytes[j];
  }
  *which = 0;
  return L->named_off[0]; /* unreachable for pos < total */
}

/*
 * Record i of launch k.  Non-injected accesses are uniform 8-aligned positions
 * over the named buffers; they write (probability 1/2) only buffers named
 * through a mutable pointer.  Injected accesses (probability
 * inj_threshold / 2^64) are, by kind: (0) a write into a read-only named
 * buffer, (1) a read or write into an allocated but unnamed buffer, (2) a read
 * or write into free space; an infeasible kind falls through to the next one.
 * key_* are synth_key(seed, tag, k) for the tags named in each parameter.
 */
SYNTH_FN uint64_t synth_record(const synth_world *W, const synth_launch *L, uint64_t key_inj,
                               uint64_t key_kind, uint64_t key_pos, uint64_t key_rw,
                               uint64_t key_pos2, uint64_t i) {
  uint64_t off = 0, w = 0;
  uint32_t which = 0;
  int done = 0;
  if (synth_at(key_inj, i) < W->inj_threshold) {
    uint32_t kind = (uint32_t)synth_below(synth_at(key_kind, i), 3);
    uint32_t t;
    uint64_t rp = synth_at(key_pos, i);
    uint64_t rw = synth_at(key_rw, i) & 1u;
    for (t = 0; t < 3 && !done; ++t) {
      uint32_t kk = (kind + t) % 3u;
      if (kk == 0 && L->n_const > 0 && L->const_bytes_total >= 8) {
        off = synth_named_pos(L, synth_below(rp, L->const_bytes_total >> 3) << 3, 1, &which);
        w = 1;
        done = 1;
      } else if (kk == 1 && W->n_alloc > L->n_named) {
        uint64_t j = synth_below(rp, (uint64_t)(W->n_alloc - L->n_named));
        uint32_t s;
        for (s = 0; s < L->n_named; ++s)
          if (j >= L->named_idx_sorted[s]) ++j;
        off = W->alloc_off[j] +
              (synth_below(synth_at(key_pos2, i), W->alloc_bytes[j] >> 3) << 3);
        w = rw;
        done = 1;
      } else if (kk == 2 && W->free_total >= 8) {
        uint64_t pos = synth_below(rp, W->free_total >> 3) << 3;
        uint32_t lo = 0, hi = W->n_free; /* last f with free_cum[f] <= pos */
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (W->free_cum[mid] <= pos) lo = mid; else hi = mid;
        }
        off = W->free_off[lo] + (pos - W->free_cum[lo]);
        w = rw;
        done = 1;
      }
    }
  }
  if (!done) {
    if (L->n_named == 0 || L->named_bytes_total < 8) {
      /* a launch that names nothing touches free space (or buffer 0) */
      uint64_t rp = synth_at(key_pos, i);
      if (W->free_total >= 8) {
        uint64_t pos = synth_below(rp, W->free_total >> 3) << 3;
        uint32_t lo = 0, hi = W->n_free;
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (W->free_cum[mid] <= pos) lo = mid; else hi = mid;
        }
        off = W->free_off[lo] + (pos - W->free_cum[lo]);
      } else {
        off = W->alloc_off[0] + (synth_below(rp, W->alloc_bytes[0] >> 3) << 3);
      }
      w = synth_at(key_rw, i) & 1u;
    } else {
      off = synth_named_pos(L, synth_below(synth_at(key_pos, i), L->named_bytes_total >> 3) << 3,
                            0, &which);
      w = L->named_mut[which] ? (synth_at(key_rw, i) & 1u) : 0u;
    }
  }
  return (W->pool_base + off) | w;
}

/* Initial content of the 32-bit word at pool-relative word index w. */
SYNTH_FN uint32_t synth_content_word(uint64_t key_content, uint64_t w) {
  return (uint32_t)(synth_at(key_content, w) >> 32);
}

/* Value the application's launch k stores at pool offset `off` (8-aligned);
 * key_wval = synth_key(seed, SYNTH_T_WVAL, k). */
SYNTH_FN uint64_t synth_write_value(uint64_t key_wval, uint64_t off) {
  return synth_at(key_wval, off >> 3);
}

#endif /* SYNTH_GEN_H */
