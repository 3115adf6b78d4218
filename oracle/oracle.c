/*
 * oracle.c — TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C, single thread,
 * linear scans: the definitions of the hot path of validated-speculation
 * concurrent checkpoint/restore (PhoenixOS, arXiv 2405.12079), nothing faster.
 */
#include "oracle.h"

#include <string.h>

/* Index of the buffer whose [base, base + bytes) contains v, or -1. */
static int32_t containing_buffer(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc,
                                 uint64_t v) {
  uint32_t b;
  for (b = 0; b < nalloc; ++b)
    if (abase[b] <= v && v - abase[b] < abytes[b]) return (int32_t)b;
  return -1;
}

/* Section 4.1: an argument value that falls within an allocated buffer names
 * the whole buffer; Section 6: const pointers name read buffers, mutable
 * pointers written buffers (which the kernel may also read). */
static int pointer_interval(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc,
                            uint64_t v, uint32_t mode, orc_interval *iv) {
  int32_t b = containing_buffer(abase, abytes, nalloc, v);
  if (b < 0) return 0;
  iv->lo = abase[b];
  iv->hi = abase[b] + abytes[b];
  iv->mode = mode;
  iv->_pad = 0;
  return 1;
}

static void add_interval(orc_interval *list, uint32_t *n, orc_interval c) {
  uint32_t j;
  for (j = 0; j < *n; ++j)
    if (list[j].lo == c.lo && list[j].hi == c.hi) {
      list[j].mode |= c.mode;
      return;
    }
  list[(*n)++] = c;
}

uint32_t orc_spec_build(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc,
                        const orc_arg *args, uint32_t nargs, orc_interval *out, uint32_t cap) {
  /* every argument yields at most (struct bytes / 8) candidates; count first */
  uint32_t a, total = 0, n = 0, i, j;
  for (a = 0; a < nargs; ++a)
    total += (args[a].kind == ORC_ARG_STRUCT) ? (uint32_t)(args[a].bytes / 8) : 1u;
  orc_interval list[total ? total : 1];
  for (a = 0; a < nargs; ++a) {
    const orc_arg *g = &args[a];
    orc_interval c;
    if (g->kind == ORC_ARG_PTR_CONST) {
      if (pointer_interval(abase, abytes, nalloc, g->value, ORC_R, &c)) add_interval(list, &n, c);
    } else if (g->kind == ORC_ARG_PTR_MUT) {
      if (pointer_interval(abase, abytes, nalloc, g->value, ORC_R | ORC_W, &c))
        add_interval(list, &n, c);
    } else if (g->kind == ORC_ARG_STRUCT) {
      /* an opaque struct: each 8-byte chunk may be a written buffer pointer */
      const uint8_t *s = (const uint8_t *)g->host_struct;
      uint64_t off;
      for (off = 0; s && off + 8 <= g->bytes; off += 8) {
        uint64_t v;
        memcpy(&v, s + off, 8);
        if (pointer_interval(abase, abytes, nalloc, v, ORC_R | ORC_W, &c))
          add_interval(list, &n, c);
      }
    } else if (g->kind == ORC_ARG_RANGE) {
      /* API with a specified write range, e.g. a copy writing [dst, dst + count) */
      if (g->bytes > 0 && (g->mode & (ORC_R | ORC_W)) && g->value + g->bytes > g->value) {
        c.lo = g->value;
        c.hi = g->value + g->bytes;
        c.mode = g->mode & (ORC_R | ORC_W);
        c._pad = 0;
        add_interval(list, &n, c);
      }
    }
    /* scalars name nothing */
  }
  /* sort by (lo, hi): insertion sort */
  for (i = 1; i < n; ++i) {
    orc_interval x = list[i];
    j = i;
    while (j > 0 && (list[j - 1].lo > x.lo || (list[j - 1].lo == x.lo && list[j - 1].hi > x.hi))) {
      list[j] = list[j - 1];
      --j;
    }
    list[j] = x;
  }
  for (i = 0; i < n && i < cap; ++i) out[i] = list[i];
  return n;
}

int orc_check(const orc_interval *iv, uint32_t niv, uint64_t addr, int is_write) {
  uint32_t j;
  int inside = 0, allowed = 0;
  for (j = 0; j < niv; ++j) {
    if (iv[j].hi >= 8 && iv[j].lo <= addr && addr <= iv[j].hi - 8) {
      inside = 1;
      if (is_write ? (iv[j].mode & ORC_W) : (iv[j].mode & ORC_R)) allowed = 1;
    }
  }
  if (allowed) return 0;
  return inside ? ORC_REASON_MODE : ORC_REASON_NO_INTERVAL;
}

int32_t orc_victim(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc, uint64_t addr) {
  return containing_buffer(abase, abytes, nalloc, addr);
}

uint64_t orc_validate(const orc_interval *iv, uint32_t niv, const uint64_t *rec, uint64_t n,
                      uint32_t flags, uint32_t launch_id, const uint64_t *abase,
                      const uint64_t *abytes, uint32_t nalloc, orc_violation *out, uint64_t cap) {
  uint64_t i, nv = 0;
  for (i = 0; i < n; ++i) {
    uint64_t a = rec[i] & ~7ull;
    int w = (int)(rec[i] & 1u);
    int reason;
    if (w && !(flags & ORC_V_WRITES)) continue;
    if (!w && !(flags & ORC_V_READS)) continue;
    reason = orc_check(iv, niv, a, w);
    if (!reason) continue;
    if (nv < cap) {
      orc_violation *v = &out[nv];
      memset(v, 0, sizeof *v);
      v->index = i;
      v->addr = a;
      v->launch_id = launch_id;
      v->is_write = (uint8_t)w;
      v->reason = (uint8_t)reason;
      v->victim = orc_victim(abase, abytes, nalloc, a);
    }
    ++nv;
  }
  return nv;
}

void orc_track(const orc_interval *iv, uint32_t niv, const uint64_t *rec, uint64_t n,
               const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc, uint64_t pool_base,
               uint64_t page_bytes, uint64_t n_pages, uint8_t *dirty, uint8_t *victim) {
  uint64_t i;
  for (i = 0; i < n; ++i) {
    uint64_t a = rec[i] & ~7ull, p;
    if (!(rec[i] & 1u) || a < pool_base) continue;
    p = (a - pool_base) / page_bytes;
    if (p >= n_pages) continue;
    if (orc_check(iv, niv, a, 1) == 0)
      dirty[p] = 1;
    else if (orc_victim(abase, abytes, nalloc, a) >= 0)
      victim[p] = 1;
  }
}

void orc_write_interval_pages(const orc_interval *iv, uint32_t niv, uint64_t pool_base,
                              uint64_t page_bytes, uint64_t n_pages, uint8_t *pages) {
  uint32_t j;
  for (j = 0; j < niv; ++j) {
    uint64_t p, p0, p1;
    if (!(iv[j].mode & ORC_W) || iv[j].hi <= iv[j].lo || iv[j].hi <= pool_base) continue;
    p0 = iv[j].lo < pool_base ? 0 : (iv[j].lo - pool_base) / page_bytes;
    p1 = (iv[j].hi - 1 - pool_base) / page_bytes;
    for (p = p0; p <= p1 && p < n_pages; ++p) pages[p] = 1;
  }
}

void orc_touched_pages(const uint64_t *rec, uint64_t n, const uint64_t *abase,
                       const uint64_t *abytes, uint32_t nalloc, uint64_t pool_base,
                       uint64_t page_bytes, uint64_t n_pages, uint8_t *pages) {
  uint64_t i;
  for (i = 0; i < n; ++i) {
    uint64_t a = rec[i] & ~7ull, p;
    if (a < pool_base || orc_victim(abase, abytes, nalloc, a) < 0) continue;
    p = (a - pool_base) / page_bytes;
    if (p < n_pages) pages[p] = 1;
  }
}

uint64_t orc_snapshot(const uint8_t *pool, uint64_t pool_base, const uint64_t *abase,
                      const uint64_t *abytes, uint32_t nalloc, uint8_t *image) {
  uint64_t off = 0;
  uint32_t b;
  for (b = 0; b < nalloc; ++b) {
    memcpy(image + off, pool + (abase[b] - pool_base), abytes[b]);
    off += abytes[b];
  }
  return off;
}

void orc_restore(uint8_t *pool, uint64_t pool_base, const uint64_t *abase,
                 const uint64_t *abytes, uint32_t nalloc, const uint8_t *image) {
  uint64_t off = 0;
  uint32_t b;
  for (b = 0; b < nalloc; ++b) {
    memcpy(pool + (abase[b] - pool_base), image + off, abytes[b]);
    off += abytes[b];
  }
}

void orc_gather(const uint8_t *src, uint8_t *dst, const uint64_t *src_off,
                const uint64_t *dst_off, const uint64_t *bytes, uint64_t nseg) {
  uint64_t i;
  for (i = 0; i < nseg; ++i) memcpy(dst + dst_off[i], src + src_off[i], bytes[i]);
}

#define ORC_GOLDEN 0x9E3779B97F4A7C15ull

static uint64_t orc_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_page_hash(const uint8_t *page, uint64_t page_bytes, uint64_t index) {
  uint64_t h = orc_mix(ORC_GOLDEN * (index + 1)), off;
  for (off = 0; off + 8 <= page_bytes; off += 8) {
    uint64_t w;
    memcpy(&w, page + off, 8);
    h = orc_mix(h ^ w) + ORC_GOLDEN;
  }
  return h;
}

void orc_hash_pages(const uint8_t *buf, uint64_t page_bytes, uint64_t npages, uint64_t index0,
                    uint64_t *out) {
  uint64_t i;
  for (i = 0; i < npages; ++i) out[i] = orc_page_hash(buf + i * page_bytes, page_bytes, index0 + i);
}
