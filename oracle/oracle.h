/*
 * oracle.h — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU statement of what the validated-
 * speculation checkpoint/restore hot path computes (PhoenixOS, arXiv
 * 2405.12079).  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this code; the product library never does, and this code
 * shares nothing with it.  Every function is a brute-force definition:
 * linear scans, no blocking, no early exits beyond what the definition says.
 *
 * Readings of the paper where it is silent (all addresses are byte addresses):
 *  - an access record is a 64-bit word: address in bits 3..63 (8-aligned),
 *    bit 0 = write; an access covers [a, a+8) and is inside an interval iff
 *    lo <= a and a + 8 <= hi (half-open intervals);
 *  - a pointer argument "falls within" buffer b iff base_b <= v < base_b + bytes_b;
 *  - a struct argument is a row of 8-byte little-endian chunks, each one a
 *    potential mutable pointer;
 *  - identical intervals are merged by OR-ing their modes; the result is sorted
 *    by (lo, hi).
 */
#ifndef PHOS_ORACLE_H
#define PHOS_ORACLE_H
#include <stdint.h>

enum { ORC_R = 1u, ORC_W = 2u };
enum { ORC_ARG_SCALAR = 0, ORC_ARG_PTR_CONST = 1, ORC_ARG_PTR_MUT = 2, ORC_ARG_STRUCT = 3,
       ORC_ARG_RANGE = 4 };
enum { ORC_V_READS = 1u, ORC_V_WRITES = 2u };
enum { ORC_REASON_NO_INTERVAL = 1, ORC_REASON_MODE = 2 };

typedef struct { uint64_t lo, hi; uint32_t mode, _pad; } orc_interval;
typedef struct { uint32_t kind, mode; uint64_t value, bytes; const void *host_struct; } orc_arg;
typedef struct {
  uint64_t index, addr;
  uint32_t launch_id;
  uint8_t is_write, reason;
  uint16_t _p;
  int32_t victim;
  uint32_t _q;
} orc_violation;

/* Speculated interval set of one launch (Section 4.1, "Tracing with speculation
 * on GPU API arguments", signature filtering, API-specified ranges; Section 6,
 * read-set speculation).  Returns the number of intervals (<= cap written). */
uint32_t orc_spec_build(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc,
                        const orc_arg *args, uint32_t nargs, orc_interval *out, uint32_t cap);

/* Section 4.1 "Runtime validation": 0 = valid, else ORC_REASON_*. */
int orc_check(const orc_interval *iv, uint32_t niv, uint64_t addr, int is_write);

/* Index of the allocated buffer containing addr, or -1 (linear scan). */
int32_t orc_victim(const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc, uint64_t addr);

/* Violations of one launch's records in ascending index order.  Returns the
 * number of violations; at most cap are written. */
uint64_t orc_validate(const orc_interval *iv, uint32_t niv, const uint64_t *rec, uint64_t n,
                      uint32_t flags, uint32_t launch_id, const uint64_t *abase,
                      const uint64_t *abytes, uint32_t nalloc, orc_violation *out, uint64_t cap);

/* Write-set tracking of one launch (Section 4.3): dirty[p] |= 1 for every page p
 * holding a write that passes validation; victim[p] |= 1 for every page p
 * holding a write that fails validation and lies inside an allocated buffer.
 * One byte per page; page index = (a - pool_base) / page_bytes. */
void orc_track(const orc_interval *iv, uint32_t niv, const uint64_t *rec, uint64_t n,
               const uint64_t *abase, const uint64_t *abytes, uint32_t nalloc, uint64_t pool_base,
               uint64_t page_bytes, uint64_t n_pages, uint8_t *dirty, uint8_t *victim);

/* Pages of the launch's write intervals (one byte per page, OR-ed in). */
void orc_write_interval_pages(const orc_interval *iv, uint32_t niv, uint64_t pool_base,
                              uint64_t page_bytes, uint64_t n_pages, uint8_t *pages);

/* Section 6: pages a launch touches (reads or writes) inside allocated buffers. */
void orc_touched_pages(const uint64_t *rec, uint64_t n, const uint64_t *abase,
                       const uint64_t *abytes, uint32_t nalloc, uint64_t pool_base,
                       uint64_t page_bytes, uint64_t n_pages, uint8_t *pages);

/* Section 2.2 data state: the checkpoint image is every buffer's bytes, in
 * ascending base order, back to back (gaps excluded).  pool points at the
 * byte whose address is pool_base.  Returns image bytes written. */
uint64_t orc_snapshot(const uint8_t *pool, uint64_t pool_base, const uint64_t *abase,
                      const uint64_t *abytes, uint32_t nalloc, uint8_t *image);

/* Inverse of orc_snapshot: write the image's bytes back into the buffers. */
void orc_restore(uint8_t *pool, uint64_t pool_base, const uint64_t *abase,
                 const uint64_t *abytes, uint32_t nalloc, const uint8_t *image);

/* Gather copy: dst[dst_off[i] .. +bytes[i]) = src[src_off[i] .. +bytes[i]). */
void orc_gather(const uint8_t *src, uint8_t *dst, const uint64_t *src_off,
                const uint64_t *dst_off, const uint64_t *bytes, uint64_t nseg);

/* Page fingerprints for comparing images too large to hold twice: a 64-bit
 * hash of one page's bytes, keyed by its page index (so equal content at two
 * different places hashes differently).  The splitmix64 output function
 * (Steele, Lea and Flood, OOPSLA 2014) is folded over the page's 8-byte
 * little-endian words in order: h <- mix(h ^ word) + golden, starting from
 * mix(golden * (index + 1)).  page_bytes is a multiple of 8. */
uint64_t orc_page_hash(const uint8_t *page, uint64_t page_bytes, uint64_t index);

/* out[i] = orc_page_hash(buf + i * page_bytes, page_bytes, index0 + i), i < npages. */
void orc_hash_pages(const uint8_t *buf, uint64_t page_bytes, uint64_t npages, uint64_t index0,
                    uint64_t *out);

#endif
