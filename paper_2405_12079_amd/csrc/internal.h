// internal.h — device-side data layout shared by the runtime and the gfx950
// kernels of libphos.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phos.h"

namespace phos {

constexpr uint32_t kMaxIv = 64;          // intervals per speculated set
constexpr uint32_t kNone = 0xFFFFFFFFu;  // "no buffer / no image page"
constexpr uint32_t kFree = 0, kClaimed = 1, kDone = 2;  // per-page copy state
// restore from pageable host memory: the page is held by the host's DMA
// (kHost), or held and asked for by a waiting launch (kWanted)
constexpr uint32_t kHost = 3, kWanted = 4;

// Validation tiling: 256 threads = 4 wave64s; each wave owns a contiguous
// quarter of the tile; each lane reads two records (one 16-byte load) per
// 128-record step, four steps in flight.
constexpr uint32_t kVThreads = 256;
constexpr uint32_t kVWaves = 4;
constexpr uint32_t kVStep = 128;                 // records per wave step
constexpr uint32_t kVUnroll = 4;                 // steps in flight
constexpr uint32_t kVQuantum = kVWaves * kVStep * kVUnroll;  // tile_recs multiple (2048)
constexpr uint32_t kWcap = 256;                  // per-wave violation list in LDS
constexpr uint32_t kVPend = 64;                  // per-wave failing writes kept for the tile's end
constexpr uint32_t kTrackWords = 8192;           // LDS dirty-bitmap words (32 KiB)
constexpr uint32_t kSeg = 1024;                  // tiles per scan segment
constexpr uint32_t kFuseTiles = 4096;            // calls up to this many tiles use one finish kernel

// The fixed workspace of phos_validate_noalloc: one array in device memory
// per GPU, held until the process ends.  Byte offsets: the append cursor and
// the segment sums (8 words, cleared by every call), the tile counts and
// tile offsets of at most kFuseTiles tiles, then kNaViol violation records.
constexpr uint64_t kNaViol = 1ull << 17;                        // 131,072 records (4 MiB)
constexpr uint64_t kNaClearWords = 8;                           // cursor + segment sums
constexpr uint64_t kNaOffCount = 256;
constexpr uint64_t kNaOffTileOff = kNaOffCount + 4ull * kFuseTiles;
constexpr uint64_t kNaOffViol = kNaOffTileOff + 8ull * kFuseTiles;
constexpr uint64_t kNaBytes = kNaOffViol + 32ull * kNaViol;   // 4,243,712 B

// Copy kernels.
constexpr uint32_t kCThreads = 256;
constexpr uint32_t kBgCopyThreads = 512;            // copying waves of a background block
constexpr uint32_t kBgThreads = kBgCopyThreads + 64; // plus one claiming wave
constexpr uint32_t kUnitPages = 4;  // pages per copy-on-write work unit
constexpr uint32_t kVictimUnit = 64;  // victim-list entries per copy-on-write work unit

// Interval in the form the kernel tests: an access at a is inside iff
// (a - lo) <= span (unsigned), span = hi - lo - 8.  Empty-for-8-byte
// intervals get lo = ~0, span = 0.
struct DevIv {
  uint64_t lo, span;
  uint32_t mode, pad;
};
struct DevSpec {
  uint32_t niv, pad;
  DevIv iv[kMaxIv];
};

// One launch's slice of a validation call.
struct VLaunch {
  const uint64_t *rec;
  uint64_t n;
  uint32_t iv_off, niv;  // intervals ivs[iv_off .. iv_off + niv) (batch only)
  uint32_t launch_id, tile0;
};

struct VArgs {
  const VLaunch *launches;  // device table (batch) or nullptr (single launch below)
  VLaunch single;
  const DevIv *ivs;         // flat interval table (batch)
  const uint32_t *tile_launch;  // launch of every tile (batch)
  uint32_t nlaunch, ntiles;
  uint32_t flags, tile_recs;
  uint64_t pool_base, pool_bytes;
  uint32_t page_shift, n_pages;
  const uint32_t *page_buf;  // per pool page: buffer index or kNone
  uint8_t *dirty, *victim;   // page maps: one byte per pool page (padded to 32)
  uint32_t *victim_seq;      // per pool page: the latest launch with a failing write there
  uint32_t *victim_first;    // per pool page: the earliest such launch (~0: none)
  uint32_t seq0;             // sequence number of the call's first launch (then +1 per launch)
  uint32_t *vlist;           // victim pages newly marked (appended)
  uint32_t *vmeta;           // [0] appended, [1] CoW cursor, [2] CoW exit ticket, [3] overflow
  uint32_t vlist_cap;
  phos_violation *scratch;
  uint64_t scratch_cap;
  unsigned long long *cursor;     // scratch append cursor (reset by the scan)
  uint32_t *tile_count;           // violations per tile
  unsigned long long *tile_off;   // scratch offset per tile
  unsigned long long *seg_sum;    // violations per kSeg tiles (reset by the scan)
};

// Page-granular copy between the pool and an image under per-page states.
// Every field defaults to zero / null, so a field added later can never reach
// a kernel as stack garbage.
struct CopyArgs {
  uint8_t *pool = nullptr;               // byte at pool_base
  uint8_t *image = nullptr;              // byte 0 of the image
  uint32_t *state = nullptr;             // per pool page: kFree / kClaimed / kDone
  const uint32_t *img_page = nullptr;    // per pool page: image page or kNone
  unsigned long long *stat = nullptr;    // pages copied by this kernel family
  uint32_t *err = nullptr;               // bit 0: a bounded wait expired
  uint32_t page_shift = 0, n_pages = 0;
  uint32_t to_image = 0;                 // 1: pool -> image (checkpoint); 0: image -> pool (restore)
  uint32_t spin_limit = 0;
  uint32_t nt = 0;                       // non-temporal page copies
  uint32_t deep = 0;                     // copies keep 16 loads in flight per thread
  uint32_t pause_limit = 0;              // background: longest hold (polls) per batch
  uint32_t hold_ticks = 0;               // ... only this long (GPU clock, 100 MHz) after it starts; 0: always
  uint32_t chunk_pages = 0;              // pages per image piece (with image_chunks)
  const unsigned long long *image_chunks = nullptr;  // image pieces (device table) or nullptr
  // Recopy background only: pages already marked in either page map are left
  // to the recopy (nullptr: copy every page).
  const uint8_t *skip_dirty = nullptr, *skip_victim = nullptr;
  // Restore with pageable pieces: a waiter that finds a page held by the
  // host asks for it here (pinned host memory: [0] reservation count, then
  // want_cap entries, written once per page with system-scope atomics so the
  // host sees them at once) and waits for the page's state to become done,
  // which the host publishes with a small kernel after the page's DMA.
  uint32_t *want = nullptr;
  uint32_t want_cap = 0;
  // Checkpoint into a host image: copy-on-write pages go first to a device
  // staging area of stage_cap pages (slots taken in order from *stage_head;
  // stage_page[slot] = the pool page), straight to the host image after.
  uint8_t *stage = nullptr;
  uint32_t *stage_page = nullptr;
  unsigned long long *stage_head = nullptr;
  uint32_t stage_cap = 0;
  // Blocking policy (stage_block = 1): the area is a ring, slot s at position
  // s % stage_cap, drained to the image by the host's copy engines while the
  // checkpoint runs.  A page needing slot s >= stage_cap waits until the
  // drain of slot s - stage_cap has been published (free_seq[pos] reaches
  // s - stage_cap + 1; device memory, written by the copy engine).  A filled
  // slot is published to the host as fill[pos] = (s + 1) << 32 | pool page
  // (pinned host memory, a system-scope store).  A page whose wait gave up
  // goes straight to the image and its slot stays unpublished (the error
  // word records the expiry; the drain then stops there).
  uint32_t stage_block = 0;
  uint64_t *fill = nullptr;
  uint32_t *free_seq = nullptr;
  // Restore: blocks copying pages a launch needs now (on demand) count
  // themselves here while they copy; the background copy claims no new
  // pages while it is nonzero, so on-demand copies get the link first.
  unsigned long long *demand = nullptr;
  // Background copy completion: [0] blocks finished, [1] set to 1 by the last
  // (a checkpoint's background copy; nullptr: not kept).  Copy-on-write
  // skips its page scan once [1] is set (skip_when_finished).
  unsigned long long *bg_exit = nullptr;
  uint32_t skip_when_finished = 0;
  // Shared background pass of two checkpoints (launch_background_pair): the
  // fields above describe the copy-on-write image (every page); these the
  // recopy image, whose pages already traced as written (skip_dirty,
  // skip_victim) are left to its recopy.
  uint8_t *image2 = nullptr;
  uint32_t *state2 = nullptr;
  unsigned long long *stat2 = nullptr;
  unsigned long long *stat_read = nullptr;  // pool pages the shared pass read
};

// Pages [p0, p0 + np) per range, in work units of kUnitPages.
struct PageRanges {
  uint32_t n, pad;
  uint32_t units_prefix[kMaxIv + 1];
  uint32_t p0[kMaxIv];
  uint32_t np[kMaxIv];
};

// Victim pages for copy-on-write: the list validation appends to (and the
// page map, scanned if the list overflowed).
struct VictimList {
  const uint32_t *list;
  uint32_t *meta;  // as VArgs::vmeta; nullptr: no victim work
  uint32_t cap;
  const uint8_t *map;
  uint32_t map_words;
  // 1: scan the whole map and leave the list and its cursor alone (the
  // caller cannot order the list's appends before this launch)
  uint32_t scan_map;
  // Non-null: the launch's own bucket of victim pages, bucket[*bstart ..
  // *bend) (the pages whose earliest failing write is this launch's), in
  // place of the appended list; the list's cursor is left alone.
  const uint32_t *bucket = nullptr;
  const uint32_t *bstart = nullptr, *bend = nullptr;
};

// Batched-copy work queue: segments, exclusive byte prefix, a chunk cursor.
struct BatchQ {
  const phos_copy_seg *segs;
  const unsigned long long *byte_prefix;  // nseg + 1 entries
  const unsigned long long *hdr;          // [0] nseg, [1] total bytes, [2] requests
  unsigned long long *cursor;             // next chunk (reset before each drain)
  unsigned long long *done;               // per request: bytes copied
  const unsigned long long *req_total;    // per request: bytes to copy (or nullptr)
  unsigned long long *req_time;           // per request: completion stamp; [-1] = start
  uint64_t chunk_bytes;
};

// A twin kernel (Section 4.1): an application kernel, y[j] <- 3 * y[j] + x[i]
// with j = idx[i] (or i), whose instrumented twin checks every global access
// against the speculated intervals before making it.
struct TwinArgs {
  const uint64_t *x;
  uint64_t *y;
  const int64_t *idx;  // element offsets from y, or nullptr (j = i)
  uint64_t n;
  uint32_t flags, launch_id;  // PHOS_V_* (0: the uninstrumented kernel)
  uint64_t pool_base, pool_bytes;
  uint32_t page_shift, vlist_cap;
  const uint32_t *page_buf;
  uint8_t *dirty, *victim;
  uint32_t *victim_seq;  // as VArgs
  uint32_t seq;          // this launch's sequence number
  uint32_t *vlist, *vmeta;
  phos_violation *out;  // unordered
  uint64_t cap;
  unsigned long long *count;
  uint32_t *overflow;          // set to 1 when the count exceeds cap (sticky)
  // an open copy-on-write checkpoint's page states (nullptr: none), and the
  // word raised when a failing write lands on a page it has not copied
  const uint32_t *cow_state;
  uint32_t *misspec;
};

// ---------------------------------------------------------------- launchers
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_validate(const VArgs &a, const DevSpec *single, bool track, hipStream_t s);
// overflow: optional word set to 1 (sticky) when the call's count exceeds cap
hipError_t launch_vscan(unsigned long long *seg_sum, uint32_t nseg, unsigned long long *seg_prefix,
                        uint64_t *n_out, unsigned long long *cursor, uint64_t cap,
                        uint32_t *overflow, hipStream_t s);
hipError_t launch_vfinish(const uint32_t *tile_count, const unsigned long long *tile_off,
                          uint32_t ntiles, const phos_violation *scratch, uint64_t scratch_cap,
                          phos_violation *out, uint64_t cap, uint64_t *n_out,
                          unsigned long long *cursor, unsigned long long *seg_sum,
                          uint32_t *overflow, hipStream_t s);
hipError_t launch_vscatter(const uint32_t *tile_count, const unsigned long long *tile_off,
                           uint32_t ntiles, const unsigned long long *seg_prefix,
                           const phos_violation *scratch, uint64_t scratch_cap,
                           phos_violation *out, uint64_t cap, hipStream_t s);
// victim_blocks: blocks added for the victim list (its length is only known
// on the device)
hipError_t launch_cow(const CopyArgs &c, const PageRanges &r, const VictimList &v, bool wait,
                      uint32_t max_grid, uint32_t victim_blocks, hipStream_t s);
hipError_t launch_mark_pieces(const uint32_t *img_page, uint32_t *state, uint32_t n_pages,
                              uint32_t chunk_pages, const uint8_t *flag, uint32_t value,
                              unsigned long long *count, hipStream_t s);
hipError_t launch_background(const CopyArgs &c, uint32_t grab, uint32_t batch, uint32_t grid,
                             hipStream_t s);
// One background pass for a copy-on-write and a recopy checkpoint open
// together (device images): each pool page is read once and written to each
// image whose claim this pass won.
hipError_t launch_background_pair(const CopyArgs &c, uint32_t grab, uint32_t batch, uint32_t grid,
                                  hipStream_t s);
// Final pages of a pre-copy round: dirty pages, and victim pages whose
// latest failing write came from a launch numbered <= thr (those are
// unmarked in the victim map), minus the pages of `exclude`.
hipError_t launch_finallist(const uint8_t *dirty, uint8_t *victim, const uint32_t *victim_seq,
                            uint32_t thr, const uint32_t *exclude, uint32_t nwords,
                            uint32_t n_pages, uint32_t *list, unsigned int *count, hipStream_t s);
// exclude: optional word mask (32 pages a word) of pages left out of the list
// Victim buckets of the launches numbered s0 .. s0 + n - 1 (their pages
// appended to the victim list since *seg0), after the list's end at *cursor.
// bse: the n buckets' bounds, interleaved (start, end).  The snapshot, taken
// before the validation, also clears the n counts.
hipError_t launch_vb_snap(const uint32_t *vmeta, uint32_t cap, uint32_t *seg0, uint32_t *bse,
                          uint32_t n, hipStream_t s);
hipError_t launch_vb_build(const uint32_t *vlist, const uint32_t *vmeta, uint32_t cap,
                           const uint32_t *seg0, const uint32_t *victim_first, uint32_t n_pages,
                           uint32_t s0, uint32_t n, uint32_t *bse, uint32_t *cursor,
                           uint32_t *bucket, uint32_t bucket_cap, hipStream_t s);
hipError_t launch_pagelist(const uint8_t *a, const uint8_t *b, uint32_t nwords, uint32_t n_pages,
                           uint32_t *list, unsigned int *count, hipStream_t s,
                           const uint32_t *exclude = nullptr);
hipError_t launch_gather_pages(const CopyArgs &c, const uint32_t *list, const unsigned int *count,
                               uint32_t grid, hipStream_t s);
hipError_t launch_unstage(const CopyArgs &c, uint32_t grid, hipStream_t s);
hipError_t launch_precopy(const CopyArgs &c, const uint32_t *list, const unsigned int *count,
                          uint8_t *dirty, uint32_t grid, hipStream_t s);
hipError_t launch_demand(const CopyArgs &c, const uint64_t *rec, uint64_t n, uint64_t pool_base,
                         unsigned long long *faulted, uint32_t max_grid, hipStream_t s);
hipError_t launch_states_to_bits(const uint32_t *state, uint32_t n_pages, uint32_t *bits,
                                 hipStream_t s);
hipError_t launch_bytes_to_bits(const uint8_t *bytes, uint32_t nwords, uint32_t *bits,
                                hipStream_t s);
hipError_t launch_batch_reset(const BatchQ &q, hipStream_t s);
hipError_t launch_read_clock(unsigned long long *out, hipStream_t s);  // GPU wall clock
hipError_t launch_twin(const TwinArgs &a, const DevSpec &spec, uint64_t blocks, uint32_t n_cu,
                       hipStream_t s);
hipError_t launch_batch_copy(const BatchQ &q, uint32_t grid, uint32_t threads, hipStream_t s);
// Device-resident segments: header, byte prefix and cursor reset (one block);
// bad: word raised when a segment is malformed (the call then copies nothing)
hipError_t launch_segs_prefix(const phos_copy_seg *segs, uint64_t nseg, unsigned long long *hdr,
                              unsigned long long *prefix, unsigned long long *cursor,
                              uint32_t *bad, hipStream_t s);
hipError_t launch_plain_copy(const BatchQ &q, uint64_t nchunks, uint32_t threads, hipStream_t s);

// Device address of this GPU's copy of the fixed validation workspace
// (kNaBytes).  Looked up once per device, which must be current; later calls
// return the kept address.
hipError_t noalloc_workspace(int device, uint8_t **out);

// Completion stamps of a batch's last run ([0] start, [1 + r] request r),
// host-visible (pinned), and the GPU wall-clock rate in kHz.
const volatile unsigned long long *batch_stamps(const phos_batch *b);
// The batch copy's default configuration (environment overrides applied) and
// the configuration check phos_batch_create applies.
phos_batch_cfg batch_default_cfg();
bool batch_cfg_ok(const phos_batch_cfg &c);
double batch_clock_khz(const phos_batch *b);

}  // namespace phos
