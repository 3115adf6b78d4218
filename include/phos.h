/*
 * phos.h — C ABI of the MI355X (gfx950) hot path of concurrent GPU
 * checkpoint/restore with validated speculation (PhoenixOS, arXiv 2405.12079).
 *
 * Paper map:
 *   Section 4.1  speculation from launch arguments, runtime validation
 *                -> phos_spec_register, phos_validate, phos_validate_batch
 *   Section 4.1  the validator fused into a kernel (twin) -> phos_twin_scale_add
 *   Section 4.2  soft copy-on-write            -> phos_ckpt_begin / _cow / _end,
 *                device staging for a host image -> phos_ckpt_staging
 *   Section 4.3  soft recopy (dirty tracking)   -> PHOS_V_TRACK, phos_ckpt_recopy,
 *                phos_ckpt_start (deferred background copy)
 *   Sections 4.3, 7  iterative recopy           -> phos_ckpt_precopy, phos_ckpt_precopy_final
 *   Section 5    chunked device-to-host drain   -> phos_ckpt_end (host_image)
 *   Section 6    concurrent on-demand restore   -> phos_restore_begin / _on_demand / _end
 *   (no paper analog) batched persistent copy and a serving loop
 *                -> phos_batch_*, phos_copy_plain, phos_copy_batch(_tuned),
 *                   phos_serve_run
 *   Section 2.2  image manifest                 -> phos_manifest_write / _check,
 *                phos_restore_begin_manifest
 *
 * Conventions.  Every call returns a phos_status; nothing throws across the
 * ABI; on failure phos_last_error() holds a thread-local message.  "Device
 * memory" means memory the GPU can dereference (hipMalloc'd, or pinned host
 * memory from hipHostMalloc).  Calls that take a stream are asynchronous on
 * it unless stated; their outputs are valid after that stream synchronizes.
 * A context and its handles are single-threaded: calls on one context must
 * come from one host thread at a time.
 *
 * Addresses.  The application's device memory is one pool [pool_base,
 * pool_base + pool_bytes), split into pages of page_bytes (a power of two,
 * 4 KiB .. 2 MiB); pool_base is page aligned.  Buffers are page-aligned,
 * whole pages, non-overlapping and inside the pool, so every pool page
 * belongs to at most one buffer.  The checkpoint image holds every buffer's
 * bytes back to back in ascending base order (gaps excluded).
 *
 * Access records.  A kernel's access stream is an array of uint64_t records:
 * bits 3..63 are the byte address (8-aligned), bit 0 is 1 for a write; bits
 * 1..2 are ignored.  A record covers [a, a + 8).
 */
#ifndef PHOS_H
#define PHOS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PHOS_OK = 0,
  PHOS_E_INVAL = 1,    /* bad argument: null pointer, misaligned or overlapping buffers, ... */
  PHOS_E_NOMEM = 2,    /* device or pinned host allocation failed                          */
  PHOS_E_HIP = 3,      /* a HIP runtime call failed; phos_last_error() names it            */
  PHOS_E_STATE = 4,    /* call out of protocol order (e.g. cow before begin)               */
  PHOS_E_OVERFLOW = 5, /* more results than the caller's capacity (true count returned)    */
  PHOS_E_MISSPEC = 6,  /* the protocol invariant cannot be kept: fall back to stop-the-world */
  PHOS_E_TIMEOUT = 7   /* a bounded device-side wait expired (results are not valid)        */
} phos_status;

enum { PHOS_R = 1u, PHOS_W = 2u }; /* interval / access mode bits */

/* Launch-argument kinds (Section 4.1: API classes and signature filtering). */
enum {
  PHOS_ARG_SCALAR = 0,    /* not a pointer: names nothing                                 */
  PHOS_ARG_PTR_CONST = 1, /* const pointer: names the containing buffer for reading (R)   */
  PHOS_ARG_PTR_MUT = 2,   /* mutable pointer: names the containing buffer, R|W            */
  PHOS_ARG_STRUCT = 3,    /* opaque struct of `bytes` bytes at host_struct: every 8-byte
                             chunk is treated as a mutable pointer                       */
  PHOS_ARG_RANGE = 4      /* API with a specified range: [value, value + bytes), mode bits */
};

/* Validation flags. */
enum {
  PHOS_V_READS = 1u,  /* report reads outside the read set                            */
  PHOS_V_WRITES = 2u, /* report writes outside the write set                          */
  PHOS_V_TRACK = 4u,  /* set the context's dirty bitmap for validated writes and its
                         victim bitmap for failing writes inside a buffer (Section 4.3) */
  PHOS_V_SYNC = 8u    /* wait for the call (not under stream capture) and return
                         PHOS_E_OVERFLOW if its violations exceed cap                  */
};

enum { PHOS_COW = 1, PHOS_RECOPY = 2 }; /* checkpoint protocols */

/* Checkpoint / restore flags. */
enum {
  PHOS_CKPT_DEFER_BACKGROUND = 1u, /* start the background copy only at phos_ckpt_end
                                      (deterministic copy sets, for testing)            */
  PHOS_RST_DEFER_BACKGROUND = 1u,  /* start the background restore only at phos_restore_end */
  PHOS_RST_PREFETCH_SPEC = 2u      /* also bring in every page of the launch's speculated
                                      buffers, not only the pages its records touch     */
};

typedef struct phos_ctx phos_ctx;
typedef struct phos_ckpt phos_ckpt;
typedef struct phos_rst phos_rst;
typedef struct phos_batch phos_batch;
typedef uint32_t phos_spec; /* handle of a registered interval set */

typedef struct { uint64_t base, bytes; } phos_buffer;
typedef struct {
  uint32_t kind, mode;     /* PHOS_ARG_*; mode bits for PHOS_ARG_RANGE                */
  uint64_t value, bytes;   /* argument value; RANGE/STRUCT byte count                */
  const void *host_struct; /* PHOS_ARG_STRUCT: host copy of the struct's bytes       */
} phos_arg;
typedef struct { uint64_t lo, hi; uint32_t mode, _pad; } phos_interval; /* [lo, hi) */

/* One violation (32 bytes).  reason 1: the address is in no speculated
 * interval; reason 2: it is inside one but that interval lacks the mode.
 * victim: index of the buffer containing addr, or -1. */
typedef struct {
  uint64_t index, addr;
  uint32_t launch_id;
  uint8_t is_write, reason;
  uint16_t _p;
  int32_t victim;
  uint32_t _q;
} phos_violation;

typedef struct {
  uint64_t bg_pages;     /* pages copied by the background copy                */
  uint64_t cow_pages;    /* pages copied before a launch (copy-on-write)       */
  uint64_t recopy_pages; /* pages recopied after the re-quiesce                */
  uint64_t image_bytes;  /* bytes of the image                                 */
  uint64_t precopy_pages; /* pages copied by pre-copy rounds                   */
  uint64_t staged_pages;  /* copy-on-write pages that went through staging      */
  uint64_t bg_read_pages; /* pool pages its background pass read: bg_pages, or
                             for phos_ckpt_start_pair the pages read once for
                             both images (reported by the copy-on-write one; 0
                             for the recopy one) */
  double bg_ms;           /* GPU time of its background pass, from when it could
                             start to its end (HIP events) */
  uint64_t stage_batches; /* blocking staging: batches the drain moved (one
                             engine copy each); 0 otherwise */
} phos_ckpt_stats;

typedef struct {
  uint64_t bg_pages;     /* pages brought in by the background restore */
  uint64_t demand_pages; /* pages brought in before a launch           */
  uint64_t dma_pages;    /* pages of pageable image pieces (DMA)       */
  uint64_t asked_pages;  /* ... of which launches asked for first        */
  double dma_ms;         /* host time from begin until the DMA finished */
  double dma_first_ms;   /* ... until its first batch of pages was published */
  double dma_first_issue_ms;  /* ... until its first copy was queued        */
  double dma_first_copy_ms;   /* ... until that batch's copies had landed   */
  double bg_ms;          /* GPU time of the background restore (HIP events) */
} phos_rst_stats;

/* ---------------------------------------------------------------- context */

/* Create a context for the pool [pool_base, pool_base + pool_bytes) on HIP
 * device `device`.  pool_base must be page aligned; pool_bytes a multiple of
 * page_bytes; page_bytes a power of two in [4 KiB, 2 MiB].  The caller owns
 * the pool memory.  E_INVAL on bad sizes, E_NOMEM / E_HIP on allocation.
 *
 * Status.  The asynchronous calls raise sticky status words on the device
 * that phos_stream_status reports: a validation with more violations than
 * its cap (PHOS_E_OVERFLOW) and a device-side segment batch with a malformed
 * segment (PHOS_E_INVAL).  An expired device wait (PHOS_E_TIMEOUT) and a
 * misspeculation of an inline validator (PHOS_E_MISSPEC) are reported by the
 * phos_ckpt_end / phos_restore_end of the checkpoint or restore they spoil.
 * Tuning, read from the environment here (defaults in brackets):
 *   PHOS_SPIN_LIMIT      polls before a device wait gives up [1 << 22]
 *   PHOS_BG_GRID         background copy blocks [2 x CUs; at most CUs when
 *                        reading a host image]; PHOS_COW_GRID [4 x CUs];
 *                        PHOS_BG_GRID_HOST when copying into a host image [8]
 *   PHOS_BG_BATCH        pages a background block claims per batch [64];
 *                        PHOS_BG_BATCH_PCIE when the image is in host memory [4]
 *   PHOS_COPY_NT         streaming (non-temporal) device copies [1]
 *   PHOS_COW_DEEP        copy-on-write copies keep 16 loads in flight per
 *                        thread instead of 8 [1]
 *   PHOS_COW_VICTIM_WINDOW  launches whose victim pages one copy-on-write
 *                        call takes [128]; PHOS_COW_VICTIM_FIRST the first
 *                        such call after the tracking window opens [16]
 *   PHOS_VTILE_MAX       largest validation tile, records [16384 / 32768 tracked]
 *   PHOS_VFINISH_MAX_TILES  calls up to this many tiles (at most 4096) order
 *                        their violations in one kernel [4096]
 *   PHOS_RST_PAUSE       restore: polls (about 0.5 us each) the background
 *                        holds back per batch while on-demand copies run [64];
 *                        0 lets them share the link
 *   PHOS_RST_HOLD_MS     restore: that hold applies only this long after the
 *                        background copy starts, 0: always [200]
 *   PHOS_RST_DEEP_DEMAND / PHOS_RST_DEEP_BG  restore from host memory: 16
 *                        loads in flight per thread in on-demand [1] /
 *                        background [0] copies
 *   PHOS_TWIN_BLOCKS_PER_CU  twin kernel blocks per CU [4; 5 with PHOS_V_TRACK]
 *   PHOS_DRAIN_CHUNK_KB  image drain to a host image: chunk size [16384; 0 =
 *                        one copy]; PHOS_DRAIN_WINDOW chunks in flight [2]
 *   PHOS_STAGE_THREADS   blocking CoW staging: host threads moving drained
 *                        pages into the image [4]
 *   PHOS_STAGE_HIGH_PCT  ... the ring's fill (percent) that starts its drain
 *                        during the checkpoint [50]; the rest drains at the end */
phos_status phos_create(int device, uint64_t pool_base, uint64_t pool_bytes, uint32_t page_bytes,
                        phos_ctx **out);
/* Synchronizes the device, frees everything the context owns. */
phos_status phos_destroy(phos_ctx *ctx);

/* Section 4.1: the process's allocation table, as intercepted allocations.
 * bufs: host array of n buffers, ascending base, page aligned, whole pages,
 * non-overlapping, inside the pool (E_INVAL otherwise).  Replaces the table;
 * synchronous; E_STATE while a checkpoint or restore is open. */
phos_status phos_buffers_register(phos_ctx *ctx, const phos_buffer *bufs, uint32_t n);

/* Bytes of the checkpoint image (sum of buffer sizes). */
phos_status phos_image_bytes(phos_ctx *ctx, uint64_t *bytes);

/* ------------------------------------------------------------- speculation */

/* Section 4.1 (argument-based speculation with signature filtering, API
 * specified ranges) and Section 6 (const pointers as the read set): turn one
 * launch's arguments into a sorted interval set and keep it under a handle.
 * A pointer names the buffer b with base_b <= value < base_b + bytes_b, whole;
 * pointers naming no buffer and scalars are dropped; identical intervals are
 * merged by OR-ing modes.  At most 64 intervals (E_INVAL beyond); RANGE with
 * no mode bits or a wrapping range is E_INVAL.  Host-only, synchronous. */
phos_status phos_spec_register(phos_ctx *ctx, uint32_t launch_id, const phos_arg *args,
                               uint32_t nargs, phos_spec *out);
/* Copy a registered interval set to host memory: *n = count, at most cap written. */
phos_status phos_spec_intervals(phos_ctx *ctx, phos_spec spec, phos_interval *out, uint32_t cap,
                                uint32_t *n);
phos_status phos_spec_release(phos_ctx *ctx, phos_spec spec);

/* -------------------------------------------------------------- validation */

/* Section 4.1 runtime validation of one launch's access stream.  Each record
 * whose access [a, a+8) is not inside a speculated interval holding the mode
 * it needs is a violation (reads checked iff PHOS_V_READS, writes iff
 * PHOS_V_WRITES).  Violations are written to `out` (device memory, 16-byte
 * aligned, cap entries; E_INVAL if misaligned) in ascending record index,
 * and the count to *n_violations (device
 * memory, one uint64_t).  With PHOS_V_TRACK the dirty / victim bitmaps are
 * updated.  d_records: device memory, 8-byte aligned (16-byte alignment is
 * faster).  Asynchronous on `stream`; if *n_violations > cap the contents of
 * out are unspecified and the overflow is reported by phos_stream_status,
 * or by this call itself with PHOS_V_SYNC (PHOS_E_OVERFLOW, the true count
 * in *n_violations).  Validation calls on one context are serialized by the
 * library. */
phos_status phos_validate(phos_ctx *ctx, phos_spec spec, const uint64_t *d_records, uint64_t n,
                          uint32_t flags, phos_violation *out, uint64_t cap,
                          uint64_t *n_violations, hipStream_t stream);

/* For callers that cannot allocate device memory: code recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same validation as phos_validate (same arguments, results, asynchrony and
 * flags), but its workspace is a fixed array in device memory, one per GPU,
 * held until the process ends (about 4 MiB), so the call allocates nothing.
 * Limits, checked before any device work (PHOS_E_INVAL): cap <= 131,072
 * violation records, and at most 4,096 validation tiles: 67,108,864 records
 * per call untracked and 134,217,728 with PHOS_V_TRACK at the default
 * largest tiles (16,384 and 32,768 records; PHOS_VTILE_MAX).  Every
 * call on one GPU shares the array and leaves its last contents there;
 * each call clears the counters it needs first.  Calls that overlap on one
 * GPU (different streams of one context not ordered by the library, or
 * different contexts) race on the array and must be ordered by the caller. */
phos_status phos_validate_noalloc(phos_ctx *ctx, phos_spec spec, const uint64_t *d_records,
                                  uint64_t n, uint32_t flags, phos_violation *out, uint64_t cap,
                                  uint64_t *n_violations, hipStream_t stream);

/* Many launches in one pass: launch i uses specs[i], records d_records[i]
 * (n[i] of them); host arrays of nlaunch entries.  Output ordered by
 * (position i in the call, record index). */
phos_status phos_validate_batch(phos_ctx *ctx, const phos_spec *specs,
                                const uint64_t *const *d_records, const uint64_t *n,
                                uint32_t nlaunch, uint32_t flags, phos_violation *out,
                                uint64_t cap, uint64_t *n_violations, hipStream_t stream);

/* Section 4.1 twin kernel: an application kernel with the validator fused
 * into it.  The kernel computes y[j] = 3 * y[j] + x[i] (uint64, wrapping) for
 * i < n, with j = idx[i] (an element offset from y, may be negative) or j = i
 * when idx is NULL.  flags = 0 runs it uninstrumented (spec, out, cap and
 * n_violations unused).  Otherwise it is the instrumented twin: every global
 * access it makes is checked against `spec` as phos_validate checks a
 * record -- per element i the reads of x[i], idx[i] and y[j] (PHOS_V_READS)
 * and the write of y[j] (PHOS_V_WRITES) -- and PHOS_V_TRACK updates the
 * dirty / victim bitmaps as phos_validate does.  Every access is made either
 * way, as in the paper; acting on a reported failure is the caller's
 * protocol.  Violations (index = i) go to `out` in no particular order, the
 * count to *n_violations (device memory, zeroed by the call; E_INVAL if
 * flags != 0 and it is NULL).  x, y, idx: device memory, 8-byte aligned; the
 * caller guarantees every y + j lies in memory it may write.  Asynchronous
 * on `stream` (PHOS_V_SYNC as for phos_validate).  Section 4.2 with an
 * inline validator: the write is made before its check fails, so with a
 * copy-on-write checkpoint open (and PHOS_V_WRITES or PHOS_V_TRACK) a
 * failing write inside a buffer, on a page that checkpoint has not copied
 * yet, is a misspeculation: that checkpoint's phos_ckpt_end returns
 * PHOS_E_MISSPEC, and the caller takes a stop-the-world checkpoint instead. */
phos_status phos_twin_scale_add(phos_ctx *ctx, phos_spec spec, const uint64_t *x, uint64_t *y,
                                const int64_t *idx, uint64_t n, uint32_t flags,
                                phos_violation *out, uint64_t cap, uint64_t *n_violations,
                                hipStream_t stream);

/* Synchronous: wait for the work enqueued on `stream`, then report and clear
 * the sticky status the context's asynchronous calls raised so far:
 * PHOS_E_INVAL if a phos_copy_batch* call met a malformed segment (that call
 * copied nothing), else PHOS_E_OVERFLOW if a validation or twin call found
 * more violations than its cap, else PHOS_OK. */
phos_status phos_stream_status(phos_ctx *ctx, hipStream_t stream);

/* Clear the dirty and victim bitmaps, the victim list and the launch
 * numbering of validation (the next validated launch is number 1 again;
 * asynchronous on stream).  E_STATE while a recopy checkpoint is open: its
 * recopy list is read from these maps. */
phos_status phos_track_reset(phos_ctx *ctx, hipStream_t stream);
/* Synchronous copy of a bitmap to host: which 0 = dirty, 1 = victim.  Bit p%32
 * of word p/32 is pool page p; nwords >= ceil(pool pages / 32). */
phos_status phos_track_read(phos_ctx *ctx, uint32_t which, uint32_t *host_words, uint64_t nwords);

/* ------------------------------------------------------------- checkpoint */

/* Section 4.2 / 4.3: open a concurrent checkpoint.  The caller has quiesced
 * the application (its streams are idle).  image: device memory of
 * phos_image_bytes() bytes that receives the image (pinned host memory means
 * copying straight to the host; E_INVAL for pageable memory).  host_image: optional pinned host memory
 * filled from image by phos_ckpt_end (NULL: none).  The background copy of
 * every page starts on copy_stream unless PHOS_CKPT_DEFER_BACKGROUND.
 * Opening resets the dirty / victim bitmaps (and the launch numbering of
 * validation) when no other checkpoint is open.  At most one checkpoint per
 * protocol may be open (E_STATE). */
phos_status phos_ckpt_begin(phos_ctx *ctx, uint32_t protocol, uint32_t flags, void *image,
                            void *host_image, hipStream_t copy_stream, phos_ckpt **out);

/* Section 4.2, CoW staging for a checkpoint into a host image (pinned): the
 * copy-on-write copies, which a launch waits for, go first into `staging`
 * (device memory, the caller's, `bytes` rounded down to whole pages) at HBM
 * speed instead of over PCIe; once it is full they go straight to the host
 * image.  phos_ckpt_end moves the staged pages into the image.  Call after
 * phos_ckpt_begin and before the first phos_ckpt_cow (E_STATE otherwise, or
 * for a recopy checkpoint); bytes below one page: no staging.  E_INVAL for
 * a device image or staging that is not 16-byte aligned device memory.
 * The staging memory must stay allocated until phos_ckpt_end returns. */
phos_status phos_ckpt_staging(phos_ckpt *ck, void *staging, uint64_t bytes);

/* Policies of phos_ckpt_staging_policy. */
enum {
  PHOS_STAGE_HOST_DIRECT = 0, /* a full area: copies go straight to the host image */
  PHOS_STAGE_BLOCK = 1        /* a full area: copies wait for a slot the drain frees */
};

/* Section 4.2, CoW staging with a policy for a full area.
 * PHOS_STAGE_HOST_DIRECT is phos_ckpt_staging.  PHOS_STAGE_BLOCK makes the
 * area a ring of bytes / page_bytes slots that the host drains into the host
 * image while the checkpoint runs: a host thread the call starts moves
 * batches of consecutive slots (up to 16 MiB) with the copy engines into
 * pinned bounce buffers, no compute queue taking part, and PHOS_STAGE_THREADS
 * (default 4) more host threads move the pages to their places in the
 * image.  Every copy-on-write page takes the next slot; when the ring is full
 * the copy waits until the drain has freed the slot it needs (a bounded
 * wait: if it gives up the page goes straight to the image and phos_ckpt_end
 * reports PHOS_E_TIMEOUT).  phos_ckpt_end waits for the drain of the last
 * slot; stats.staged_pages counts the pages that went through the ring.
 * Pinned host memory: 12 bytes per slot of control words and 8 bounce
 * buffers of min(slots, 16 MiB / page_bytes) pages.  Same preconditions and
 * errors as phos_ckpt_staging, plus E_INVAL for an unknown policy and
 * E_HIP when the copy engines cannot be reached.  The staging memory must
 * stay allocated until phos_ckpt_end returns. */
phos_status phos_ckpt_staging_policy(phos_ckpt *ck, void *staging, uint64_t bytes,
                                     uint32_t policy);

/* Start the background copy of a checkpoint opened with
 * PHOS_CKPT_DEFER_BACKGROUND now, on its copy_stream, after the work already
 * enqueued on `after` (NULL: no wait).  Lets a caller keep the bandwidth-bound
 * copy away from bandwidth-bound work it must finish first (e.g. the
 * validation of the launches) and beside latency-bound launches instead.
 * E_STATE if the background copy has started or the recopy is done. */
phos_status phos_ckpt_start(phos_ckpt *ck, hipStream_t after);

/* Sections 4.2 and 4.3 with both checkpoints open in one window: a
 * copy-on-write checkpoint `cow` (its image frozen at its begin) and a recopy
 * checkpoint `recopy` (its image taken at its recopy), both begun with
 * PHOS_CKPT_DEFER_BACKGROUND on one context, into device images.  Starts
 * their background copies as one pass on cow's copy stream (after the work
 * already on `after`, if not NULL): until a page is written the two images
 * hold the same bytes, so the pass reads each pool page once and stores it
 * to each image that still needs it (a page is claimed in each image on its
 * own, as by phos_ckpt_start; pages already traced as written are left to
 * the recopy).  Copy-on-write, pre-copy rounds, the recopy and the ends work
 * as with separate passes; recopy's copy stream waits for this pass.
 * E_INVAL: not a copy-on-write and a recopy checkpoint of one context, or a
 * host image or staging area; E_STATE: a background copy already started. */
phos_status phos_ckpt_start_pair(phos_ckpt *cow, phos_ckpt *recopy, hipStream_t after);

/* Section 4.2: before the launch described by `spec` runs on app_stream,
 * copy every page it may write that the checkpoint has not copied yet: the
 * pages of its write intervals and the victim pages marked by validation.
 * A page already being copied is waited for.  Asynchronous on app_stream;
 * the launch must be enqueued after this call.  PROTOCOL COW only.
 * The validation that marks a launch's victim pages must be complete in
 * app_stream order before this call (enqueued on app_stream, or waited for
 * with an event).  While every call comes from one stream and every tracking
 * validation went to that same stream, the host skips a call whose write
 * pages earlier calls already asked for when no validation has run since
 * (those pages are done before the launch, in stream order); with tracking
 * validations on other streams each call scans the whole victim map.
 * Victim pages by launch: in that one-stream case, for a spec validated once
 * (with tracking) since the checkpoint opened, the victim pages are sorted by
 * the launch that writes them first, and a call copies those of a window of
 * launches (from the first not yet taken through at least this one,
 * PHOS_COW_VICTIM_WINDOW of them, PHOS_COW_VICTIM_FIRST for the first call,
 * never past the end of the validation call that numbered them) instead of
 * every victim page marked so far.  A checkpoint into a host image with a
 * staging area (host-direct, or a blocking ring of at least half the pool's
 * pages) takes them all in the first call. */
phos_status phos_ckpt_cow(phos_ckpt *ck, phos_spec spec, hipStream_t app_stream);

/* Section 4.3: re-quiesce (copy_stream waits for app_stream) and recopy every
 * dirty or victim page into the image after the background copy; app_stream
 * then waits for the recopy.  PROTOCOL RECOPY only.  The background copy of
 * a recopy checkpoint skips pages already marked dirty or victim when it
 * reaches them: the recopy copies those pages anyway, so the image is the
 * same and the concurrent copy moves fewer bytes. */
phos_status phos_ckpt_recopy(phos_ckpt *ck, hipStream_t app_stream);

/* Sections 4.3 and 7, iterative recopy: a pre-copy round.  In app_stream
 * order, every page marked dirty so far is unmarked and copied into the
 * image now, while the application keeps running; a page written again
 * later is marked again by validation and copied at the re-quiesce, which
 * then moves fewer pages.  Victim marks are kept for the re-quiesce.  Call
 * between launches: every launch validated so far must be enqueued on
 * app_stream before this call, and later validations issued after it in
 * app_stream order (a mark made concurrently could be lost).  Asynchronous
 * on app_stream.  E_STATE unless an open recopy checkpoint not yet
 * recopied. */
phos_status phos_ckpt_precopy(phos_ckpt *ck, hipStream_t app_stream);

/* Sections 4.3 and 7, iterative recopy with the window's remaining launches
 * known (their access streams validated ahead, as the speculation allows):
 * a pre-copy round that copies only pages whose last write in the window has
 * been issued on app_stream already, and unmarks them.
 *  - Dirty pages outside every write interval of the `upcoming` specs: no
 *    remaining launch may write them validly.
 *  - Victim pages outside those intervals whose latest failing write
 *    (validation numbers launches in validation order) came from a launch
 *    issued already: the n_validated_ahead most recently validated launches
 *    are the ones still to come.
 * A later write to such a page can only be a violation found by a later
 * validation, which marks it again, and the recopy at the re-quiesce copies
 * every marked page.  Unlike phos_ckpt_precopy, launches validated ahead of
 * their turn do no harm.  upcoming: the specs of every launch of the window
 * still to be issued on app_stream (any order; n_upcoming 0: none), of which
 * the first n_validated_ahead have been validated (validations follow the
 * launch order).  Every tracking validation so far must be complete in
 * app_stream order (on app_stream or waited for); with tracking validations
 * on other streams victim pages are left to the recopy.  E_INVAL for an
 * unknown spec or n_validated_ahead above n_upcoming or above the launches
 * validated since the maps were cleared; E_STATE for a copy-on-write
 * checkpoint, after the recopy, or under stream capture (the mask is built
 * on the host at the call).  Asynchronous on app_stream. */
phos_status phos_ckpt_precopy_final(phos_ckpt *ck, const phos_spec *upcoming, uint32_t n_upcoming,
                                    uint32_t n_validated_ahead, hipStream_t app_stream);

/* Finish: wait for every copy (and app_stream), drain image to host_image if
 * given, free the handle.  A recopy checkpoint not yet recopied is recopied
 * first (ending is a quiesce point).  The drain (Section 5) is issued in
 * chunks from the calling thread with a few in flight, so device-to-host
 * copies the application issues meanwhile wait for a few chunks, not for
 * the whole image.  E_TIMEOUT if a device wait expired.  E_MISSPEC for a
 * copy-on-write checkpoint if an instrumented launch (phos_twin_scale_add)
 * wrote outside its speculation into a page the checkpoint had not copied
 * (Section 4.2: the image is then not the state at t1; take a stop-the-world
 * checkpoint).  The handle is freed in every case. */
phos_status phos_ckpt_end(phos_ckpt *ck, hipStream_t app_stream, phos_ckpt_stats *stats);

/* Synchronous: copied-page bitmap of an open checkpoint (bit p = pool page p);
 * for a recopy checkpoint, the pages its background copy has copied. */
phos_status phos_ckpt_copied(phos_ckpt *ck, uint32_t *host_words, uint64_t nwords);

/* ----------------------------------------------------------------- restore */

/* Section 6: open a concurrent restore from `image` (phos_image_bytes()
 * bytes, layout as written by a checkpoint).  The background copy of every
 * page into the pool starts on copy_stream unless PHOS_RST_DEFER_BACKGROUND.
 * Device or pinned host memory is read by the kernels directly; a pageable
 * host image cannot be, so its pages are held at begin and moved by the copy
 * engines (HSA runtime copies, no HIP stream or kernel) from a library
 * thread, the pages a launch asks for first (the launch waits until they
 * land).  E_HIP if that DMA failed (or no HSA agent matches the device);
 * E_TIMEOUT if a device wait expired.  One restore per context at a time. */
phos_status phos_restore_begin(phos_ctx *ctx, uint32_t flags, const void *image,
                               hipStream_t copy_stream, phos_rst **out);

/* Section 2.2: an image holds the buffers' bytes only, so a restore must go
 * into the same buffers.  A manifest records them: magic "PHOSIMG1",
 * version 1, the protocol (PHOS_COW / PHOS_RECOPY, 0: none), the page size,
 * the buffer count and the image bytes (a 32-byte header), then per buffer
 * its pool-relative offset and size (2 x uint64), then an FNV-1a 64 checksum
 * of everything before it.  Host only, synchronous.  phos_manifest_write
 * writes the context's manifest (out NULL: only *bytes, the size;
 * E_OVERFLOW if cap is smaller).  phos_manifest_check returns E_INVAL unless
 * the manifest is intact and its page size, buffer count, image bytes and
 * buffer sizes (in order) equal the context's registered buffers (their
 * places in the pool may differ).  phos_restore_begin_manifest checks, then
 * opens the restore as phos_restore_begin. */
phos_status phos_manifest_write(phos_ctx *ctx, uint32_t protocol, void *out, uint64_t cap,
                                uint64_t *bytes);
phos_status phos_manifest_check(phos_ctx *ctx, const void *manifest, uint64_t bytes);
phos_status phos_restore_begin_manifest(phos_ctx *ctx, uint32_t flags, const void *image,
                                        const void *manifest, uint64_t manifest_bytes,
                                        hipStream_t copy_stream, phos_rst **out);

/* As phos_restore_begin, with the image split into nchunks pieces of
 * chunk_bytes each (a multiple of the page size; the last may be partly
 * used): image byte i lives at chunks[i / chunk_bytes] + i % chunk_bytes.
 * For host images too large for one pinned allocation, or larger than the
 * host lets a process pin: each piece may be device, pinned or pageable
 * memory, pageable pieces going the DMA way described above. */
phos_status phos_restore_begin_chunked(phos_ctx *ctx, uint32_t flags, const void *const *chunks,
                                       uint32_t nchunks, uint64_t chunk_bytes,
                                       hipStream_t copy_stream, phos_rst **out);

/* Section 6: before a launch runs on app_stream, bring in every page inside a
 * buffer that its records touch (and, with PHOS_RST_PREFETCH_SPEC, every page
 * of its speculated intervals) that is not present yet.  d_faulted: optional
 * device uint64_t, incremented by the number of pages this call copied. */
phos_status phos_restore_on_demand(phos_rst *rs, phos_spec spec, const uint64_t *d_records,
                                   uint64_t n, hipStream_t app_stream, uint64_t *d_faulted);

/* Synchronous: present-page bitmap (bit p = pool page p). */
phos_status phos_restore_present(phos_rst *rs, uint32_t *host_words, uint64_t nwords);

/* Wait for the background restore and app_stream; free the handle. */
phos_status phos_restore_end(phos_rst *rs, hipStream_t app_stream, phos_rst_stats *stats);

/* ----------------------------------------------------- batched copy / serving */

/* One copy segment of a request: bytes from src to dst (device memory;
 * addresses and size multiples of 16), belonging to request req. */
typedef struct { uint64_t src, dst, bytes; uint32_t req, _p; } phos_copy_seg;

typedef struct {
  uint64_t chunk_bytes; /* work unit claimed by one workgroup (64 KiB .. 4 MiB) */
  uint32_t wg_per_cu;   /* resident workgroups per compute unit (1 .. 16)       */
  uint32_t threads;     /* threads per workgroup: 256, 512 or 1024             */
} phos_batch_cfg;

typedef struct phos_seglist phos_seglist;

/* A batched copier (no paper analog; the paper copies buffer by buffer in
 * 4 MB chunks, Section 5): a device-resident work queue of up to max_segs
 * segments of up to max_reqs requests, and one HIP graph holding a reset
 * kernel and a persistent copy kernel whose workgroups claim chunk_bytes
 * pieces of the concatenated segment stream until it is drained.  The graph
 * is captured once and replayed for every batch.  cfg NULL: defaults. */
phos_status phos_batch_create(int device, uint64_t max_segs, uint32_t max_reqs,
                              const phos_batch_cfg *cfg, phos_batch **out);
phos_status phos_batch_destroy(phos_batch *b);
/* Load segments (host array, nseg <= max_segs, req < max_reqs) into the
 * device queue, asynchronously on stream through pinned staging.  E_INVAL
 * on misaligned segments. */
phos_status phos_batch_load(phos_batch *b, const phos_copy_seg *segs, uint64_t nseg,
                            hipStream_t stream);
/* Replay the graph on stream: one persistent launch copies every loaded
 * segment; per-request copied bytes are reset, then accumulate in the device
 * array of phos_batch_done_bytes (max_reqs entries). */
phos_status phos_batch_run(phos_batch *b, hipStream_t stream);
/* phos_batch_load followed by phos_batch_run. */
phos_status phos_batch_copy(phos_batch *b, const phos_copy_seg *segs, uint64_t nseg,
                            hipStream_t stream);
phos_status phos_batch_done_bytes(phos_batch *b, uint64_t **d_done);
/* Synchronous: completion time of requests 0..n-1 of the last run, in ms
 * after the run started, from the GPU wall clock (-1: not completed). */
phos_status phos_batch_times(phos_batch *b, double *ms, uint32_t n);
phos_status phos_batch_get_cfg(phos_batch *b, phos_batch_cfg *cfg);
/* Change the configuration (synchronizes the device and re-captures). */
phos_status phos_batch_set_cfg(phos_batch *b, const phos_batch_cfg *cfg);

/* Plain path: a device-resident segment list (synchronous upload) and one
 * ordinary launch per call, one workgroup per chunk, no graph. */
phos_status phos_seglist_create(int device, const phos_copy_seg *segs, uint64_t nseg,
                                phos_seglist **out);
phos_status phos_seglist_destroy(phos_seglist *l);
phos_status phos_copy_plain(const phos_seglist *l, uint64_t chunk_bytes, uint32_t threads,
                            hipStream_t stream);

/* Autotuner: time every candidate of chunk {64 KiB .. 4 MiB} x wg_per_cu
 * {1, 2, 4, 8} x threads {256, 512, 1024} on the given segments (host
 * array; their addresses must be valid device memory; the copies are really
 * performed) and return the fastest.  Results are cached in memory and in
 * the text file cache_path (may be NULL) under a key of the segment-size
 * distribution (log2 of total bytes, segment count and mean size). */
phos_status phos_batch_tune(int device, const phos_copy_seg *segs, uint64_t nseg,
                            const char *cache_path, phos_batch_cfg *best, double *best_ms);

/* Segments already in device memory (or pinned host memory), copied by the
 * context (no paper analog; the paper copies buffer by buffer in 4 MB
 * chunks, Section 5).  d_segs: nseg phos_copy_seg entries, 8-byte aligned;
 * each segment's src, dst and bytes must be non-NULL 16-byte multiples, or
 * the whole call copies nothing and phos_stream_status reports E_INVAL; req
 * is ignored.  Segments must not overlap one another's destinations or
 * sources.  Asynchronous on `stream`; calls of one context must not overlap
 * (they share its segment header).  phos_copy_batch: one workgroup writes
 * the byte prefix of the segment stream, then one persistent launch copies
 * it in chunks with the default configuration (1 MiB chunks, 2 workgroups of
 * 512 threads per CU; PHOS_BATCH_CHUNK / _WG_PER_CU / _THREADS override).
 * phos_copy_batch_tuned: the same pair of kernels captured in a HIP graph
 * and replayed; the first call for a (d_segs, nseg) pair reads the segments
 * back (synchronously), runs phos_batch_tune on them (which performs the
 * copies; cache file: $PHOS_TUNE_CACHE) and captures the graph with the
 * configuration it picks; later calls with the same pair replay it (the
 * segments' contents may change between calls; the choice is kept). */
phos_status phos_copy_batch(phos_ctx *ctx, const phos_copy_seg *d_segs, uint64_t nseg,
                            hipStream_t stream);
phos_status phos_copy_batch_tuned(phos_ctx *ctx, const phos_copy_seg *d_segs, uint64_t nseg,
                                  hipStream_t stream);

/* Run the loaded queue with the plain kernel (one workgroup per chunk, no
 * graph, no persistence) — the per-request path the batch is compared with. */
phos_status phos_batch_run_plain(phos_batch *b, hipStream_t stream);

/* ------------------------------------------------------------- serving loop */
/* No paper analog.  Requests arrive at host-clock times, are admitted in
 * arrival order when their destination fits in an HBM budget, and complete
 * when their copies are done.  PHOS_SERVE_PLAIN serves one request at a time
 * (FIFO, one launch each).  PHOS_SERVE_BATCHED is continuous batching:
 * admitted bulk requests share each iteration (up to quantum_bytes each,
 * iter_bytes in total, shortest remaining work first) of the persistent
 * graph-captured copy, two iterations in flight; requests arriving meanwhile
 * join the next iteration; bursts run at once on their own stream. */
enum { PHOS_SERVE_PLAIN = 0, PHOS_SERVE_BATCHED = 1 };
enum { PHOS_REQ_CKPT = 0, PHOS_REQ_RESTORE = 1, PHOS_REQ_BURST = 2 };

typedef struct {
  double arrival_s;          /* arrival, seconds after the run starts                    */
  uint32_t type;             /* PHOS_REQ_*                                                */
  uint32_t nseg;             /* CKPT / RESTORE: copy segments                             */
  uint64_t bytes;            /* destination bytes to admit (page multiple)                */
  const phos_copy_seg *segs; /* host array: src = device address, dst = byte offset into
                                the request's destination allocation                    */
  const uint64_t *d_records; /* BURST: device access records, addresses are offsets into
                                the destination (offset | is_write)                      */
  uint64_t nrec;
  uint32_t *d_state;         /* BURST: per-page claim words (2 = already present)         */
  uint64_t image;            /* BURST: device address of the source image of the pages    */
} phos_serve_req;

typedef struct {
  uint32_t mode;           /* PHOS_SERVE_*                                      */
  uint32_t page_bytes;     /* allocation and burst page size                    */
  uint64_t budget_bytes;   /* destination budget (bytes of d_arena)             */
  void *d_arena;           /* device memory receiving every destination         */
  uint64_t quantum_bytes;  /* BATCHED: per request per iteration                */
  uint64_t iter_bytes;     /* BATCHED: per iteration                            */
  phos_batch_cfg cfg;      /* copy kernel configuration                         */
  uint32_t keep;           /* nonzero: never reuse a destination (for checking)  */
  uint32_t _pad;
  uint64_t small_bytes;    /* BATCHED order inside an iteration: requests with at
                              most this many bytes left go first, shortest first;
                              the rest follow in arrival order (UINT64_MAX:
                              shortest remaining first for every request)       */
} phos_serve_cfg;

typedef struct {
  double admit_ms;   /* host clock, ms after the run start                        */
  double done_ms;    /* completion: the copy kernel's GPU wall-clock stamp mapped
                        to the host clock (bursts: when the host saw it finish)   */
  double latency_ms; /* done_ms - arrival                                        */
  uint64_t dst_off;  /* destination offset in d_arena                             */
} phos_serve_out;

typedef struct {
  double wall_ms;        /* first arrival to last completion            */
  uint64_t bytes;        /* bytes copied (bulk segments + faulted pages) */
  uint64_t iterations;   /* BATCHED: copy iterations launched           */
  uint32_t max_active;   /* most requests admitted at once              */
} phos_serve_stats;

/* Serve n requests (sorted by arrival) on device; out[i] per request.
 * Destinations are freed at completion (their bytes stay in d_arena until
 * reused).  E_INVAL if a request cannot ever fit the budget. */
phos_status phos_serve_run(int device, const phos_serve_cfg *cfg, const phos_serve_req *reqs,
                           uint32_t n, phos_serve_out *out, phos_serve_stats *stats);

const char *phos_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PHOS_H */
