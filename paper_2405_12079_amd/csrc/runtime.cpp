// runtime.cpp — host side of libphos: context, speculation (interval sets),
// validation orchestration, and the soft copy-on-write, soft recopy and
// concurrent-restore protocols (PhoenixOS, arXiv 2405.12079, Sections 4-6),
// driving the gfx950 kernels in kernels.hip.
#include <hip/hip_runtime.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "phos.h"
#include "util.h"

using namespace phos;

// ------------------------------------------------------------------ errors
namespace phos {
static thread_local std::string g_err;

phos_status fail(phos_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

uint32_t env_u32(const char *name, uint32_t dflt) {
  const char *v = getenv(name);
  if (!v || !*v) return dflt;
  return (uint32_t)strtoul(v, nullptr, 0);
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
  if (prev_ != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
  if (prev_ >= 0) (void)hipSetDevice(prev_);
}
}  // namespace phos

extern "C" const char *phos_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------------- structures
struct HostSpec {
  bool used = false;
  uint32_t launch_id = 0;
  uint64_t gen = 0;               // registration number: a reused handle is a new spec
  std::vector<phos_interval> iv;  // sorted by (lo, hi)
  // victim buckets: validated vb_n times (with tracking) since the buckets'
  // generation vb_gen started, the last time as launch number vb_seq
  uint64_t vb_gen = 0;
  uint32_t vb_n = 0, vb_seq = 0;
};

constexpr uint32_t kVBuckets = 1u << 16;  // launches numbered per tracking window with buckets

// Events around a background copy on the context's background stream: its
// start (after the work it follows) and its end; timed, for the stats.
struct BgEvents {
  hipEvent_t start = nullptr, done = nullptr;
  void destroy() {
    if (start) (void)hipEventDestroy(start);
    if (done) (void)hipEventDestroy(done);
    start = done = nullptr;
  }
  double ms() const {
    float m = 0;
    if (!start || !done || hipEventElapsedTime(&m, start, done) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    return m;
  }
};

constexpr uint32_t kSlotCounters = 8;
struct Slot {  // per-protocol reusable device state of a checkpoint / restore
  uint32_t *state = nullptr;               // per pool page
  unsigned long long *counters = nullptr;  // [0] chunk cursor, [1..5] stats, [6..7] background
                                           // completion (a restore: [4] on-demand copies)
  uint32_t *list = nullptr;                // recopy page list
  unsigned int *list_count = nullptr;
};

struct phos_ctx {
  int device = 0;
  uint64_t pool_base = 0, pool_bytes = 0;
  uint32_t page_bytes = 0, page_shift = 0, n_pages = 0, nwords = 0;
  std::vector<phos_buffer> bufs;
  std::vector<uint32_t> h_img_page, h_img_pool;  // pool page -> image page, and back
  uint64_t image_bytes = 0;
  uint32_t n_cu = 256;

  uint32_t *d_page_buf = nullptr, *d_img_page = nullptr;
  uint8_t *d_dirty = nullptr, *d_victim = nullptr;  // page maps, n_pages padded to 32
  uint32_t *d_vlist = nullptr, *d_vmeta = nullptr;  // victim pages appended by validation
  // per pool page (padded to 32): the largest sequence number of a launch
  // with a failing write there; validated launches are numbered from 1 in
  // validation order since the maps were last cleared
  uint32_t *d_victim_seq = nullptr;
  uint32_t vseq = 0;
  // Section 4.2, victim pages by launch: the earliest failing launch of each
  // page, and per launch number a bucket of the victim pages it writes first
  // (vbucket[vbse[2 (s - 1)] .. vbse[2 (s - 1) + 1]), start and end
  // interleaved), built after each tracking validation on the device, with
  // the bounds read back to h_vbse (pinned, same layout) behind vb_evt.  vb_broken: some victim marks since the
  // window opened have no buckets (copy-on-write takes the appended list).
  uint32_t *d_vfirst = nullptr, *d_vbse = nullptr, *d_vbucket = nullptr;
  uint32_t *d_vbseg0 = nullptr, *d_vbcursor = nullptr;
  uint32_t *h_vbse = nullptr;
  hipEvent_t vb_evt = nullptr;
  bool vb_evt_used = false, vb_broken = false;
  uint64_t vb_gen = 1;
  uint32_t vb_hi = 0;  // the highest launch number whose bounds have been read back
  // per launch number: the last launch number of the validation call that
  // built its bucket (0: no bucket)
  std::vector<uint32_t> vb_last = std::vector<uint32_t>(kVBuckets + 1, 0);
  uint32_t cow_victim_window = 128;  // buckets a copy-on-write call takes at once
  uint32_t cow_victim_first = 16;    // ... the first call of a tracking window (its stall)
  uint32_t vlist_cap = 0;
  // status words the kernels raise (device memory, kErr* entries): a bounded
  // wait expired; a validation found more violations than its cap; a
  // device-side batch met a malformed segment; a write out of speculation
  // landed on a page an open copy-on-write checkpoint had not copied
  uint32_t *d_err = nullptr;
  // this GPU's fixed validation workspace (phos_validate_noalloc; kNaBytes,
  // not owned: it lives until the process ends)
  uint8_t *na_ws = nullptr;

  // device-resident segment batches (phos_copy_batch*): [hdr 4][prefix cap+1]
  // and a chunk cursor; tuned calls replay a captured graph per (segments,
  // count) with the autotuner's configuration
  unsigned long long *d_bq = nullptr, *d_bcursor = nullptr;
  uint64_t bq_cap = 0;
  struct SegGraph {
    const phos_copy_seg *segs;
    uint64_t nseg;
    phos_batch_cfg cfg;
    hipGraphExec_t exec;
    hipGraph_t graph;
    uint64_t last_use;
  };
  std::vector<SegGraph> seg_graphs;
  uint64_t seg_clock = 0;
  hipStream_t cap_stream = nullptr;  // capture stream of those graphs

  // validation workspace
  phos_violation *d_scratch = nullptr;
  uint64_t scratch_cap = 0;
  unsigned long long *d_cursor = nullptr;
  uint32_t *d_tile_count = nullptr;
  unsigned long long *d_tile_off = nullptr;
  uint64_t tile_cap = 0;
  unsigned long long *d_seg_sum = nullptr, *d_seg_prefix = nullptr;
  uint64_t seg_cap = 0;
  hipEvent_t v_evt = nullptr;
  bool v_evt_used = false;
  hipStream_t v_stream = nullptr;  // stream of the last validation

  // batch descriptors ([VLaunch x n][DevIv x m]) cached on the device by
  // content, uploaded once through pinned staging
  // Uploaded batch descriptors, keyed by what determines them: the tile
  // size and, per launch, the spec (handle and registration number), the
  // record pointer and count.  A repeated call finds its descriptors without
  // building them again.
  struct VBatch {
    uint64_t hash;
    std::vector<uint64_t> key;
    uint8_t *dev;
    uint64_t last_use;
  };
  uint64_t spec_gen = 0;
  std::vector<VBatch> vcache;
  uint64_t vclock = 0;
  void *h_vstage = nullptr;
  size_t vstage_cap = 0;
  hipEvent_t vstage_evt = nullptr;
  bool vstage_used = false;

  std::vector<HostSpec> specs;
  std::vector<uint32_t> free_specs;
  // workspace outgrown by a larger call: kept until destroy, because a
  // captured graph may still hold its address
  std::vector<void *> retired;

  Slot slots[3];  // [1] CoW, [2] recopy, [0] restore
  phos_ckpt *open_ckpt[3] = {nullptr, nullptr, nullptr};
  phos_rst *open_rst = nullptr;

  hipStream_t aux = nullptr;     // private stream for synchronous reads
  // Stream of the persistent background copies (created on first use), with
  // a hardware queue of its own: streams created the ordinary way share a
  // few hardware queues round robin, and an application kernel queued behind
  // a background copy in a shared queue would wait for the whole copy (a
  // copy-on-write, pre-copy or on-demand kernel waiting for one of its pages
  // could then not even start).  A stream with a compute-unit mask never
  // shares its queue; the mask here enables every unit.
  hipStream_t bgq = nullptr;
  hipEvent_t bgq_in = nullptr;   // work before a background copy, for bgq to wait on
  unsigned long long *h_pinned = nullptr;  // small pinned readback area
  uint32_t *h_want = nullptr;  // pageable restore: pages asked for by waiting launches (pinned)
  // pageable restore: the two pinned bounce slots the DMA thread stages
  // runs through, a pinned run of kDone words (the states it publishes), and
  // the HSA agents its copy-engine copies name (found at the first such restore)
  uint8_t *h_bounce = nullptr;
  uint32_t *h_done = nullptr;
  bool hsa_inited = false, hsa_ready = false;
  hsa_agent_t gpu_agent{0}, cpu_agent{0};

  uint32_t bg_grid = 1024, cow_grid = 1024, spin_limit = 1u << 22, copy_nt = 0;
  uint32_t bg_grid_host = 8;  // background blocks copying into a host image
  // restore: how long (polls of ~0.5 us) the background holds back per batch
  // while on-demand copies run (0: never), and 16 loads in flight per thread
  // for the on-demand / background copies of an image in host memory
  uint32_t rst_pause = 64, rst_deep_demand = 1, rst_deep_bg = 0;
  uint32_t rst_hold_ms = 200;  // restore: hold only this long after the background starts (0: always)
  uint32_t stage_threads = 4;  // blocking staging: host threads moving drained pages into the image
  uint32_t stage_high_pct = 50;  // ... and the ring's fill (percent) that starts its drain
  uint32_t cow_deep = 1;  // copy-on-write copies keep 16 loads in flight per thread
  uint64_t drain_chunk = 16u << 20;  // image drain to host: chunk bytes (0: one copy)
  uint32_t drain_window = 2;        // ... and chunks in flight
  uint32_t finish_tiles = kFuseTiles;  // calls up to this many tiles order in one workgroup
  // Victim pages: a tracking validation (or twin) may have appended to the
  // list since the last copy-on-write call, which then strides over it with
  // its whole grid.  The host knows this in device order only while every
  // such call went to one stream (victim_stream).
  bool victims_pending = false;
  bool victim_stream_set = false, victim_streams_many = false;
  hipStream_t victim_stream = nullptr;
  uint32_t tile_max = 8 * kVQuantum;    // largest validation tile (records)
  uint32_t tile_max_track = 16 * kVQuantum;  // ... with dirty tracking (fewer map flushes)
  uint32_t bg_batch = 64;               // background groups claimed at once per block
  uint32_t bg_batch_pcie = 4;           // ... when the copy reads host memory
};

struct phos_ckpt {
  phos_ctx *ctx;
  uint32_t protocol, flags;
  uint8_t *image;
  void *host_image;
  hipStream_t copy;
  Slot *slot;
  bool recopied = false;
  bool bg_started = false;
  uint32_t pair = 0;  // shared background pass: 1 copy-on-write side, 2 recopy side
  BgEvents bg;  // around the background copy (on the context's bgq)
  bool bg_known_done = false;
  hipStream_t cow_stream = nullptr;  // the one stream CoW calls came from
  bool cow_streams_many = false;
  // pages of the write intervals earlier CoW calls on cow_stream asked for
  // (one bit per pool page; empty until the first call)
  std::vector<uint64_t> requested;
  bool host = false;  // the image is in host memory (copies cross PCIe)
  // victim buckets of launch numbers 1 .. vb_covered (of bucket generation
  // vb_cov_gen) have been handed to copy-on-write calls
  uint64_t vb_cov_gen = 0;
  uint32_t vb_covered = 0;
  // copy-on-write staging area (device memory, the caller's) for a host image
  uint8_t *stage = nullptr;
  uint32_t *d_stage_page = nullptr;
  unsigned long long *d_stage_head = nullptr;
  uint32_t stage_cap = 0;
  // blocking policy: the area is a ring the host drains during the checkpoint
  bool stage_block = false;
  uint64_t *h_fill = nullptr;      // pinned: per slot (sequence number + 1) << 32 | pool page
  uint32_t *h_free_src = nullptr;  // pinned: the sequence numbers the drain publishes
  uint32_t *d_free_seq = nullptr;  // device: per slot, sequence number + 1 of its last drained occupant
  std::thread drainer;
  std::atomic<bool> drain_stop{false}, drain_abort{false};
  std::atomic<uint64_t> drain_final{0};  // slots taken in all (set with drain_stop)
  phos_status drain_status = PHOS_OK;
  std::string drain_error;
  uint64_t drained_pages = 0, drain_copies = 0;
  uint8_t *h_bounce = nullptr;     // pinned: the drain's bounce buffers
  uint32_t drain_batch_slots = 0, drain_threads = 0, drain_high_pct = 50;
  // final-page pre-copy rounds: the pages the remaining launches may write,
  // one bit per pool page (pinned host copy, device copy, upload event)
  uint32_t *h_mask = nullptr, *d_mask = nullptr;
  hipEvent_t mask_evt = nullptr;
  bool mask_used = false;
  ~phos_ckpt() {
    if (drainer.joinable()) {  // not ended: let the kernels finish, then stop the drain
      (void)hipDeviceSynchronize();
      drain_abort.store(true, std::memory_order_release);
      drainer.join();
    }
    if (h_fill) (void)hipHostFree(h_fill);
    if (h_free_src) (void)hipHostFree(h_free_src);
    if (h_bounce) (void)hipHostFree(h_bounce);
    if (d_free_seq) (void)hipFree(d_free_seq);
    if (mask_used) (void)hipEventSynchronize(mask_evt);
    if (mask_evt) (void)hipEventDestroy(mask_evt);
    if (h_mask) (void)hipHostFree(h_mask);
    if (d_mask) (void)hipFree(d_mask);
  }
};

constexpr uint32_t kErrWait = 0, kErrOverflow = 1, kErrSegment = 2, kErrMisspec = 3, kErrWords = 4;

constexpr uint32_t kWantCap = 16384;      // asked-for pages the host can see per restore
constexpr uint64_t kDmaRunBytes = 4u << 20;  // largest single bulk DMA (one bounce slot)
constexpr uint64_t kBounceBytes = 2 * kDmaRunBytes;  // two staging slots

struct phos_rst {
  phos_ctx *ctx;
  uint32_t flags;
  const uint8_t *image;
  hipStream_t copy;
  Slot *slot;
  bool bg_started = false;
  unsigned long long *d_chunks = nullptr;  // image pieces (device table) or nullptr
  uint32_t chunk_pages = 0;
  // pieces in pageable host memory: the kernels cannot read them, so their
  // pages are held for the host at begin, moved by the copy engines from a
  // host thread, and published as present when the DMA has landed
  uint8_t *d_pageable = nullptr;           // per piece: 1 = pageable
  bool want = false;                       // waiters ask the host (the context's h_want)
  bool host_image = false;                 // the image (or a piece) is in host memory
  std::thread dma_thread;
  uint64_t dma_pages = 0;
  phos_status dma_status = PHOS_OK;
  std::string dma_error;
  std::chrono::steady_clock::time_point t_begin;
  double dma_ms = 0, dma_first_ms = -1, dma_first_issue_ms = -1, dma_first_copy_ms = -1;
  uint64_t asked_pages = 0;
  BgEvents bg;  // around the background copy (on the context's bgq)
  ~phos_rst() {
    if (dma_thread.joinable()) dma_thread.join();
    bg.destroy();
  }
};

#define HIP_TRY(x)                                                                  \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return fail(PHOS_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

template <class T>
static phos_status dalloc(T **p, size_t count) {
  *p = nullptr;
  if (!count) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) return fail(PHOS_E_NOMEM, "hipMalloc(%zu): %s", count * sizeof(T),
                                   hipGetErrorString(e));
  return PHOS_OK;
}

#define TRY(x)                        \
  do {                                \
    phos_status s_ = (x);             \
    if (s_ != PHOS_OK) return s_;     \
  } while (0)

static bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

// ------------------------------------------------------------------ context
static phos_status ctx_free(phos_ctx *c) {
  (void)hipDeviceSynchronize();
  void *ptrs[] = {c->d_page_buf, c->d_img_page, c->d_dirty, c->d_victim, c->d_err, c->d_vlist,
                  c->d_vmeta, c->d_victim_seq, c->d_vfirst, c->d_vbse,
                  c->d_vbucket, c->d_vbseg0, c->d_vbcursor, c->d_scratch,
                  c->d_cursor, c->d_tile_count, c->d_tile_off, c->d_seg_sum, c->d_seg_prefix};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (Slot &s : c->slots) {
    if (s.state) (void)hipFree(s.state);
    if (s.counters) (void)hipFree(s.counters);
    if (s.list) (void)hipFree(s.list);
    if (s.list_count) (void)hipFree(s.list_count);
  }
  if (c->h_vstage) (void)hipHostFree(c->h_vstage);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->h_vbse) (void)hipHostFree(c->h_vbse);
  if (c->vb_evt) (void)hipEventDestroy(c->vb_evt);
  if (c->h_want) (void)hipHostFree(c->h_want);
  if (c->h_bounce) (void)hipHostFree(c->h_bounce);
  if (c->hsa_inited) (void)hsa_shut_down();
  for (auto &g : c->seg_graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  if (c->d_bq) (void)hipFree(c->d_bq);
  if (c->d_bcursor) (void)hipFree(c->d_bcursor);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->v_evt) (void)hipEventDestroy(c->v_evt);
  if (c->vstage_evt) (void)hipEventDestroy(c->vstage_evt);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->bgq) (void)hipStreamDestroy(c->bgq);
  if (c->bgq_in) (void)hipEventDestroy(c->bgq_in);
  for (void *p : c->retired) (void)hipFree(p);
  for (auto &e : c->vcache) (void)hipFree(e.dev);
  delete c;
  return PHOS_OK;
}

extern "C" phos_status phos_create(int device, uint64_t pool_base, uint64_t pool_bytes,
                                   uint32_t page_bytes, phos_ctx **out) {
  if (!out) return fail(PHOS_E_INVAL, "phos_create: out is NULL");
  *out = nullptr;
  if (!is_pow2(page_bytes) || page_bytes < 4096 || page_bytes > (2u << 20))
    return fail(PHOS_E_INVAL, "page_bytes %u must be a power of two in [4 KiB, 2 MiB]", page_bytes);
  if (!pool_base || pool_base % page_bytes || !pool_bytes || pool_bytes % page_bytes)
    return fail(PHOS_E_INVAL, "pool base/size must be non-zero multiples of the page size");
  if (pool_bytes / page_bytes >= 0xFFFFFFF0ull)
    return fail(PHOS_E_INVAL, "pool has too many pages");
  if (pool_base + pool_bytes < pool_base) return fail(PHOS_E_INVAL, "pool wraps the address space");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(PHOS_E_INVAL, "no HIP device %d", device);
  DeviceGuard g(device);
  phos_ctx *c = new phos_ctx;
  c->device = device;
  c->pool_base = pool_base;
  c->pool_bytes = pool_bytes;
  c->page_bytes = page_bytes;
  c->page_shift = (uint32_t)__builtin_ctzll(page_bytes);
  c->n_pages = (uint32_t)(pool_bytes / page_bytes);
  c->nwords = (c->n_pages + 31) / 32;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = (uint32_t)prop.multiProcessorCount;
  c->bg_grid = env_u32("PHOS_BG_GRID", 2 * c->n_cu);
  c->bg_grid_host = std::max<uint32_t>(1, env_u32("PHOS_BG_GRID_HOST", 8));
  c->cow_grid = env_u32("PHOS_COW_GRID", 4 * c->n_cu);
  c->bg_batch = env_u32("PHOS_BG_BATCH", 64);
  c->bg_batch_pcie = env_u32("PHOS_BG_BATCH_PCIE", 4);
  c->copy_nt = env_u32("PHOS_COPY_NT", 1);  // streaming copies: keep the application's L2 lines
  c->finish_tiles = std::min<uint32_t>(kFuseTiles, env_u32("PHOS_VFINISH_MAX_TILES", kFuseTiles));
  c->tile_max = std::max<uint32_t>(kVQuantum, env_u32("PHOS_VTILE_MAX", 8 * kVQuantum) /
                                                  kVQuantum * kVQuantum);
  c->tile_max_track = std::max<uint32_t>(
      kVQuantum, env_u32("PHOS_VTILE_MAX", 16 * kVQuantum) / kVQuantum * kVQuantum);
  c->spin_limit = env_u32("PHOS_SPIN_LIMIT", 1u << 22);
  c->rst_pause = env_u32("PHOS_RST_PAUSE", 64);
  c->rst_hold_ms = std::min<uint32_t>(env_u32("PHOS_RST_HOLD_MS", 200), 40000);
  c->stage_threads = env_u32("PHOS_STAGE_THREADS", 4);
  c->cow_victim_window =
      std::min<uint32_t>(kVBuckets, std::max<uint32_t>(1, env_u32("PHOS_COW_VICTIM_WINDOW", 128)));
  c->cow_victim_first = std::min<uint32_t>(
      c->cow_victim_window, std::max<uint32_t>(1, env_u32("PHOS_COW_VICTIM_FIRST", 16)));
  c->stage_high_pct = env_u32("PHOS_STAGE_HIGH_PCT", 50);
  c->drain_chunk = (uint64_t)env_u32("PHOS_DRAIN_CHUNK_KB", 16384) << 10;
  c->drain_window = env_u32("PHOS_DRAIN_WINDOW", 2);
  c->rst_deep_demand = env_u32("PHOS_RST_DEEP_DEMAND", 1);
  c->cow_deep = env_u32("PHOS_COW_DEEP", 1);
  c->rst_deep_bg = env_u32("PHOS_RST_DEEP_BG", 0);
  phos_status st = PHOS_OK;
#define CK(x)                  \
  do {                         \
    st = (x);                  \
    if (st != PHOS_OK) {       \
      ctx_free(c);             \
      return st;               \
    }                          \
  } while (0)
  CK(dalloc(&c->d_page_buf, c->n_pages));
  CK(dalloc(&c->d_img_page, c->n_pages));
  CK(dalloc(&c->d_dirty, 32ull * c->nwords));
  CK(dalloc(&c->d_victim, 32ull * c->nwords));
  CK(dalloc(&c->d_victim_seq, 32ull * c->nwords));
  CK(dalloc(&c->d_err, kErrWords));
  c->vlist_cap = 2 * c->n_pages + 4096;
  CK(dalloc(&c->d_vlist, c->vlist_cap));
  CK(dalloc(&c->d_vmeta, 4));
  CK(dalloc(&c->d_vfirst, 32ull * c->nwords));
  CK(dalloc(&c->d_vbse, 2ull * kVBuckets));
  CK(dalloc(&c->d_vbucket, c->vlist_cap));
  CK(dalloc(&c->d_vbseg0, 1));
  CK(dalloc(&c->d_vbcursor, 1));
  c->scratch_cap = 1u << 20;
  CK(dalloc(&c->d_scratch, c->scratch_cap));
  CK(dalloc(&c->d_cursor, 1));
  c->tile_cap = 1u << 16;
  CK(dalloc(&c->d_tile_count, c->tile_cap));
  CK(dalloc(&c->d_tile_off, c->tile_cap));
  c->seg_cap = c->tile_cap / kSeg + 1;
  CK(dalloc(&c->d_seg_sum, c->seg_cap));
  CK(dalloc(&c->d_seg_prefix, c->seg_cap));
  auto hipck = [&](hipError_t e, const char *what) {
    if (e != hipSuccess) {
      fail(PHOS_E_HIP, "%s: %s", what, hipGetErrorString(e));
      return false;
    }
    return true;
  };
  if (!hipck(hipMemset(c->d_page_buf, 0xFF, c->n_pages * 4ull), "hipMemset") ||
      !hipck(hipMemset(c->d_img_page, 0xFF, c->n_pages * 4ull), "hipMemset") ||
      !hipck(hipMemset(c->d_dirty, 0, c->nwords * 32ull), "hipMemset") ||
      !hipck(hipMemset(c->d_victim, 0, c->nwords * 32ull), "hipMemset") ||
      !hipck(hipMemset(c->d_victim_seq, 0, c->nwords * 128ull), "hipMemset") ||
      !hipck(hipMemset(c->d_vfirst, 0xFF, c->nwords * 128ull), "hipMemset") ||
      !hipck(hipMemset(c->d_vbcursor, 0, 4), "hipMemset") ||
      !hipck(hipHostMalloc((void **)&c->h_vbse, 8ull * kVBuckets, hipHostMallocDefault),
             "hipHostMalloc") ||
      !hipck(hipEventCreateWithFlags(&c->vb_evt, hipEventDisableTiming), "hipEventCreate") ||
      !hipck(hipMemset(c->d_err, 0, 4 * kErrWords), "hipMemset") ||
      !hipck(hipMemset(c->d_vmeta, 0, 16), "hipMemset") ||
      !hipck(hipMemset(c->d_cursor, 0, 8), "hipMemset") ||
      !hipck(hipMemset(c->d_seg_sum, 0, c->seg_cap * 8), "hipMemset") ||
      !hipck(hipEventCreateWithFlags(&c->v_evt, hipEventDisableTiming), "hipEventCreate") ||
      !hipck(hipEventCreateWithFlags(&c->vstage_evt, hipEventDisableTiming), "hipEventCreate") ||
      !hipck(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking), "hipStreamCreate") ||
      !hipck(hipHostMalloc((void **)&c->h_pinned, 4096, hipHostMallocDefault), "hipHostMalloc") ||
      !hipck(hipHostMalloc((void **)&c->h_want, 4ull * (kWantCap + 1), hipHostMallocDefault),
             "hipHostMalloc") ||
      !hipck(hipHostMalloc((void **)&c->h_bounce, kBounceBytes + kDmaRunBytes / 1024,
                           hipHostMallocDefault), "hipHostMalloc") ||
      !hipck(noalloc_workspace(device, &c->na_ws), "hipGetSymbolAddress (fixed workspace)") ||
      !hipck(hipDeviceSynchronize(), "hipDeviceSynchronize")) {
    ctx_free(c);
    return PHOS_E_HIP;
  }
#undef CK
  *out = c;
  return PHOS_OK;
}

extern "C" phos_status phos_destroy(phos_ctx *c) {
  if (!c) return fail(PHOS_E_INVAL, "phos_destroy: NULL context");
  DeviceGuard g(c->device);
  for (phos_ckpt *k : c->open_ckpt) delete k;
  delete c->open_rst;
  return ctx_free(c);
}

extern "C" phos_status phos_buffers_register(phos_ctx *c, const phos_buffer *bufs, uint32_t n) {
  if (!c || (!bufs && n)) return fail(PHOS_E_INVAL, "phos_buffers_register: NULL argument");
  if (c->open_ckpt[1] || c->open_ckpt[2] || c->open_rst)
    return fail(PHOS_E_STATE, "buffers cannot change while a checkpoint or restore is open");
  const uint64_t end = c->pool_base + c->pool_bytes;
  for (uint32_t i = 0; i < n; ++i) {
    const phos_buffer &b = bufs[i];
    if (!b.bytes || b.base % c->page_bytes || b.bytes % c->page_bytes)
      return fail(PHOS_E_INVAL, "buffer %u is not page aligned whole pages", i);
    if (b.base < c->pool_base || b.base + b.bytes > end || b.base + b.bytes < b.base)
      return fail(PHOS_E_INVAL, "buffer %u lies outside the pool", i);
    if (i && b.base < bufs[i - 1].base + bufs[i - 1].bytes)
      return fail(PHOS_E_INVAL, "buffer %u overlaps or is out of order", i);
  }
  std::vector<uint32_t> page_buf(c->n_pages, kNone), img_page(c->n_pages, kNone);
  uint64_t img = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t p0 = (uint32_t)((bufs[i].base - c->pool_base) >> c->page_shift);
    const uint32_t np = (uint32_t)(bufs[i].bytes >> c->page_shift);
    for (uint32_t q = 0; q < np; ++q) {
      page_buf[p0 + q] = i;
      img_page[p0 + q] = (uint32_t)((img >> c->page_shift) + q);
    }
    img += bufs[i].bytes;
  }
  DeviceGuard g(c->device);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(c->d_page_buf, page_buf.data(), c->n_pages * 4ull, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_img_page, img_page.data(), c->n_pages * 4ull, hipMemcpyHostToDevice));
  c->bufs.assign(bufs, bufs + n);
  c->image_bytes = img;
  c->h_img_page.swap(img_page);
  c->h_img_pool.assign(img >> c->page_shift, kNone);
  for (uint32_t p = 0; p < c->n_pages; ++p)
    if (c->h_img_page[p] != kNone) c->h_img_pool[c->h_img_page[p]] = p;
  return PHOS_OK;
}

extern "C" phos_status phos_image_bytes(phos_ctx *c, uint64_t *bytes) {
  if (!c || !bytes) return fail(PHOS_E_INVAL, "phos_image_bytes: NULL argument");
  *bytes = c->image_bytes;
  return PHOS_OK;
}

// -------------------------------------------------------------- speculation
// Index of the buffer containing v (binary search over the sorted table), or -1.
static int64_t find_buffer(const std::vector<phos_buffer> &bufs, uint64_t v) {
  auto it = std::upper_bound(bufs.begin(), bufs.end(), v,
                             [](uint64_t x, const phos_buffer &b) { return x < b.base; });
  if (it == bufs.begin()) return -1;
  --it;
  return (v - it->base < it->bytes) ? (int64_t)(it - bufs.begin()) : -1;
}

extern "C" phos_status phos_spec_register(phos_ctx *c, uint32_t launch_id, const phos_arg *args,
                                          uint32_t nargs, phos_spec *out) {
  if (!c || !out || (!args && nargs)) return fail(PHOS_E_INVAL, "phos_spec_register: NULL argument");
  std::vector<phos_interval> iv;
  auto add_ptr = [&](uint64_t v, uint32_t mode) {
    const int64_t b = find_buffer(c->bufs, v);
    if (b >= 0) iv.push_back({c->bufs[b].base, c->bufs[b].base + c->bufs[b].bytes, mode, 0});
  };
  for (uint32_t i = 0; i < nargs; ++i) {
    const phos_arg &a = args[i];
    switch (a.kind) {
      case PHOS_ARG_SCALAR:
        break;
      case PHOS_ARG_PTR_CONST:
        add_ptr(a.value, PHOS_R);
        break;
      case PHOS_ARG_PTR_MUT:
        add_ptr(a.value, PHOS_R | PHOS_W);
        break;
      case PHOS_ARG_STRUCT: {
        if (a.bytes && !a.host_struct) return fail(PHOS_E_INVAL, "arg %u: struct without bytes", i);
        const uint8_t *s = (const uint8_t *)a.host_struct;
        for (uint64_t off = 0; off + 8 <= a.bytes; off += 8) {
          uint64_t v;
          memcpy(&v, s + off, 8);
          add_ptr(v, PHOS_R | PHOS_W);
        }
        break;
      }
      case PHOS_ARG_RANGE:
        if (!(a.mode & (PHOS_R | PHOS_W)) || (a.mode & ~(PHOS_R | PHOS_W)))
          return fail(PHOS_E_INVAL, "arg %u: range needs mode bits R and/or W", i);
        if (a.value + a.bytes < a.value) return fail(PHOS_E_INVAL, "arg %u: range wraps", i);
        if (a.bytes) iv.push_back({a.value, a.value + a.bytes, a.mode, 0});
        break;
      default:
        return fail(PHOS_E_INVAL, "arg %u: unknown kind %u", i, a.kind);
    }
  }
  std::sort(iv.begin(), iv.end(), [](const phos_interval &x, const phos_interval &y) {
    return x.lo != y.lo ? x.lo < y.lo : x.hi < y.hi;
  });
  std::vector<phos_interval> merged;
  for (const phos_interval &x : iv) {
    if (!merged.empty() && merged.back().lo == x.lo && merged.back().hi == x.hi)
      merged.back().mode |= x.mode;
    else
      merged.push_back(x);
  }
  if (merged.size() > kMaxIv)
    return fail(PHOS_E_INVAL, "launch names %zu intervals (max %u)", merged.size(), kMaxIv);
  uint32_t h;
  if (!c->free_specs.empty()) {
    h = c->free_specs.back();
    c->free_specs.pop_back();
  } else {
    h = (uint32_t)c->specs.size();
    c->specs.emplace_back();
  }
  c->specs[h].used = true;
  c->specs[h].launch_id = launch_id;
  c->specs[h].gen = ++c->spec_gen;
  c->specs[h].vb_gen = 0;
  c->specs[h].iv = std::move(merged);
  *out = h;
  return PHOS_OK;
}

static HostSpec *get_spec(phos_ctx *c, phos_spec s) {
  if (!c || s >= c->specs.size() || !c->specs[s].used) return nullptr;
  return &c->specs[s];
}

extern "C" phos_status phos_spec_intervals(phos_ctx *c, phos_spec s, phos_interval *out,
                                           uint32_t cap, uint32_t *n) {
  HostSpec *h = get_spec(c, s);
  if (!h || !n || (!out && cap)) return fail(PHOS_E_INVAL, "phos_spec_intervals: bad argument");
  *n = (uint32_t)h->iv.size();
  for (uint32_t i = 0; i < *n && i < cap; ++i) out[i] = h->iv[i];
  return PHOS_OK;
}

extern "C" phos_status phos_spec_release(phos_ctx *c, phos_spec s) {
  HostSpec *h = get_spec(c, s);
  if (!h) return fail(PHOS_E_INVAL, "phos_spec_release: unknown spec %u", s);
  h->used = false;
  h->iv.clear();
  c->free_specs.push_back(s);
  return PHOS_OK;
}

static DevIv to_dev(const phos_interval &x) {
  DevIv d;
  if (x.hi >= x.lo + 8 && x.hi >= 8) {
    d.lo = x.lo;
    d.span = x.hi - x.lo - 8;
  } else {
    d.lo = ~0ull;
    d.span = 0;
  }
  d.mode = x.mode;
  d.pad = 0;
  return d;
}

static void fill_devspec(const HostSpec &h, DevSpec *d) {
  d->niv = (uint32_t)h.iv.size();
  d->pad = 0;
  for (uint32_t i = 0; i < d->niv; ++i) d->iv[i] = to_dev(h.iv[i]);
}

// -------------------------------------------------------------- validation
static phos_status ensure_workspace(phos_ctx *c, uint64_t ntiles, uint64_t cap) {
  if (ntiles <= c->tile_cap && cap <= c->scratch_cap) return PHOS_OK;
  HIP_TRY(hipDeviceSynchronize());
  if (ntiles > c->tile_cap) {
    uint64_t nc = std::max<uint64_t>(ntiles, c->tile_cap * 2);
    c->retired.push_back(c->d_tile_count);
    c->retired.push_back(c->d_tile_off);
    c->retired.push_back(c->d_seg_sum);
    c->retired.push_back(c->d_seg_prefix);
    c->d_tile_count = nullptr;
    c->d_tile_off = c->d_seg_sum = c->d_seg_prefix = nullptr;
    c->tile_cap = c->seg_cap = 0;
    TRY(dalloc(&c->d_tile_count, nc));
    TRY(dalloc(&c->d_tile_off, nc));
    const uint64_t ns = nc / kSeg + 1;
    TRY(dalloc(&c->d_seg_sum, ns));
    TRY(dalloc(&c->d_seg_prefix, ns));
    HIP_TRY(hipMemset(c->d_seg_sum, 0, ns * 8));
    c->tile_cap = nc;
    c->seg_cap = ns;
  }
  if (cap > c->scratch_cap) {
    uint64_t nc = std::max<uint64_t>(cap, c->scratch_cap * 2);
    c->retired.push_back(c->d_scratch);
    c->d_scratch = nullptr;
    c->scratch_cap = 0;
    TRY(dalloc(&c->d_scratch, nc));
    c->scratch_cap = nc;
  }
  HIP_TRY(hipDeviceSynchronize());
  return PHOS_OK;
}

// Records per workgroup tile: large tiles amortize the per-tile set-up and
// the dirty-map flush, small ones keep the grid's active window of the
// record stream narrow (measured faster on HBM); small calls keep >= ~512
// tiles to fill the GPU.
static uint32_t pick_tile(const phos_ctx *c, uint64_t total, uint32_t flags) {
  const uint64_t cap = (flags & PHOS_V_TRACK) ? c->tile_max_track : c->tile_max;
  uint64_t t = kVQuantum;
  while (t * 2 <= cap && t * 2 * 512 <= total) t *= 2;
  return (uint32_t)t;
}

static VArgs base_vargs(phos_ctx *c, uint32_t flags, uint32_t tile_recs) {
  VArgs a;
  memset(&a, 0, sizeof a);
  a.flags = flags;
  a.tile_recs = tile_recs;
  a.pool_base = c->pool_base;
  a.pool_bytes = c->pool_bytes;
  a.page_shift = c->page_shift;
  a.n_pages = c->n_pages;
  a.page_buf = c->d_page_buf;
  a.dirty = c->d_dirty;
  a.victim = c->d_victim;
  a.victim_seq = c->d_victim_seq;
  a.victim_first = c->d_vfirst;
  a.vlist = c->d_vlist;
  a.vmeta = c->d_vmeta;
  a.vlist_cap = c->vlist_cap;
  a.scratch = c->d_scratch;
  a.scratch_cap = c->scratch_cap;
  a.cursor = c->d_cursor;
  a.tile_count = c->d_tile_count;
  a.tile_off = c->d_tile_off;
  a.seg_sum = c->d_seg_sum;
  return a;
}

// A new tracking window: no page has a failing write yet, no bucket exists.
static phos_status vb_reset(phos_ctx *c, hipStream_t s) {
  // the last window's bucket bounds have landed before the new window's do
  if (c->vb_evt_used) HIP_TRY(hipEventSynchronize(c->vb_evt));
  HIP_TRY(launch_fill_u32(c->d_vfirst, 32ull * c->nwords, ~0u, s));
  HIP_TRY(launch_fill_u32(c->d_vbcursor, 1, 0, s));
  ++c->vb_gen;
  c->vb_broken = false;
  std::fill(c->vb_last.begin(), c->vb_last.begin() + c->vb_hi + 1, 0u);
  c->vb_hi = 0;
  return PHOS_OK;
}

// A tracking validation numbered spec h's launch `seq`.
static void note_vb(phos_ctx *c, HostSpec *h, uint32_t seq) {
  if (h->vb_gen != c->vb_gen) {
    h->vb_gen = c->vb_gen;
    h->vb_n = 0;
  }
  ++h->vb_n;
  h->vb_seq = seq;
}

static void note_victims(phos_ctx *c, hipStream_t s) {
  c->victims_pending = true;
  if (!c->victim_stream_set) {
    c->victim_stream_set = true;
    c->victim_stream = s;
  } else if (c->victim_stream != s) {
    c->victim_streams_many = true;
  }
}

// Validations share the context's workspace, so they are serialized: a call
// on another stream than the previous one waits for it.  Under stream
// capture no event is used (captured validations must share one stream).
static phos_status run_validation(phos_ctx *c, const VArgs &a, const DevSpec *single,
                                  phos_violation *out, uint64_t cap, uint64_t *n_out,
                                  hipStream_t s, unsigned long long *seg_prefix = nullptr) {
  if (!seg_prefix) seg_prefix = c->d_seg_prefix;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cs));
  const bool capturing = cs != hipStreamCaptureStatusNone;
  if (!capturing && c->v_evt_used && s != c->v_stream) HIP_TRY(hipStreamWaitEvent(s, c->v_evt, 0));
  const bool track = (a.flags & PHOS_V_TRACK) != 0;
  // victim buckets for this call's launches (not under capture: a replay
  // would number its launches anew)
  if (track && (capturing || a.seq0 + a.nlaunch - 1 > kVBuckets)) c->vb_broken = true;
  const bool buckets = track && !c->vb_broken && a.nlaunch;
  if (buckets)
    HIP_TRY(launch_vb_snap(c->d_vmeta, c->vlist_cap, c->d_vbseg0, c->d_vbse + 2ull * (a.seq0 - 1),
                           a.nlaunch, s));
  HIP_TRY(launch_validate(a, single, track, s));
  if (track) note_victims(c, s);
  if (buckets) {
    const uint32_t k0 = a.seq0 - 1, n = a.nlaunch;
    HIP_TRY(launch_vb_build(c->d_vlist, c->d_vmeta, c->vlist_cap, c->d_vbseg0, c->d_vfirst,
                            c->n_pages, a.seq0, n, c->d_vbse + 2ull * k0, c->d_vbcursor,
                            c->d_vbucket, c->vlist_cap, s));
    HIP_TRY(hipMemcpyAsync(c->h_vbse + 2ull * k0, c->d_vbse + 2ull * k0, 8ull * n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(c->vb_evt, s));
    c->vb_evt_used = true;
    c->vb_hi = a.seq0 + n - 1;
    for (uint32_t q = a.seq0; q <= c->vb_hi; ++q) c->vb_last[q] = c->vb_hi;
  }
  uint32_t *overflow = c->d_err + kErrOverflow;
  if (a.ntiles <= c->finish_tiles) {
    HIP_TRY(launch_vfinish(a.tile_count, a.tile_off, a.ntiles, a.scratch, a.scratch_cap, out, cap,
                           n_out, a.cursor, a.seg_sum, overflow, s));
  } else {
    const uint32_t nseg = (a.ntiles + kSeg - 1) / kSeg;
    HIP_TRY(launch_vscan(a.seg_sum, nseg, seg_prefix, n_out, a.cursor, cap, overflow, s));
    HIP_TRY(launch_vscatter(a.tile_count, a.tile_off, a.ntiles, seg_prefix, a.scratch,
                            a.scratch_cap, out, cap, s));
  }
  if (!capturing) {
    HIP_TRY(hipEventRecord(c->v_evt, s));
    c->v_evt_used = true;
    c->v_stream = s;
  }
  return PHOS_OK;
}

static const uint32_t kKernelFlags = PHOS_V_READS | PHOS_V_WRITES | PHOS_V_TRACK;
static const uint32_t kFlagMask = kKernelFlags | PHOS_V_SYNC;

// PHOS_V_SYNC: wait for the call and report whether its true count exceeds cap.
static phos_status sync_count(phos_ctx *c, const uint64_t *n_out, uint64_t cap, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(PHOS_E_STATE, "PHOS_V_SYNC waits for the stream: not under stream capture");
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 16, n_out, 8, hipMemcpyDefault, s));
  HIP_TRY(hipStreamSynchronize(s));
  const uint64_t n = c->h_pinned[16];
  if (n > cap)
    return fail(PHOS_E_OVERFLOW, "%llu violations for a capacity of %llu (*n_violations holds the "
                "true count; the contents of out are unspecified)", (unsigned long long)n,
                (unsigned long long)cap);
  return PHOS_OK;
}

extern "C" phos_status phos_twin_scale_add(phos_ctx *c, phos_spec spec, const uint64_t *x,
                                           uint64_t *y, const int64_t *idx, uint64_t n,
                                           uint32_t flags, phos_violation *out, uint64_t cap,
                                           uint64_t *n_violations, hipStream_t stream) {
  if (!c) return fail(PHOS_E_INVAL, "phos_twin_scale_add: NULL context");
  if ((flags & ~kFlagMask) || (n && (!x || !y)) ||
      (flags && (!n_violations || (cap && !out) || (((uintptr_t)out) & 15))))
    return fail(PHOS_E_INVAL, "phos_twin_scale_add: bad argument");
  if (((uintptr_t)x | (uintptr_t)y | (uintptr_t)idx) & 7)
    return fail(PHOS_E_INVAL, "x, y and idx must be 8-byte aligned");
  DevSpec ds;
  ds.niv = 0;
  ds.pad = 0;
  TwinArgs a;
  memset(&a, 0, sizeof a);
  if (flags) {
    HostSpec *h = get_spec(c, spec);
    if (!h) return fail(PHOS_E_INVAL, "phos_twin_scale_add: unknown spec %u", spec);
    fill_devspec(*h, &ds);
    a.launch_id = h->launch_id;
  }
  a.x = x;
  a.y = y;
  a.idx = idx;
  a.n = n;
  a.flags = flags;
  a.pool_base = c->pool_base;
  a.pool_bytes = c->pool_bytes;
  a.page_shift = c->page_shift;
  a.page_buf = c->d_page_buf;
  a.dirty = c->d_dirty;
  a.victim = c->d_victim;
  a.victim_seq = c->d_victim_seq;
  a.seq = ++c->vseq;
  if (flags & PHOS_V_TRACK) c->vb_broken = true;  // the twin's victims have no buckets
  a.vlist = c->d_vlist;
  a.vmeta = c->d_vmeta;
  a.vlist_cap = c->vlist_cap;
  a.out = out;
  a.cap = out ? cap : 0;
  a.count = reinterpret_cast<unsigned long long *>(n_violations);
  a.overflow = c->d_err + kErrOverflow;
  // Section 4.2: with the validator inside the kernel a failing write is
  // made before it is reported, so one landing on a page the open
  // copy-on-write checkpoint has not copied is a misspeculation
  phos_ckpt *cow = c->open_ckpt[PHOS_COW];
  a.cow_state = cow ? cow->slot->state : nullptr;
  a.misspec = c->d_err + kErrMisspec;
  a.flags = flags & kKernelFlags;
  DeviceGuard g(c->device);
  if (flags) HIP_TRY(launch_fill_u64(a.count, 1, 0, stream));
  const uint64_t blocks = (n + 4 * 256 - 1) / (4 * 256);  // four elements per thread
  HIP_TRY(launch_twin(a, ds, blocks, c->n_cu, stream));
  if (flags & PHOS_V_TRACK) note_victims(c, stream);
  if (flags & PHOS_V_SYNC) return sync_count(c, n_violations, a.cap, stream);
  return PHOS_OK;
}

extern "C" phos_status phos_validate(phos_ctx *c, phos_spec spec, const uint64_t *d_records,
                                     uint64_t n, uint32_t flags, phos_violation *out,
                                     uint64_t cap, uint64_t *n_violations, hipStream_t stream) {
  HostSpec *h = get_spec(c, spec);
  if (!h) return fail(PHOS_E_INVAL, "phos_validate: unknown spec %u", spec);
  if ((n && !d_records) || (cap && !out) || (((uintptr_t)out) & 15) || !n_violations ||
      (flags & ~kFlagMask))
    return fail(PHOS_E_INVAL, "phos_validate: bad argument");
  if (((uintptr_t)d_records) & 7) return fail(PHOS_E_INVAL, "records must be 8-byte aligned");
  const uint32_t tile = pick_tile(c, n, flags);
  const uint64_t ntiles = (n + tile - 1) / tile;
  if (ntiles >= 0xFFFFFFF0ull) return fail(PHOS_E_INVAL, "too many records");
  DeviceGuard g(c->device);
  TRY(ensure_workspace(c, ntiles, cap));
  DevSpec ds;
  fill_devspec(*h, &ds);
  VArgs a = base_vargs(c, flags & kKernelFlags, tile);
  a.launches = nullptr;
  a.single.rec = d_records;
  a.single.n = n;
  a.single.launch_id = h->launch_id;
  a.single.tile0 = 0;
  a.seq0 = ++c->vseq;
  a.nlaunch = 1;
  a.ntiles = (uint32_t)ntiles;
  TRY(run_validation(c, a, &ds, out, cap, n_violations, stream));
  if (flags & PHOS_V_TRACK) note_vb(c, h, a.seq0);
  if (flags & PHOS_V_SYNC) return sync_count(c, n_violations, cap, stream);
  return PHOS_OK;
}

// phos_validate with the fixed per-GPU workspace in place of the context's
// (which grows on demand): nothing is allocated, so the call can be captured
// into a graph or made where allocation is not allowed.  Limits: at most
// kFuseTiles tiles (the one-kernel ordering) and a cap of kNaViol records.
extern "C" phos_status phos_validate_noalloc(phos_ctx *c, phos_spec spec,
                                             const uint64_t *d_records, uint64_t n,
                                             uint32_t flags, phos_violation *out, uint64_t cap,
                                             uint64_t *n_violations, hipStream_t stream) {
  HostSpec *h = get_spec(c, spec);
  if (!h) return fail(PHOS_E_INVAL, "phos_validate_noalloc: unknown spec %u", spec);
  if ((n && !d_records) || (cap && !out) || (((uintptr_t)out) & 15) || !n_violations ||
      (flags & ~kFlagMask))
    return fail(PHOS_E_INVAL, "phos_validate_noalloc: bad argument");
  if (((uintptr_t)d_records) & 7) return fail(PHOS_E_INVAL, "records must be 8-byte aligned");
  const uint32_t tile = pick_tile(c, n, flags);
  const uint64_t ntiles = (n + tile - 1) / tile;
  if (ntiles > kFuseTiles)
    return fail(PHOS_E_INVAL, "phos_validate_noalloc: %llu records need %llu tiles of %u; the "
                "fixed workspace holds %u tiles (at most %llu records per call)",
                (unsigned long long)n, (unsigned long long)ntiles, tile, kFuseTiles,
                (unsigned long long)kFuseTiles * tile);
  if (cap > kNaViol)
    return fail(PHOS_E_INVAL, "phos_validate_noalloc: cap %llu exceeds the fixed workspace's %llu "
                "violation records", (unsigned long long)cap, (unsigned long long)kNaViol);
  if (!c->na_ws) return fail(PHOS_E_STATE, "phos_validate_noalloc: no fixed workspace");
  DeviceGuard g(c->device);
  DevSpec ds;
  fill_devspec(*h, &ds);
  VArgs a = base_vargs(c, flags & kKernelFlags, tile);
  unsigned long long *clear = reinterpret_cast<unsigned long long *>(c->na_ws);
  a.cursor = clear;
  a.seg_sum = clear + 1;
  a.tile_count = reinterpret_cast<uint32_t *>(c->na_ws + kNaOffCount);
  a.tile_off = reinterpret_cast<unsigned long long *>(c->na_ws + kNaOffTileOff);
  a.scratch = reinterpret_cast<phos_violation *>(c->na_ws + kNaOffViol);
  a.scratch_cap = kNaViol;
  a.launches = nullptr;
  a.single.rec = d_records;
  a.single.n = n;
  a.single.launch_id = h->launch_id;
  a.single.tile0 = 0;
  a.seq0 = ++c->vseq;
  a.nlaunch = 1;
  a.ntiles = (uint32_t)ntiles;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cs));
  const bool capturing = cs != hipStreamCaptureStatusNone;
  // the context's validations run in call order, as with phos_validate
  if (!capturing && c->v_evt_used && stream != c->v_stream)
    HIP_TRY(hipStreamWaitEvent(stream, c->v_evt, 0));
  // the previous call on this GPU left the cursor and sums at zero unless it
  // failed part-way: clear them (with a kernel, which graph capture takes)
  HIP_TRY(launch_fill_u64(clear, kNaClearWords, 0, stream));
  HIP_TRY(launch_validate(a, &ds, (a.flags & PHOS_V_TRACK) != 0, stream));
  if (a.flags & PHOS_V_TRACK) {
    note_victims(c, stream);
    c->vb_broken = true;  // no victim buckets without the context's workspace
  }
  HIP_TRY(launch_vfinish(a.tile_count, a.tile_off, a.ntiles, a.scratch, a.scratch_cap, out, cap,
                         n_violations, a.cursor, a.seg_sum, c->d_err + kErrOverflow, stream));
  if (!capturing) {
    HIP_TRY(hipEventRecord(c->v_evt, stream));
    c->v_evt_used = true;
    c->v_stream = stream;
  }
  if (flags & PHOS_V_SYNC) return sync_count(c, n_violations, cap, stream);
  return PHOS_OK;
}

extern "C" phos_status phos_validate_batch(phos_ctx *c, const phos_spec *specs,
                                           const uint64_t *const *d_records, const uint64_t *n,
                                           uint32_t nlaunch, uint32_t flags, phos_violation *out,
                                           uint64_t cap, uint64_t *n_violations,
                                           hipStream_t stream) {
  if (!c || (nlaunch && (!specs || !d_records || !n)) || (cap && !out) || (((uintptr_t)out) & 15) ||
      !n_violations ||
      (flags & ~kFlagMask))
    return fail(PHOS_E_INVAL, "phos_validate_batch: bad argument");
  uint64_t total = 0, total_iv = 0;
  for (uint32_t i = 0; i < nlaunch; ++i) {
    HostSpec *h = get_spec(c, specs[i]);
    if (!h) return fail(PHOS_E_INVAL, "launch %u: unknown spec %u", i, specs[i]);
    if ((n[i] && !d_records[i]) || (((uintptr_t)d_records[i]) & 7))
      return fail(PHOS_E_INVAL, "launch %u: records NULL or misaligned", i);
    total += n[i];
    total_iv += h->iv.size();
  }
  const uint32_t tile = pick_tile(c, total, flags);
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < nlaunch; ++i) tiles += (n[i] + tile - 1) / tile;
  if (tiles >= 0xFFFFFFF0ull) return fail(PHOS_E_INVAL, "too many records");
  const size_t head = nlaunch * sizeof(VLaunch) + total_iv * sizeof(DevIv);
  // the cache key, and its hash (64-bit words, FNV-1a style mixing)
  std::vector<uint64_t> key(2 + 3ull * nlaunch);
  key[0] = tile;
  key[1] = nlaunch;
  for (uint32_t i = 0; i < nlaunch; ++i) {
    key[2 + 3 * i] = ((uint64_t)specs[i] << 32) ^ c->specs[specs[i]].gen;
    key[3 + 3 * i] = (uint64_t)(uintptr_t)d_records[i];
    key[4 + 3 * i] = n[i];
  }
  uint64_t hsh = 1469598103934665603ull;
  for (uint64_t w : key) hsh = (hsh ^ w) * 1099511628211ull, hsh ^= hsh >> 29;
  DeviceGuard g(c->device);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cs));
  const bool capturing = cs != hipStreamCaptureStatusNone;
  if (!capturing) TRY(ensure_workspace(c, tiles, cap));
  else if (tiles > c->tile_cap || cap > c->scratch_cap)
    return fail(PHOS_E_STATE, "workspace must be grown by an uncaptured call first");
  phos_ctx::VBatch *hit = nullptr;
  for (auto &e : c->vcache)
    if (e.hash == hsh && e.key == key) hit = &e;
  if (!hit) {
    if (capturing) return fail(PHOS_E_STATE, "batch descriptors must be uploaded before capture");
    // host image of the descriptor table, the flat interval table and the
    // launch of every tile
    std::vector<uint8_t> blob(head + 4 * tiles);
    VLaunch *L = reinterpret_cast<VLaunch *>(blob.data());
    DevIv *IV = reinterpret_cast<DevIv *>(blob.data() + nlaunch * sizeof(VLaunch));
    uint32_t *TL = reinterpret_cast<uint32_t *>(blob.data() + head);
    uint64_t ivo = 0, t0 = 0;
    for (uint32_t i = 0; i < nlaunch; ++i) {
      const HostSpec &h = c->specs[specs[i]];
      L[i].rec = d_records[i];
      L[i].n = n[i];
      L[i].iv_off = (uint32_t)ivo;
      L[i].niv = (uint32_t)h.iv.size();
      L[i].launch_id = h.launch_id;
      L[i].tile0 = (uint32_t)t0;
      for (const phos_interval &x : h.iv) IV[ivo++] = to_dev(x);
      const uint64_t nt = (n[i] + tile - 1) / tile;
      for (uint64_t t = 0; t < nt; ++t) TL[t0 + t] = i;
      t0 += nt;
    }
    if (c->vcache.size() >= 256) {  // evict the least recently used
      auto lru = std::min_element(c->vcache.begin(), c->vcache.end(),
                                  [](const phos_ctx::VBatch &x, const phos_ctx::VBatch &y) {
                                    return x.last_use < y.last_use;
                                  });
      c->retired.push_back(lru->dev);
      c->vcache.erase(lru);
    }
    if (blob.size() > c->vstage_cap) {
      if (c->vstage_used) HIP_TRY(hipEventSynchronize(c->vstage_evt));
      if (c->h_vstage) (void)hipHostFree(c->h_vstage);
      c->h_vstage = nullptr;
      const size_t cap2 = std::max<size_t>(blob.size(), 1 << 16) * 2;
      if (hipHostMalloc(&c->h_vstage, cap2, hipHostMallocDefault) != hipSuccess)
        return fail(PHOS_E_NOMEM, "hipHostMalloc(%zu)", cap2);
      c->vstage_cap = cap2;
      c->vstage_used = false;
    }
    uint8_t *dev = nullptr;
    TRY(dalloc(&dev, blob.size()));
    if (c->vstage_used) HIP_TRY(hipEventSynchronize(c->vstage_evt));
    memcpy(c->h_vstage, blob.data(), blob.size());
    if (c->v_evt_used && stream != c->v_stream) HIP_TRY(hipStreamWaitEvent(stream, c->v_evt, 0));
    HIP_TRY(hipMemcpyAsync(dev, c->h_vstage, blob.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(c->vstage_evt, stream));
    c->vstage_used = true;
    c->vcache.push_back({hsh, std::move(key), dev, 0});
    hit = &c->vcache.back();
  }
  hit->last_use = ++c->vclock;
  VArgs a = base_vargs(c, flags & kKernelFlags, tile);
  a.launches = reinterpret_cast<const VLaunch *>(hit->dev);
  a.ivs = reinterpret_cast<const DevIv *>(hit->dev + nlaunch * sizeof(VLaunch));
  a.tile_launch = reinterpret_cast<const uint32_t *>(hit->dev + head);
  a.nlaunch = nlaunch;
  a.ntiles = (uint32_t)tiles;
  a.seq0 = c->vseq + 1;  // launch i is numbered seq0 + i
  c->vseq += nlaunch;
  static DevSpec unused;  // kernel parameter of the single-launch path
  TRY(run_validation(c, a, &unused, out, cap, n_violations, stream));
  if (flags & PHOS_V_TRACK)
    for (uint32_t i = 0; i < nlaunch; ++i) note_vb(c, &c->specs[specs[i]], a.seq0 + i);
  if (flags & PHOS_V_SYNC) return sync_count(c, n_violations, cap, stream);
  return PHOS_OK;
}

extern "C" phos_status phos_stream_status(phos_ctx *c, hipStream_t s) {
  if (!c) return fail(PHOS_E_INVAL, "phos_stream_status: NULL context");
  DeviceGuard g(c->device);
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 8, c->d_err, 4 * kErrWords, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const uint32_t *w = reinterpret_cast<const uint32_t *>(c->h_pinned + 8);
  const bool ov = w[kErrOverflow] != 0, seg = w[kErrSegment] != 0;
  if (ov) HIP_TRY(launch_fill_u32(c->d_err + kErrOverflow, 1, 0, s));
  if (seg) HIP_TRY(launch_fill_u32(c->d_err + kErrSegment, 1, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (seg)
    return fail(PHOS_E_INVAL, "a phos_copy_batch call met a segment that is not 16-byte aligned "
                "or has a NULL address, and copied nothing%s",
                ov ? "; a validation also found more violations than its capacity" : "");
  if (ov) return fail(PHOS_E_OVERFLOW, "a validation found more violations than its capacity");
  return PHOS_OK;
}

static bool device_readable(const void *p, bool *in_host);

// ------------------------------------------- device-resident segment batches
// (no paper analog; the paper copies buffer by buffer in 4 MB chunks,
// Section 5)
static phos_status ensure_bq(phos_ctx *c, uint64_t nseg) {
  if (c->d_bq && nseg <= c->bq_cap) return PHOS_OK;
  HIP_TRY(hipDeviceSynchronize());
  for (auto &g : c->seg_graphs) {  // they name the old queue
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  c->seg_graphs.clear();
  if (c->d_bq) (void)hipFree(c->d_bq);
  c->d_bq = nullptr;
  const uint64_t cap = std::max<uint64_t>({nseg, 2 * c->bq_cap, 1024});
  c->bq_cap = 0;
  TRY(dalloc(&c->d_bq, 4 + cap + 1));
  if (!c->d_bcursor) TRY(dalloc(&c->d_bcursor, 1));
  c->bq_cap = cap;
  return PHOS_OK;
}

// The segment header and prefix, then the persistent copy (the same kernel
// as the batch graph's), on stream s.
static phos_status enqueue_seg_copy(phos_ctx *c, const phos_copy_seg *d_segs, uint64_t nseg,
                                    const phos_batch_cfg &cfg, hipStream_t s) {
  HIP_TRY(launch_segs_prefix(d_segs, nseg, c->d_bq, c->d_bq + 4, c->d_bcursor,
                             c->d_err + kErrSegment, s));
  BatchQ q;
  memset(&q, 0, sizeof q);
  q.segs = d_segs;
  q.hdr = c->d_bq;
  q.byte_prefix = c->d_bq + 4;
  q.cursor = c->d_bcursor;
  q.chunk_bytes = cfg.chunk_bytes;
  HIP_TRY(launch_batch_copy(q, cfg.wg_per_cu * c->n_cu, cfg.threads, s));
  return PHOS_OK;
}

static phos_status seg_args_ok(phos_ctx *c, const phos_copy_seg *d_segs, uint64_t nseg,
                               const char *who) {
  if (!c || (nseg && !d_segs)) return fail(PHOS_E_INVAL, "%s: NULL argument", who);
  if (((uintptr_t)d_segs) & 7) return fail(PHOS_E_INVAL, "%s: segments must be 8-byte aligned", who);
  if (nseg > (1ull << 32)) return fail(PHOS_E_INVAL, "%s: too many segments", who);
  if (nseg && !device_readable(d_segs, nullptr))
    return fail(PHOS_E_INVAL, "%s: segments must be in device (or pinned host) memory", who);
  return PHOS_OK;
}

extern "C" phos_status phos_copy_batch(phos_ctx *c, const phos_copy_seg *d_segs, uint64_t nseg,
                                       hipStream_t stream) {
  TRY(seg_args_ok(c, d_segs, nseg, "phos_copy_batch"));
  if (!nseg) return PHOS_OK;
  DeviceGuard g(c->device);
  TRY(ensure_bq(c, nseg));
  return enqueue_seg_copy(c, d_segs, nseg, batch_default_cfg(), stream);
}

extern "C" phos_status phos_copy_batch_tuned(phos_ctx *c, const phos_copy_seg *d_segs,
                                             uint64_t nseg, hipStream_t stream) {
  TRY(seg_args_ok(c, d_segs, nseg, "phos_copy_batch_tuned"));
  if (!nseg) return PHOS_OK;
  DeviceGuard g(c->device);
  TRY(ensure_bq(c, nseg));
  phos_ctx::SegGraph *hit = nullptr;
  for (auto &e : c->seg_graphs)
    if (e.segs == d_segs && e.nseg == nseg) hit = &e;
  if (!hit) {
    // first call for these segments: read them (synchronously), tune on
    // them (the tuner performs the copies), capture the graph
    std::vector<phos_copy_seg> h(nseg);
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(h.data(), d_segs, nseg * sizeof(phos_copy_seg), hipMemcpyDefault));
    for (uint64_t i = 0; i < nseg; ++i) {
      const phos_copy_seg &x = h[i];
      if (((x.src | x.dst | x.bytes) & 15) || (x.bytes && (!x.src || !x.dst)))
        return fail(PHOS_E_INVAL, "segment %llu: addresses and size must be non-NULL 16-byte "
                    "multiples", (unsigned long long)i);
      h[i].req = 0;  // the tuner's per-request accounting is not needed
    }
    phos_batch_cfg cfg = batch_default_cfg();
    TRY(phos_batch_tune(c->device, h.data(), nseg, getenv("PHOS_TUNE_CACHE"), &cfg, nullptr));
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (c->seg_graphs.size() >= 16) {  // evict the least recently used
      auto lru = std::min_element(c->seg_graphs.begin(), c->seg_graphs.end(),
                                  [](const phos_ctx::SegGraph &x, const phos_ctx::SegGraph &y) {
                                    return x.last_use < y.last_use;
                                  });
      HIP_TRY(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(lru->exec);
      (void)hipGraphDestroy(lru->graph);
      c->seg_graphs.erase(lru);
    }
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const phos_status st = enqueue_seg_copy(c, d_segs, nseg, cfg, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
    if (st != PHOS_OK || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return st != PHOS_OK ? st : fail(PHOS_E_HIP, "graph capture: %s", hipGetErrorString(e2));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(PHOS_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    }
    c->seg_graphs.push_back({d_segs, nseg, cfg, exec, graph, 0});
    hit = &c->seg_graphs.back();
  }
  hit->last_use = ++c->seg_clock;
  HIP_TRY(hipGraphLaunch(hit->exec, stream));
  return PHOS_OK;
}

// ------------------------------------------------------------ image manifest
// Section 2.2: the checkpointed state is the process's buffers; an image is
// their bytes back to back in ascending base order.  The manifest says which
// buffers those were, so a restore can refuse an image that does not match
// the buffers registered for it.
namespace {
constexpr char kManifestMagic[8] = {'P', 'H', 'O', 'S', 'I', 'M', 'G', '1'};
struct ManifestHead {
  char magic[8];
  uint32_t version, protocol;
  uint32_t page_bytes, n_buffers;
  uint64_t image_bytes;
};
static_assert(sizeof(ManifestHead) == 32, "manifest header is 32 bytes");
uint64_t fnv1a(const uint8_t *p, uint64_t n) {
  uint64_t h = 1469598103934665603ull;
  for (uint64_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}
uint64_t manifest_bytes(uint64_t n_buffers) { return sizeof(ManifestHead) + 16 * n_buffers + 8; }
}  // namespace

extern "C" phos_status phos_manifest_write(phos_ctx *c, uint32_t protocol, void *out, uint64_t cap,
                                           uint64_t *bytes) {
  if (!c || !bytes) return fail(PHOS_E_INVAL, "phos_manifest_write: NULL argument");
  if (protocol > PHOS_RECOPY) return fail(PHOS_E_INVAL, "unknown protocol %u", protocol);
  const uint64_t need = manifest_bytes(c->bufs.size());
  *bytes = need;
  if (!out) return PHOS_OK;  // size query
  if (cap < need) return fail(PHOS_E_OVERFLOW, "manifest needs %llu bytes", (unsigned long long)need);
  std::vector<uint8_t> m(need);
  ManifestHead h;
  memcpy(h.magic, kManifestMagic, 8);
  h.version = 1;
  h.protocol = protocol;
  h.page_bytes = c->page_bytes;
  h.n_buffers = (uint32_t)c->bufs.size();
  h.image_bytes = c->image_bytes;
  memcpy(m.data(), &h, sizeof h);
  uint8_t *p = m.data() + sizeof h;
  for (const phos_buffer &b : c->bufs) {
    const uint64_t rel[2] = {b.base - c->pool_base, b.bytes};
    memcpy(p, rel, 16);
    p += 16;
  }
  const uint64_t sum = fnv1a(m.data(), need - 8);
  memcpy(p, &sum, 8);
  memcpy(out, m.data(), need);
  return PHOS_OK;
}

extern "C" phos_status phos_manifest_check(phos_ctx *c, const void *manifest, uint64_t bytes) {
  if (!c || !manifest) return fail(PHOS_E_INVAL, "phos_manifest_check: NULL argument");
  const uint8_t *m = static_cast<const uint8_t *>(manifest);
  ManifestHead h;
  if (bytes < sizeof h + 8) return fail(PHOS_E_INVAL, "manifest: %llu bytes is too short",
                                        (unsigned long long)bytes);
  memcpy(&h, m, sizeof h);
  if (memcmp(h.magic, kManifestMagic, 8) || h.version != 1)
    return fail(PHOS_E_INVAL, "manifest: not an image manifest of this format");
  if (bytes != manifest_bytes(h.n_buffers))
    return fail(PHOS_E_INVAL, "manifest: %llu bytes for %u buffers", (unsigned long long)bytes,
                h.n_buffers);
  uint64_t sum;
  memcpy(&sum, m + bytes - 8, 8);
  if (sum != fnv1a(m, bytes - 8)) return fail(PHOS_E_INVAL, "manifest: checksum mismatch");
  if (h.page_bytes != c->page_bytes || h.n_buffers != c->bufs.size() ||
      h.image_bytes != c->image_bytes)
    return fail(PHOS_E_INVAL, "manifest: image of %u buffers, %llu bytes, %u-byte pages; this "
                "context has %zu buffers, %llu bytes, %u-byte pages", h.n_buffers,
                (unsigned long long)h.image_bytes, h.page_bytes, c->bufs.size(),
                (unsigned long long)c->image_bytes, c->page_bytes);
  // buffer i of the image goes to registered buffer i: their sizes must agree
  // (their places in the pool may differ from the checkpointed process's)
  for (uint32_t i = 0; i < h.n_buffers; ++i) {
    uint64_t rel[2];
    memcpy(rel, m + sizeof h + 16ull * i, 16);
    if (rel[1] != c->bufs[i].bytes)
      return fail(PHOS_E_INVAL, "manifest: buffer %u holds %llu bytes in the image, %llu here", i,
                  (unsigned long long)rel[1], (unsigned long long)c->bufs[i].bytes);
  }
  return PHOS_OK;
}

extern "C" phos_status phos_track_reset(phos_ctx *c, hipStream_t s) {
  if (!c) return fail(PHOS_E_INVAL, "phos_track_reset: NULL context");
  if (c->open_ckpt[PHOS_RECOPY])
    return fail(PHOS_E_STATE, "the page maps of an open recopy checkpoint cannot be reset");
  DeviceGuard g(c->device);
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(c->d_dirty), 8ull * c->nwords, 0, s));
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(c->d_victim), 8ull * c->nwords, 0, s));
  HIP_TRY(launch_fill_u32(c->d_victim_seq, 32ull * c->nwords, 0, s));
  c->vseq = 0;
  HIP_TRY(launch_fill_u32(c->d_vmeta, 4, 0, s));
  TRY(vb_reset(c, s));
  c->victims_pending = false;  // the list is empty again
  c->victim_stream_set = c->victim_streams_many = false;
  return PHOS_OK;
}

extern "C" phos_status phos_track_read(phos_ctx *c, uint32_t which, uint32_t *host, uint64_t nw) {
  if (!c || !host || which > 1 || nw < c->nwords)
    return fail(PHOS_E_INVAL, "phos_track_read: bad argument");
  DeviceGuard g(c->device);
  HIP_TRY(hipDeviceSynchronize());
  uint32_t *tmp = nullptr;
  TRY(dalloc(&tmp, c->nwords));
  hipError_t e = launch_bytes_to_bits(which ? c->d_victim : c->d_dirty, c->nwords, tmp, c->aux);
  if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, c->nwords * 4ull, hipMemcpyDeviceToHost, c->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(PHOS_E_HIP, "track readback: %s", hipGetErrorString(e));
  return PHOS_OK;
}

// ---------------------------------------------------------------- protocols
static phos_status ensure_slot(phos_ctx *c, Slot &s, bool with_list) {
  if (!s.state) TRY(dalloc(&s.state, c->n_pages));
  if (!s.counters) TRY(dalloc(&s.counters, kSlotCounters));
  if (with_list && !s.list) {
    TRY(dalloc(&s.list, c->n_pages));
    TRY(dalloc(&s.list_count, 1));
  }
  return PHOS_OK;
}

// Can this device's kernels read the memory at p (device memory or pinned
// host memory)?  Pageable host memory cannot be read without page faults.
static bool device_readable(const void *p, bool *in_host = nullptr) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    if (in_host) *in_host = true;
    return false;
  }
  if (in_host) *in_host = at.type != hipMemoryTypeDevice;
  return at.type != hipMemoryTypeUnregistered;
}

static CopyArgs copy_args(phos_ctx *c, Slot &s, uint8_t *image, bool to_image,
                          unsigned long long *stat) {
  CopyArgs a;
  a.pool = reinterpret_cast<uint8_t *>(c->pool_base);
  a.image = image;
  a.state = s.state;
  a.img_page = c->d_img_page;
  a.stat = stat;
  a.err = c->d_err + kErrWait;
  a.page_shift = c->page_shift;
  a.n_pages = c->n_pages;
  a.to_image = to_image ? 1u : 0u;
  a.spin_limit = c->spin_limit;
  a.nt = c->copy_nt;
  a.chunk_pages = 0;
  a.image_chunks = nullptr;
  return a;
}

// over_pcie: the copy reads host memory, so a claimed-but-not-copied page
// takes PCIe time to arrive; claim less far ahead for on-demand waiters.
static phos_status ensure_bgq(phos_ctx *c) {
  if (c->bgq) return PHOS_OK;
  std::vector<uint32_t> mask((c->n_cu + 31) / 32, 0xFFFFFFFFu);
  HIP_TRY(hipExtStreamCreateWithCUMask(&c->bgq, (uint32_t)mask.size(), mask.data()));
  HIP_TRY(hipEventCreateWithFlags(&c->bgq_in, hipEventDisableTiming));
  return PHOS_OK;
}

// The background stream runs after the work already enqueued on `after`;
// `after` itself does not wait for the copy (a stream sharing a hardware
// queue with the application would hold the application's kernels behind
// it), so whoever needs the copy finished waits for *done.
static phos_status bgq_after(phos_ctx *c, hipStream_t after) {
  TRY(ensure_bgq(c));
  HIP_TRY(hipEventRecord(c->bgq_in, after));
  HIP_TRY(hipStreamWaitEvent(c->bgq, c->bgq_in, 0));
  return PHOS_OK;
}

static phos_status bgq_mark(phos_ctx *c, hipEvent_t *e) {
  if (!*e) HIP_TRY(hipEventCreate(e));
  HIP_TRY(hipEventRecord(*e, c->bgq));
  return PHOS_OK;
}

static phos_status start_background_args(phos_ctx *c, Slot &s, const CopyArgs &a,
                                         hipStream_t stream, BgEvents *ev,
                                         bool over_pcie = false) {
  (void)s;
  TRY(bgq_after(c, stream));
  TRY(bgq_mark(c, &ev->start));
  // groups of 64 KiB: one page at 64 KiB pages, 16 at 4 KiB pages
  const uint32_t grab = std::max<uint32_t>(1, (64u << 10) >> c->page_shift);
  const uint32_t groups = (c->n_pages + grab - 1) / grab;
  const uint32_t batch = std::max<uint32_t>(1, over_pcie ? c->bg_batch_pcie : c->bg_batch);
  // Stores to host memory are posted: a full grid keeps megabytes of them
  // queued for a 50 GB/s link, and the application's own memory traffic
  // waits behind them (measured: launches ran only once the whole copy had
  // ended).  A few blocks fill the link.
  // Device copies: two blocks per CU (18 waves) copy faster beside the
  // application than one; reads of a host image keep one per CU.
  const uint32_t grid = !over_pcie ? c->bg_grid
                        : a.to_image ? std::min(c->bg_grid, c->bg_grid_host)
                                     : std::min(c->bg_grid, c->n_cu);
  HIP_TRY(launch_background(a, grab, batch, std::min(grid, groups), c->bgq));
  return bgq_mark(c, &ev->done);
}

static phos_status start_background(phos_ctx *c, Slot &s, uint8_t *image, bool to_image,
                                    hipStream_t stream, BgEvents *ev, bool skip_traced = false,
                                    bool over_pcie = false) {
  CopyArgs a = copy_args(c, s, image, to_image, &s.counters[1]);
  a.bg_exit = to_image ? &s.counters[6] : nullptr;  // [6], [7]: completion (reset at begin)
  if (skip_traced) {  // recopy: pages traced as written are left to the recopy
    a.skip_dirty = c->d_dirty;
    a.skip_victim = c->d_victim;
  }
  return start_background_args(c, s, a, stream, ev, over_pcie);
}

// Pages of the intervals with any of `modes`, clamped to the pool.
static PageRanges page_ranges(phos_ctx *c, const HostSpec &h, uint32_t modes) {
  PageRanges r;
  memset(&r, 0, sizeof r);
  const uint64_t end = c->pool_base + c->pool_bytes;
  for (const phos_interval &x : h.iv) {
    if (!(x.mode & modes) || x.hi <= x.lo) continue;
    const uint64_t lo = std::max(x.lo, c->pool_base), hi = std::min(x.hi, end);
    if (hi <= lo) continue;
    const uint32_t p0 = (uint32_t)((lo - c->pool_base) >> c->page_shift);
    const uint32_t p1 = (uint32_t)((hi - 1 - c->pool_base) >> c->page_shift);
    r.p0[r.n] = p0;
    r.np[r.n] = p1 - p0 + 1;
    r.units_prefix[r.n + 1] = r.units_prefix[r.n] + (r.np[r.n] + kUnitPages - 1) / kUnitPages;
    ++r.n;
  }
  return r;
}

// Bit p of `bits` for every page p of the ranges: all set? / set them.
static bool ranges_all_set(const std::vector<uint64_t> &bits, const PageRanges &r) {
  for (uint32_t i = 0; i < r.n; ++i)
    for (uint64_t p = r.p0[i], e = (uint64_t)r.p0[i] + r.np[i]; p < e;) {
      const uint64_t w = p >> 6, lo = p & 63, hi = std::min<uint64_t>(64, lo + (e - p));
      const uint64_t m = (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
      if ((bits[w] & m) != m) return false;
      p += hi - lo;
    }
  return true;
}

static void ranges_set(std::vector<uint64_t> &bits, const PageRanges &r) {
  for (uint32_t i = 0; i < r.n; ++i)
    for (uint64_t p = r.p0[i], e = (uint64_t)r.p0[i] + r.np[i]; p < e;) {
      const uint64_t w = p >> 6, lo = p & 63, hi = std::min<uint64_t>(64, lo + (e - p));
      bits[w] |= (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
      p += hi - lo;
    }
}

extern "C" phos_status phos_ckpt_begin(phos_ctx *c, uint32_t protocol, uint32_t flags, void *image,
                                       void *host_image, hipStream_t copy, phos_ckpt **out) {
  if (!c || !image || !out) return fail(PHOS_E_INVAL, "phos_ckpt_begin: NULL argument");
  if (protocol != PHOS_COW && protocol != PHOS_RECOPY)
    return fail(PHOS_E_INVAL, "unknown protocol %u", protocol);
  if (flags & ~PHOS_CKPT_DEFER_BACKGROUND) return fail(PHOS_E_INVAL, "unknown flags 0x%x", flags);
  if (((uintptr_t)image) & 15) return fail(PHOS_E_INVAL, "image must be 16-byte aligned");
  if (c->open_ckpt[protocol]) return fail(PHOS_E_STATE, "a checkpoint of this protocol is open");
  if (c->open_rst) return fail(PHOS_E_STATE, "a restore is open");
  DeviceGuard g(c->device);
  Slot &s = c->slots[protocol];
  TRY(ensure_slot(c, s, protocol == PHOS_RECOPY));
  // Quiesce point: reset per-page states, counters, and (first open
  // checkpoint) the write-set tracking bitmaps.
  // (On the private stream, synchronized here, so that a second checkpoint
  // opened beside this one does not wait for this one's background copy.)
  HIP_TRY(launch_fill_u32(s.state, c->n_pages, kFree, c->aux));
  HIP_TRY(launch_fill_u64(s.counters, kSlotCounters, 0, c->aux));
  if (s.list_count) HIP_TRY(launch_fill_u32(s.list_count, 1, 0, c->aux));
  if (!c->open_ckpt[PHOS_COW] && !c->open_ckpt[PHOS_RECOPY]) {
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(c->d_dirty), 8ull * c->nwords, 0, c->aux));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(c->d_victim), 8ull * c->nwords, 0, c->aux));
    HIP_TRY(launch_fill_u32(c->d_victim_seq, 32ull * c->nwords, 0, c->aux));
    c->vseq = 0;
    HIP_TRY(launch_fill_u32(c->d_vmeta, 4, 0, c->aux));
    TRY(vb_reset(c, c->aux));
    c->victims_pending = false;
    c->victim_stream_set = c->victim_streams_many = false;
  }
  HIP_TRY(hipStreamSynchronize(c->aux));
  phos_ckpt *k = new phos_ckpt;
  k->ctx = c;
  k->protocol = protocol;
  k->flags = flags;
  k->image = (uint8_t *)image;
  k->host_image = host_image;
  k->copy = copy;
  k->slot = &s;
  if (!device_readable(image, &k->host)) {
    delete k;
    return fail(PHOS_E_INVAL, "the image must be device or pinned host memory");
  }
  if (!(flags & PHOS_CKPT_DEFER_BACKGROUND)) {
    phos_status st = start_background(c, s, k->image, true, copy, &k->bg,
                                      protocol == PHOS_RECOPY, k->host);
    if (st != PHOS_OK) {
      k->bg.destroy();
      delete k;
      return st;
    }
    k->bg_started = true;
  }
  c->open_ckpt[protocol] = k;
  *out = k;
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_start(phos_ckpt *k, hipStream_t after) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_start: NULL checkpoint");
  if (k->bg_started) return fail(PHOS_E_STATE, "the background copy has started");
  if (k->recopied) return fail(PHOS_E_STATE, "recopy already done");
  phos_ctx *c = k->ctx;
  DeviceGuard g(c->device);
  if (after) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t he = hipEventRecord(e, after);
    if (he == hipSuccess) he = hipStreamWaitEvent(k->copy, e, 0);
    (void)hipEventDestroy(e);
    if (he != hipSuccess) return fail(PHOS_E_HIP, "phos_ckpt_start: %s", hipGetErrorString(he));
  }
  TRY(start_background(c, *k->slot, k->image, true, k->copy, &k->bg,
                       k->protocol == PHOS_RECOPY, k->host));
  k->bg_started = true;
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_start_pair(phos_ckpt *a, phos_ckpt *b, hipStream_t after) {
  if (!a || !b) return fail(PHOS_E_INVAL, "phos_ckpt_start_pair: NULL checkpoint");
  if (a->protocol != PHOS_COW || b->protocol != PHOS_RECOPY || a->ctx != b->ctx)
    return fail(PHOS_E_INVAL, "phos_ckpt_start_pair takes a copy-on-write and a recopy checkpoint "
                "of one context");
  if (a->bg_started || b->bg_started) return fail(PHOS_E_STATE, "a background copy has started");
  if (b->recopied) return fail(PHOS_E_STATE, "recopy already done");
  if (a->host || b->host || a->stage)
    return fail(PHOS_E_INVAL, "the shared background pass copies into device images only");
  phos_ctx *c = a->ctx;
  DeviceGuard g(c->device);
  if (after) TRY(bgq_after(c, after));
  TRY(bgq_after(c, a->copy));
  if (b->copy != a->copy) TRY(bgq_after(c, b->copy));
  TRY(bgq_mark(c, &a->bg.start));
  TRY(bgq_mark(c, &b->bg.start));
  Slot &sa = *a->slot, &sb = *b->slot;
  CopyArgs x = copy_args(c, sa, a->image, true, &sa.counters[1]);
  x.bg_exit = &sa.counters[6];
  x.image2 = b->image;
  x.state2 = sb.state;
  x.stat2 = &sb.counters[1];
  x.stat_read = &sa.counters[4];
  x.skip_dirty = c->d_dirty;
  x.skip_victim = c->d_victim;
  const uint32_t grab = std::max<uint32_t>(1, (64u << 10) >> c->page_shift);
  const uint32_t groups = (c->n_pages + grab - 1) / grab;
  HIP_TRY(launch_background_pair(x, grab, std::max<uint32_t>(1, c->bg_batch),
                                 std::min(c->bg_grid, groups), c->bgq));
  a->bg_started = b->bg_started = true;
  a->pair = 1;
  b->pair = 2;
  TRY(bgq_mark(c, &a->bg.done));
  TRY(bgq_mark(c, &b->bg.done));
  return PHOS_OK;
}

static phos_status dma_engines_ready(phos_ctx *c);
static void stage_drain_main(phos_ckpt *k);
namespace {
constexpr uint32_t kDrainBounces = 8;            // drain batches in flight
constexpr uint64_t kDrainBatchBytes = 16u << 20;  // largest drain batch (one bounce buffer)
}  // namespace

extern "C" phos_status phos_ckpt_staging(phos_ckpt *k, void *staging, uint64_t bytes) {
  return phos_ckpt_staging_policy(k, staging, bytes, PHOS_STAGE_HOST_DIRECT);
}

extern "C" phos_status phos_ckpt_staging_policy(phos_ckpt *k, void *staging, uint64_t bytes,
                                                uint32_t policy) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_staging: NULL checkpoint");
  if (policy != PHOS_STAGE_HOST_DIRECT && policy != PHOS_STAGE_BLOCK)
    return fail(PHOS_E_INVAL, "unknown staging policy %u", policy);
  if (k->protocol != PHOS_COW) return fail(PHOS_E_STATE, "staging needs a CoW checkpoint");
  if (k->stage || k->cow_stream) return fail(PHOS_E_STATE, "staging set twice or after a CoW call");
  phos_ctx *c = k->ctx;
  if (!k->host) return fail(PHOS_E_INVAL, "staging is for a checkpoint into a host image");
  const uint64_t cap = std::min<uint64_t>(bytes >> c->page_shift, c->n_pages);
  if (!cap) return PHOS_OK;  // no staging: every copy goes straight to the image
  bool in_host = true;
  if (!staging || ((uintptr_t)staging & 15) || !device_readable(staging, &in_host) || in_host)
    return fail(PHOS_E_INVAL, "staging must be 16-byte aligned device memory");
  DeviceGuard g(c->device);
  TRY(dalloc(&k->d_stage_page, cap));
  phos_status st = dalloc(&k->d_stage_head, 1);
  if (st == PHOS_OK && (launch_fill_u64(k->d_stage_head, 1, 0, c->aux) != hipSuccess ||
                        hipStreamSynchronize(c->aux) != hipSuccess))
    st = fail(PHOS_E_HIP, "staging set-up");
  if (st != PHOS_OK) {
    (void)hipFree(k->d_stage_page);
    if (k->d_stage_head) (void)hipFree(k->d_stage_head);
    k->d_stage_page = nullptr;
    k->d_stage_head = nullptr;
    return st;
  }
  k->stage = static_cast<uint8_t *>(staging);
  k->stage_cap = (uint32_t)cap;
  if (policy == PHOS_STAGE_BLOCK) {
    // the ring's control words, then the host's drain
    st = dma_engines_ready(c);
    k->drain_batch_slots =
        (uint32_t)std::min<uint64_t>(cap, std::max<uint64_t>(1, kDrainBatchBytes >> c->page_shift));
    k->drain_threads = std::min<uint32_t>(64, std::max<uint32_t>(1, c->stage_threads));
    k->drain_high_pct = std::min<uint32_t>(100, c->stage_high_pct);
    if (st == PHOS_OK &&
        (hipHostMalloc((void **)&k->h_fill, 8ull * cap, hipHostMallocDefault) != hipSuccess ||
         hipHostMalloc((void **)&k->h_free_src, 4ull * cap, hipHostMallocDefault) != hipSuccess ||
         hipHostMalloc((void **)&k->h_bounce,
                       (uint64_t)kDrainBounces * k->drain_batch_slots * c->page_bytes,
                       hipHostMallocDefault) != hipSuccess))
      st = fail(PHOS_E_NOMEM, "pinned staging control words and bounce buffers (%llu slots)",
                (unsigned long long)cap);
    if (st == PHOS_OK) st = dalloc(&k->d_free_seq, cap);
    if (st == PHOS_OK && (launch_fill_u32(k->d_free_seq, cap, 0, c->aux) != hipSuccess ||
                          hipStreamSynchronize(c->aux) != hipSuccess))
      st = fail(PHOS_E_HIP, "staging set-up");
    if (st != PHOS_OK) {
      k->stage = nullptr;  // the checkpoint goes on without staging
      k->stage_cap = 0;
      return st;
    }
    memset(k->h_fill, 0, 8ull * cap);
    k->stage_block = true;
    k->drainer = std::thread(stage_drain_main, k);
  }
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_cow(phos_ckpt *k, phos_spec spec, hipStream_t app) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_cow: NULL checkpoint");
  if (k->protocol != PHOS_COW) return fail(PHOS_E_STATE, "copy-on-write needs a CoW checkpoint");
  phos_ctx *c = k->ctx;
  HostSpec *h = get_spec(c, spec);
  if (!h) return fail(PHOS_E_INVAL, "phos_ckpt_cow: unknown spec %u", spec);
  DeviceGuard g(c->device);
  // Once the background copy is known to have finished, every page has been
  // copied or claimed by an earlier copy-on-write on this same stream, so
  // there is nothing left to do (not under stream capture: a graph may be
  // replayed while a later checkpoint's background copy still runs).
  if (k->cow_stream && k->cow_stream != app) k->cow_streams_many = true;
  k->cow_stream = app;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(app, &cs));
  if (cs == hipStreamCaptureStatusNone && k->bg.done && !k->cow_streams_many) {
    if (!k->bg_known_done) {
      const hipError_t q = hipEventQuery(k->bg.done);
      if (q == hipSuccess) k->bg_known_done = true;
      else if (q != hipErrorNotReady) return fail(PHOS_E_HIP, "hipEventQuery: %s", hipGetErrorString(q));
    }
    if (k->bg_known_done) return PHOS_OK;
  }
  const PageRanges r = page_ranges(c, *h, PHOS_W);
  const bool capturing = cs != hipStreamCaptureStatusNone;
  // Victim pages may be new since the last call unless the host knows
  // otherwise in device order (every tracking call on this stream).
  const bool victims_unsure =
      c->victim_streams_many || (c->victim_stream_set && c->victim_stream != app);
  const bool victims_new = c->victims_pending || victims_unsure || capturing;
  // A page an earlier call on this same stream asked for is done before
  // this launch runs (stream order): with all of this launch's write pages
  // asked for and no victim page possibly new, there is nothing to do.
  const bool exact = !capturing && !k->cow_streams_many && !victims_unsure;
  // Victim pages by launch: a spec validated once (with tracking) in this
  // tracking window is launch number h->vb_seq; the victim pages each launch
  // is the first to write form its bucket.  A call takes the buckets of a
  // window of launch numbers at once, from the first not yet taken through
  // at least this launch's (cow_victim_window of them, cow_victim_first for
  // the first call, whose copy the first launch waits for; never past the
  // end of the validation call that built them), so most calls have none to
  // take; later launches' pages wait for their window or for the background
  // copy.  A host image with a device staging area takes them all in the
  // first call: staging runs at HBM speed, while the background copy
  // crosses PCIe far behind the launches (with the blocking policy only when
  // the ring holds half the pool's pages; a smaller ring would fill and
  // stall the first launch).  Consecutive buckets lie consecutively in the bucket array, so a
  // window is one range, whose size the host knows once the bucket bounds
  // have reached it.  A launch number without a bucket sends the call to
  // the appended list.
  bool bucketed = exact && !c->vb_broken && h->vb_gen == c->vb_gen && h->vb_n == 1 &&
                  h->vb_seq >= 1 && h->vb_seq <= c->vb_hi;
  const bool all_at_once = k->stage && (!k->stage_block || 2ull * k->stage_cap >= c->n_pages);
  uint32_t win_lo = 0, win_hi = 0;  // launch numbers of the buckets this call takes (0: none)
  int64_t bucket_size = -1;          // their pages, -1: unknown
  if (bucketed) {
    if (k->vb_cov_gen != c->vb_gen) {
      k->vb_cov_gen = c->vb_gen;
      k->vb_covered = 0;
    }
    if (h->vb_seq > k->vb_covered) {
      win_lo = k->vb_covered + 1;
      for (uint32_t q = win_lo; q <= h->vb_seq && bucketed; ++q) bucketed = c->vb_last[q] != 0;
      if (bucketed)
        win_hi = std::max(h->vb_seq,
                          std::min(c->vb_last[h->vb_seq],
                                   win_lo - 1 + (all_at_once   ? kVBuckets
                                                 : win_lo == 1 ? c->cow_victim_first
                                                               : c->cow_victim_window)));
    }
  }
  if (bucketed) {
    if (!win_lo) {
      bucket_size = 0;
    } else {
      const hipError_t q = hipEventQuery(c->vb_evt);
      if (q == hipSuccess)
        bucket_size = (int64_t)c->h_vbse[2ull * (win_hi - 1) + 1] - c->h_vbse[2ull * (win_lo - 1)];
      else if (q != hipErrorNotReady)
        return fail(PHOS_E_HIP, "hipEventQuery: %s", hipGetErrorString(q));
    }
  }
  if (exact) {
    if (k->requested.empty()) k->requested.assign((c->n_pages + 63) / 64, 0);
    if ((bucketed ? bucket_size == 0 : !victims_new) && ranges_all_set(k->requested, r))
      return PHOS_OK;
  }
  CopyArgs a = copy_args(c, *k->slot, k->image, true, &k->slot->counters[2]);
  // once the background copy has finished every page is done, provided the
  // earlier copy-on-write calls (one stream) have completed
  a.bg_exit = &k->slot->counters[6];
  a.skip_when_finished = k->cow_streams_many ? 0u : 1u;
  a.deep = c->cow_deep ? 1u : 0u;
  if (k->stage) {
    a.stage = k->stage;
    a.stage_page = k->d_stage_page;
    a.stage_head = k->d_stage_head;
    a.stage_cap = k->stage_cap;
    if (k->stage_block) {
      a.stage_block = 1;
      a.fill = k->h_fill;
      a.free_seq = k->d_free_seq;
    }
  }
  // with tracking calls on other streams the list may be appended to while
  // this launch reads it: the victim map (marks only ever added, complete
  // for every call this stream has waited for) is scanned instead
  VictimList v{c->d_vlist, c->d_vmeta, c->vlist_cap, c->d_victim, c->nwords,
               victims_unsure ? 1u : 0u};
  uint32_t victim_blocks = victims_new ? c->cow_grid : 8u;
  if (bucketed) {
    if (win_lo) {
      v.bucket = c->d_vbucket;
      v.bstart = c->d_vbse + 2ull * (win_lo - 1);
      v.bend = c->d_vbse + 2ull * (win_hi - 1) + 1;
      victim_blocks = bucket_size < 0 ? c->cow_grid
                      : (uint32_t)std::min<int64_t>(c->cow_grid,
                                                    (bucket_size + kVictimUnit - 1) / kVictimUnit);
    } else {
      v.meta = nullptr;  // no victim work in this call
      victim_blocks = 0;
    }
  }
  // (a captured call may be replayed after any validation)
  HIP_TRY(launch_cow(a, r, v, true, c->cow_grid, victim_blocks, app));
  if (bucketed && win_lo) k->vb_covered = win_hi;
  if (!capturing && !bucketed) {
    c->victims_pending = false;
    // the list's pages are all taken: so are the buckets read back so far
    if (exact && !c->vb_broken) {
      k->vb_cov_gen = c->vb_gen;
      k->vb_covered = std::max(k->vb_covered, c->vb_hi);
    }
  }
  if (exact) ranges_set(k->requested, r);
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_recopy(phos_ckpt *k, hipStream_t app) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_recopy: NULL checkpoint");
  if (k->protocol != PHOS_RECOPY) return fail(PHOS_E_STATE, "recopy needs a recopy checkpoint");
  if (k->recopied) return fail(PHOS_E_STATE, "recopy already done");
  phos_ctx *c = k->ctx;
  DeviceGuard g(c->device);
  Slot &s = *k->slot;
  hipEvent_t e;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // re-quiesce: the copy stream waits for everything the application issued
  HIP_TRY(hipEventRecord(e, app));
  HIP_TRY(hipStreamWaitEvent(k->copy, e, 0));
  if (!k->bg_started) {
    TRY(start_background(c, s, k->image, true, k->copy, &k->bg, true, k->host));
    k->bg_started = true;
  }
  // the recopy follows the background copy, which left it the traced pages
  HIP_TRY(hipStreamWaitEvent(k->copy, k->bg.done, 0));
  HIP_TRY(launch_fill_u32(s.list_count, 1, 0, k->copy));
  HIP_TRY(launch_pagelist(c->d_dirty, c->d_victim, c->nwords, c->n_pages, s.list, s.list_count,
                          k->copy));
  CopyArgs a = copy_args(c, s, k->image, true, &s.counters[3]);
  HIP_TRY(launch_gather_pages(a, s.list, s.list_count, c->bg_grid, k->copy));
  // the application resumes after the recopy
  HIP_TRY(hipEventRecord(e, k->copy));
  HIP_TRY(hipStreamWaitEvent(app, e, 0));
  HIP_TRY(hipEventDestroy(e));
  k->recopied = true;
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_precopy(phos_ckpt *k, hipStream_t app) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_precopy: NULL checkpoint");
  if (k->protocol != PHOS_RECOPY) return fail(PHOS_E_STATE, "pre-copy needs a recopy checkpoint");
  if (k->recopied) return fail(PHOS_E_STATE, "recopy already done");
  phos_ctx *c = k->ctx;
  DeviceGuard g(c->device);
  Slot &s = *k->slot;
  // in the application's stream order: after the launches whose marks it
  // copies, before those validated later
  HIP_TRY(launch_fill_u32(s.list_count, 1, 0, app));
  HIP_TRY(launch_pagelist(c->d_dirty, nullptr, c->nwords, c->n_pages, s.list, s.list_count, app));
  CopyArgs a = copy_args(c, s, k->image, true, &s.counters[5]);
  HIP_TRY(launch_precopy(a, s.list, s.list_count, c->d_dirty, c->bg_grid, app));
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_precopy_final(phos_ckpt *k, const phos_spec *upcoming,
                                               uint32_t n_upcoming, uint32_t n_validated_ahead,
                                               hipStream_t app) {
  if (!k || (n_upcoming && !upcoming) || n_validated_ahead > n_upcoming)
    return fail(PHOS_E_INVAL, "phos_ckpt_precopy_final: bad argument");
  if (k->protocol != PHOS_RECOPY) return fail(PHOS_E_STATE, "pre-copy needs a recopy checkpoint");
  if (k->recopied) return fail(PHOS_E_STATE, "recopy already done");
  phos_ctx *c = k->ctx;
  if (n_validated_ahead > c->vseq) return fail(PHOS_E_INVAL, "more launches ahead than validated");
  std::vector<const HostSpec *> hs(n_upcoming);
  for (uint32_t i = 0; i < n_upcoming; ++i) {
    hs[i] = get_spec(c, upcoming[i]);
    if (!hs[i]) return fail(PHOS_E_INVAL, "upcoming launch %u: unknown spec %u", i, upcoming[i]);
  }
  DeviceGuard g(c->device);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(app, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(PHOS_E_STATE, "phos_ckpt_precopy_final cannot be captured (its mask is built now)");
  const size_t bytes = 4ull * c->nwords;
  if (!k->h_mask && hipHostMalloc(&k->h_mask, bytes, hipHostMallocDefault) != hipSuccess) {
    k->h_mask = nullptr;
    return fail(PHOS_E_NOMEM, "hipHostMalloc(%zu)", bytes);
  }
  if (!k->d_mask) TRY(dalloc(&k->d_mask, c->nwords));
  if (!k->mask_evt) HIP_TRY(hipEventCreateWithFlags(&k->mask_evt, hipEventDisableTiming));
  if (k->mask_used) HIP_TRY(hipEventSynchronize(k->mask_evt));  // the last upload has read it
  // every page any remaining launch may write (its write intervals)
  memset(k->h_mask, 0, bytes);
  for (const HostSpec *h : hs) {
    const PageRanges r = page_ranges(c, *h, PHOS_W);
    for (uint32_t i = 0; i < r.n; ++i)
      for (uint64_t p = r.p0[i], e = (uint64_t)r.p0[i] + r.np[i]; p < e;) {
        const uint32_t lo = (uint32_t)(p & 31), hi = (uint32_t)std::min<uint64_t>(32, lo + (e - p));
        k->h_mask[p >> 5] |= (hi == 32 ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        p += hi - lo;
      }
  }
  Slot &s = *k->slot;
  HIP_TRY(hipMemcpyAsync(k->d_mask, k->h_mask, bytes, hipMemcpyHostToDevice, app));
  HIP_TRY(hipEventRecord(k->mask_evt, app));
  k->mask_used = true;
  // in app_stream order: after the launches issued so far; the dirty pages
  // outside the mask have had their last valid writer issued already, and so
  // have the victim pages whose latest failing write came from a launch
  // numbered at most thr (the launches validated so far, minus those still
  // to come).  Victim pages are left alone when tracking calls went to
  // other streams: their marks are not ordered before this round.
  const bool victims_ordered =
      !c->victim_streams_many && (!c->victim_stream_set || c->victim_stream == app);
  HIP_TRY(launch_fill_u32(s.list_count, 1, 0, app));
  if (victims_ordered)
    HIP_TRY(launch_finallist(c->d_dirty, c->d_victim, c->d_victim_seq, c->vseq - n_validated_ahead,
                             k->d_mask, c->nwords, c->n_pages, s.list, s.list_count, app));
  else
    HIP_TRY(launch_pagelist(c->d_dirty, nullptr, c->nwords, c->n_pages, s.list, s.list_count, app,
                            k->d_mask));
  CopyArgs a = copy_args(c, s, k->image, true, &s.counters[5]);
  HIP_TRY(launch_precopy(a, s.list, s.list_count, c->d_dirty, c->bg_grid, app));
  return PHOS_OK;
}

// Read (after the work enqueued on s) and clear the status words of a
// checkpoint or restore: the expired-wait word, and with misspec != nullptr
// the misspeculation word.
static phos_status read_err(phos_ctx *c, hipStream_t s, bool *timeout, bool *misspec = nullptr) {
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 8, c->d_err, 4 * kErrWords, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const uint32_t *w = reinterpret_cast<const uint32_t *>(c->h_pinned + 8);
  *timeout = w[kErrWait] != 0;
  if (misspec) *misspec = w[kErrMisspec] != 0;
  if (*timeout) HIP_TRY(launch_fill_u32(c->d_err + kErrWait, 1, 0, s));
  if (misspec && *misspec) HIP_TRY(launch_fill_u32(c->d_err + kErrMisspec, 1, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PHOS_OK;
}

// Section 5: the device-to-host drain of a finished image, preemptible.  The
// copy engines serve a direction in order, so one whole-image copy would
// hold every copy the application issues in that direction until it ends
// (measured: a 64 MiB copy issued during a 16 GiB drain waited out the whole
// drain, ~0.3 s).  Chunks are issued from here with at most `window` of them
// in flight, so an application copy waits for a few chunks at most.
static phos_status drain_image(phos_ctx *c, phos_ckpt *k) {
  const uint64_t chunk = c->drain_chunk, n = c->image_bytes;
  if (!chunk || chunk >= n) {
    HIP_TRY(hipMemcpyAsync(k->host_image, k->image, n, hipMemcpyDeviceToHost, k->copy));
    return PHOS_OK;
  }
  const uint32_t window = std::max<uint32_t>(1, std::min<uint32_t>(c->drain_window, 8));
  hipEvent_t ev[8] = {};
  phos_status st = PHOS_OK;
  for (uint32_t w = 0; w < window && st == PHOS_OK; ++w)
    if (hipEventCreateWithFlags(&ev[w], hipEventDisableTiming) != hipSuccess)
      st = fail(PHOS_E_HIP, "hipEventCreate");
  uint8_t *host = static_cast<uint8_t *>(k->host_image);
  for (uint64_t off = 0, i = 0; off < n && st == PHOS_OK; off += chunk, ++i) {
    hipEvent_t &e = ev[i % window];
    hipError_t he = i >= window ? hipEventSynchronize(e) : hipSuccess;  // chunk i - window done
    if (he == hipSuccess)
      he = hipMemcpyAsync(host + off, k->image + off, std::min(chunk, n - off), hipMemcpyDeviceToHost,
                          k->copy);
    if (he == hipSuccess) he = hipEventRecord(e, k->copy);
    if (he != hipSuccess) st = fail(PHOS_E_HIP, "image drain: %s", hipGetErrorString(he));
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

// Blocking staging at the end: once every copy-on-write call has completed,
// every slot taken is published; the drain ends after the last of them.
static phos_status stage_drain_finish(phos_ckpt *k, hipStream_t app) {
  phos_ctx *c = k->ctx;
  if (!k->drainer.joinable()) return PHOS_OK;
  HIP_TRY(hipStreamSynchronize(app));
  if (k->cow_stream && k->cow_stream != app) HIP_TRY(hipStreamSynchronize(k->cow_stream));
  if (k->cow_streams_many) HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 7, k->d_stage_head, 8, hipMemcpyDeviceToHost, c->aux));
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 20, c->d_err, 4, hipMemcpyDeviceToHost, c->aux));
  HIP_TRY(hipStreamSynchronize(c->aux));
  k->drain_final.store(c->h_pinned[7], std::memory_order_release);
  // A copy whose wait for a slot gave up went straight to the image and left
  // its slot unpublished; the checkpoint has failed (PHOS_E_TIMEOUT), so the
  // drain stops at that slot instead of waiting for it.
  if (reinterpret_cast<const uint32_t *>(c->h_pinned + 20)[0] & 1u)
    k->drain_abort.store(true, std::memory_order_release);
  k->drain_stop.store(true, std::memory_order_release);
  k->drainer.join();
  if (k->drain_status != PHOS_OK)
    return fail(k->drain_status, "copy-on-write staging drain: %s", k->drain_error.c_str());
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_end(phos_ckpt *k, hipStream_t app, phos_ckpt_stats *stats) {
  if (!k) return fail(PHOS_E_INVAL, "phos_ckpt_end: NULL checkpoint");
  phos_ctx *c = k->ctx;
  DeviceGuard g(c->device);
  // ending is a quiesce point: a recopy checkpoint not yet recopied is
  // recopied now (its background copy left the traced pages to the recopy)
  if (k->protocol == PHOS_RECOPY && !k->recopied) TRY(phos_ckpt_recopy(k, app));
  Slot &s = *k->slot;
  hipEvent_t e;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(e, app));
  HIP_TRY(hipStreamWaitEvent(k->copy, e, 0));
  HIP_TRY(hipEventDestroy(e));
  if (!k->bg_started) {
    TRY(start_background(c, s, k->image, true, k->copy, &k->bg, false, k->host));
    k->bg_started = true;
  }
  HIP_TRY(hipStreamWaitEvent(k->copy, k->bg.done, 0));
  if (k->stage_block) {
    TRY(stage_drain_finish(k, app));
  } else if (k->stage) {  // staged copy-on-write pages to their places in the host image
    CopyArgs a = copy_args(c, s, k->image, true, nullptr);
    a.stage = k->stage;
    a.stage_page = k->d_stage_page;
    a.stage_head = k->d_stage_head;
    a.stage_cap = k->stage_cap;
    HIP_TRY(launch_unstage(a, c->bg_grid, k->copy));
    HIP_TRY(hipMemcpyAsync(c->h_pinned + 6, k->d_stage_head, 8, hipMemcpyDeviceToHost, k->copy));
  }
  if (k->host_image && c->image_bytes) TRY(drain_image(c, k));
  HIP_TRY(hipMemcpyAsync(c->h_pinned, s.counters, 6 * 8, hipMemcpyDeviceToHost, k->copy));
  HIP_TRY(hipStreamSynchronize(k->copy));
  HIP_TRY(hipStreamSynchronize(app));
  if (stats) {
    stats->bg_pages = c->h_pinned[1];
    stats->cow_pages = c->h_pinned[2];
    stats->recopy_pages = c->h_pinned[3];
    stats->precopy_pages = c->h_pinned[5];
    stats->staged_pages = k->stage_block ? k->drained_pages
                          : k->stage   ? std::min<uint64_t>(c->h_pinned[6], k->stage_cap)
                                       : 0;
    stats->bg_read_pages = k->pair == 1 ? c->h_pinned[4] : k->pair == 2 ? 0 : c->h_pinned[1];
    stats->bg_ms = k->bg.ms();
    stats->image_bytes = c->image_bytes;
    stats->stage_batches = k->stage_block ? k->drain_copies : 0;
  }
  bool timeout = false, misspec = false;
  TRY(read_err(c, k->copy, &timeout, k->protocol == PHOS_COW ? &misspec : nullptr));
  c->open_ckpt[k->protocol] = nullptr;
  k->bg.destroy();
  if (k->d_stage_page) (void)hipFree(k->d_stage_page);
  if (k->d_stage_head) (void)hipFree(k->d_stage_head);
  delete k;
  if (timeout) return fail(PHOS_E_TIMEOUT, "a device-side wait expired; the image is not valid");
  if (misspec)
    return fail(PHOS_E_MISSPEC, "a launch wrote outside its speculation into a page the "
                                "checkpoint had not copied; the image is not the state at the "
                                "checkpoint's start (take a stop-the-world checkpoint)");
  return PHOS_OK;
}

static phos_status states_to_host(phos_ctx *c, const uint32_t *state, uint32_t *host, uint64_t nw) {
  if (nw < c->nwords) return fail(PHOS_E_INVAL, "bitmap needs %u words", c->nwords);
  uint32_t *tmp = nullptr;
  TRY(dalloc(&tmp, c->nwords));
  hipError_t e = launch_states_to_bits(state, c->n_pages, tmp, c->aux);
  if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, c->nwords * 4ull, hipMemcpyDeviceToHost, c->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(PHOS_E_HIP, "state readback: %s", hipGetErrorString(e));
  return PHOS_OK;
}

extern "C" phos_status phos_ckpt_copied(phos_ckpt *k, uint32_t *host, uint64_t nw) {
  if (!k || !host) return fail(PHOS_E_INVAL, "phos_ckpt_copied: NULL argument");
  DeviceGuard g(k->ctx->device);
  return states_to_host(k->ctx, k->slot->state, host, nw);
}

// ------------------------------------------------------------------ restore
static CopyArgs rst_args(phos_rst *r, unsigned long long *stat, bool deep = false) {
  CopyArgs a = copy_args(r->ctx, *r->slot, const_cast<uint8_t *>(r->image), false, stat);
  a.image_chunks = r->d_chunks;
  a.chunk_pages = r->chunk_pages;
  a.want = r->want ? r->ctx->h_want : nullptr;
  a.want_cap = r->want ? kWantCap : 0;
  a.demand = r->ctx->rst_pause ? &r->slot->counters[4] : nullptr;
  a.pause_limit = std::min(r->ctx->rst_pause, r->ctx->spin_limit);
  a.hold_ticks = r->ctx->rst_hold_ms * 100000u;  // the clock runs at 100 MHz
  a.deep = deep && r->host_image ? 1u : 0u;
  return a;
}

static phos_status restore_open(phos_ctx *c, uint32_t flags, const void *image,
                                const void *const *chunks, uint32_t nchunks, uint64_t chunk_bytes,
                                hipStream_t copy, phos_rst **out);


extern "C" phos_status phos_restore_begin(phos_ctx *c, uint32_t flags, const void *image,
                                          hipStream_t copy, phos_rst **out) {
  if (!image) return fail(PHOS_E_INVAL, "phos_restore_begin: NULL image");
  if (c && !device_readable(image)) {
    // a pageable image is one piece that the DMA path moves
    const uint64_t cb = std::max<uint64_t>(c->page_bytes, (c->image_bytes + c->page_bytes - 1) /
                                                              c->page_bytes * c->page_bytes);
    const void *one[1] = {image};
    return restore_open(c, flags, image, one, 1, cb, copy, out);
  }
  return restore_open(c, flags, image, nullptr, 0, 0, copy, out);
}

extern "C" phos_status phos_restore_begin_manifest(phos_ctx *c, uint32_t flags, const void *image,
                                                   const void *manifest, uint64_t manifest_bytes,
                                                   hipStream_t copy, phos_rst **out) {
  if (out) *out = nullptr;
  TRY(phos_manifest_check(c, manifest, manifest_bytes));
  return phos_restore_begin(c, flags, image, copy, out);
}

extern "C" phos_status phos_restore_begin_chunked(phos_ctx *c, uint32_t flags,
                                                  const void *const *chunks, uint32_t nchunks,
                                                  uint64_t chunk_bytes, hipStream_t copy,
                                                  phos_rst **out) {
  if (!c || !chunks || !nchunks) return fail(PHOS_E_INVAL, "phos_restore_begin_chunked: NULL");
  if (!chunk_bytes || chunk_bytes % c->page_bytes || (chunk_bytes >> c->page_shift) > 0xFFFFFFFFull)
    return fail(PHOS_E_INVAL, "chunk_bytes must be a multiple of the page size");
  if ((uint64_t)nchunks * chunk_bytes < c->image_bytes)
    return fail(PHOS_E_INVAL, "the pieces hold less than the image");
  for (uint32_t i = 0; i < nchunks; ++i)
    if (!chunks[i] || ((uintptr_t)chunks[i] & 15))
      return fail(PHOS_E_INVAL, "piece %u NULL or not 16-byte aligned", i);
  return restore_open(c, flags, chunks[0], chunks, nchunks, chunk_bytes, copy, out);
}

// The host side of a restore from pageable pieces, on its own thread: it
// moves those pages with the copy engines in runs of up to kDmaRunBytes and,
// between runs, serves the pages waiting launches asked for (a kernel cannot
// read pageable memory, so the host is their fault handler).  Each run is
// staged in a pinned bounce slot and issued as two engine copies: the data,
// then the run's page states (a copy of kDone words that starts only when the
// data copy's completion signal reaches zero).  No compute queue or kernel
// takes part, so the DMA cannot queue behind the kernels it serves; the
// waiters poll device memory, so waiting adds no traffic on PCIe.
namespace {
struct DmaSignals {
  hsa_signal_t data{0}, state{0};
  bool used = false;
};

// Wait (bounded) for a copy-engine completion signal to reach zero.
bool wait_copy(hsa_signal_t sig, std::string *why) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hsa_signal_value_t v = hsa_signal_wait_scacquire(sig, HSA_SIGNAL_CONDITION_LT, 1,
                                                           100000000ull, HSA_WAIT_STATE_BLOCKED);
    if (v == 0) return true;
    if (v < 0) {
      *why = "the copy engine reported an error";
      return false;
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
      *why = "a copy did not complete within 60 s";
      return false;
    }
  }
}
}  // namespace

struct AgentSearch {
  uint32_t domain, bus_dev;  // the HIP device's PCI domain and (bus << 5 | device)
  hsa_agent_t gpu{0}, cpu{0};
};

static hsa_status_t match_agent(hsa_agent_t a, void *data) {
  AgentSearch *f = static_cast<AgentSearch *>(data);
  hsa_device_type_t t;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS) return HSA_STATUS_SUCCESS;
  if (t == HSA_DEVICE_TYPE_CPU && !f->cpu.handle) f->cpu = a;
  uint32_t bdf = 0, dom = 0;
  if (t == HSA_DEVICE_TYPE_GPU && !f->gpu.handle &&
      hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID, &bdf) == HSA_STATUS_SUCCESS &&
      hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_DOMAIN, &dom) == HSA_STATUS_SUCCESS &&
      dom == f->domain && (bdf >> 3) == f->bus_dev)  // BDF id: bus << 8 | device << 3 | function
    f->gpu = a;
  return HSA_STATUS_SUCCESS;
}

// The HSA agents of this context's GPU and of the host, and the pinned run
// of kDone words, for the copy-engine DMA of pageable pieces.
static phos_status dma_engines_ready(phos_ctx *c) {
  if (c->hsa_ready) return PHOS_OK;
  if (!c->hsa_inited) {
    if (hsa_init() != HSA_STATUS_SUCCESS) return fail(PHOS_E_HIP, "hsa_init failed");
    c->hsa_inited = true;
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, c->device));
  AgentSearch f;
  f.domain = (uint32_t)prop.pciDomainID;
  f.bus_dev = ((uint32_t)prop.pciBusID << 5) | (uint32_t)prop.pciDeviceID;
  if (hsa_iterate_agents(match_agent, &f) != HSA_STATUS_SUCCESS || !f.gpu.handle || !f.cpu.handle)
    return fail(PHOS_E_HIP, "no HSA agent for HIP device %d (PCI %x:%x.%x)", c->device,
                prop.pciDomainID, prop.pciBusID, prop.pciDeviceID);
  c->gpu_agent = f.gpu;
  c->cpu_agent = f.cpu;
  c->h_done = reinterpret_cast<uint32_t *>(c->h_bounce + kBounceBytes);
  for (uint64_t i = 0; i < kDmaRunBytes / 4096; ++i) c->h_done[i] = kDone;
  c->hsa_ready = true;
  return PHOS_OK;
}

// Section 4.2, blocking copy-on-write staging: the host drains the ring of
// staged pages into their places in the host image while the checkpoint runs.
// It takes slots in order as the kernels publish them (fill) and moves
// each batch of consecutive slots with one copy-engine copy into a pinned
// bounce buffer; a second copy, which starts when the first has completed,
// publishes the batch's slots as free (free_seq in device memory, where the
// waiting kernels poll).  Host threads then move the bounce's pages to their
// places in the image (staged pages are rarely consecutive in the image, and
// one engine copy per page costs far more than the page).  No compute queue
// or kernel takes part, so the drain cannot queue behind the kernels that
// wait for it.
namespace {
struct DrainShared {
  phos_ckpt *k;
  uint32_t batch_slots = 0;
  hsa_signal_t data[kDrainBounces]{}, freed[kDrainBounces]{};
  std::vector<uint32_t> pages[kDrainBounces];     // per bounce: pool page of each slot (kNone: hole)
  std::atomic<uint64_t> issued{0};                // batches handed to the copy engines
  std::atomic<uint64_t> scattered[kDrainBounces];  // per bounce: 1 + the last batch moved out of it
  std::atomic<bool> finished{false}, failed{false};
  std::string error;
  std::atomic<uint64_t> drained_pages{0};
  void fail_with(const std::string &why) {
    bool expect = false;
    if (failed.compare_exchange_strong(expect, true)) error = why;
  }
};

// Scatter worker w of nw: batches u = w, w + nw, ... (bounce u % kDrainBounces).
void drain_scatter_main(DrainShared *d, uint32_t w, uint32_t nw) {
  phos_ctx *c = d->k->ctx;
  const uint64_t pb = c->page_bytes;
  for (uint64_t u = w;; u += nw) {
    // wait until batch u is issued, or no more will be
    while (d->issued.load(std::memory_order_acquire) <= u) {
      if (d->finished.load(std::memory_order_acquire) &&
          d->issued.load(std::memory_order_acquire) <= u)
        return;
      if (d->failed.load(std::memory_order_relaxed)) return;
      std::this_thread::yield();
    }
    const uint32_t b = (uint32_t)(u % kDrainBounces);
    std::string why;
    if (!wait_copy(d->data[b], &why)) {
      d->fail_with(why);
      return;
    }
    const uint8_t *src = d->k->h_bounce + (uint64_t)b * d->batch_slots * pb;
    uint64_t n = 0;
    for (size_t i = 0; i < d->pages[b].size(); ++i) {
      const uint32_t p = d->pages[b][i];
      const uint32_t ip = p < c->n_pages ? c->h_img_page[p] : kNone;
      if (ip == kNone) continue;
      memcpy(d->k->image + (uint64_t)ip * pb, src + i * pb, pb);
      ++n;
    }
    d->drained_pages.fetch_add(n, std::memory_order_relaxed);
    d->scattered[b].store(u + 1, std::memory_order_release);
  }
}
}  // namespace

static void stage_drain_main(phos_ckpt *k) {
  phos_ctx *c = k->ctx;
  const uint32_t cap = k->stage_cap;
  const uint64_t *fill = k->h_fill;
  const uint64_t pb = c->page_bytes;
  DrainShared d;
  d.k = k;
  d.batch_slots = k->drain_batch_slots;
  for (uint32_t b = 0; b < kDrainBounces; ++b) {
    d.scattered[b].store(0);
    d.pages[b].reserve(d.batch_slots);
    if (hsa_signal_create(0, 0, nullptr, &d.data[b]) != HSA_STATUS_SUCCESS ||
        hsa_signal_create(0, 0, nullptr, &d.freed[b]) != HSA_STATUS_SUCCESS)
      d.fail_with("hsa_signal_create failed");
  }
  std::vector<std::thread> workers;
  const uint32_t nw = k->drain_threads;
  if (!d.failed.load())
    for (uint32_t w = 0; w < nw; ++w) workers.emplace_back(drain_scatter_main, &d, w, nw);
  uint64_t next = 0, u = 0;  // the next slot to drain, the next batch
  bool stopping = false;
  std::chrono::steady_clock::time_point t_stop{};
  // The ring is drained once it is about half full (the slot half a ring
  // ahead of the oldest one is published), and everything at the end: while
  // the area holds every page the launches copy, the link stays free for the
  // background copy, whose claimed pages the launches may be waiting for.
  const uint64_t high = std::max<uint64_t>(1, (uint64_t)cap * k->drain_high_pct / 100);
  while (!d.failed.load(std::memory_order_relaxed)) {
    const uint32_t pos0 = (uint32_t)(next % cap);
    const uint32_t lim = std::min<uint32_t>(d.batch_slots, cap - pos0);
    uint32_t n = 0;
    const bool stop = k->drain_stop.load(std::memory_order_acquire);
    if (stop || (uint32_t)(__atomic_load_n(&fill[(next + high - 1) % cap], __ATOMIC_ACQUIRE) >> 32) ==
                    (uint32_t)(next + high))
      while (n < lim && (uint32_t)(__atomic_load_n(&fill[pos0 + n], __ATOMIC_ACQUIRE) >> 32) ==
                            (uint32_t)(next + n + 1))
        ++n;
    if (!n) {
      if (k->drain_abort.load(std::memory_order_acquire)) break;
      if (stop) {
        if (next >= k->drain_final.load(std::memory_order_acquire)) break;
        // every kernel has ended, so every slot taken is published already
        if (!stopping) {
          stopping = true;
          t_stop = std::chrono::steady_clock::now();
        } else if (std::chrono::steady_clock::now() - t_stop > std::chrono::seconds(10)) {
          d.fail_with("a staging slot was taken but never published");
          break;
        }
      }
      __builtin_ia32_pause();
      continue;
    }
    const uint32_t b = (uint32_t)(u % kDrainBounces);
    // the bounce's previous batch has been moved out, and its free copy is done
    const auto t0 = std::chrono::steady_clock::now();
    while (u >= kDrainBounces && d.scattered[b].load(std::memory_order_acquire) < u - kDrainBounces + 1) {
      if (d.failed.load(std::memory_order_relaxed)) break;
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
        d.fail_with("moving a staged batch into the image took over 60 s");
        break;
      }
      std::this_thread::yield();
    }
    std::string why;
    if (d.failed.load() || (u >= kDrainBounces && !wait_copy(d.freed[b], &why))) {
      if (!why.empty()) d.fail_with(why);
      break;
    }
    d.pages[b].resize(n);
    for (uint32_t i = 0; i < n; ++i) d.pages[b][i] = (uint32_t)fill[pos0 + i];
    hsa_signal_store_relaxed(d.data[b], 1);
    uint8_t *dst = k->h_bounce + (uint64_t)b * d.batch_slots * pb;
    const uint8_t *src = k->stage + (uint64_t)pos0 * pb;
    if (hsa_amd_memory_async_copy(dst, c->cpu_agent, src, c->gpu_agent, n * pb, 0, nullptr,
                                  d.data[b]) != HSA_STATUS_SUCCESS) {
      hsa_signal_store_relaxed(d.data[b], 0);
      d.fail_with("hsa_amd_memory_async_copy failed");
      break;
    }
    for (uint32_t i = 0; i < n; ++i) k->h_free_src[pos0 + i] = (uint32_t)(next + i + 1);
    hsa_signal_store_relaxed(d.freed[b], 1);
    if (hsa_amd_memory_async_copy(k->d_free_seq + pos0, c->gpu_agent, k->h_free_src + pos0,
                                  c->cpu_agent, 4ull * n, 1, &d.data[b],
                                  d.freed[b]) != HSA_STATUS_SUCCESS) {
      hsa_signal_store_relaxed(d.freed[b], 0);
      d.issued.store(u + 1, std::memory_order_release);  // the data copy still gets moved
      d.fail_with("hsa_amd_memory_async_copy failed");
      break;
    }
    ++k->drain_copies;
    d.issued.store(++u, std::memory_order_release);
    next += n;
  }
  d.finished.store(true, std::memory_order_release);
  for (std::thread &t : workers) t.join();
  for (uint32_t b = 0; b < kDrainBounces; ++b) {
    std::string why;
    if (u > b && !wait_copy(d.freed[b], &why)) d.fail_with(why);
  }
  for (uint32_t b = 0; b < kDrainBounces; ++b) {
    if (d.data[b].handle) (void)hsa_signal_destroy(d.data[b]);
    if (d.freed[b].handle) (void)hsa_signal_destroy(d.freed[b]);
  }
  k->drained_pages = d.drained_pages.load();
  if (d.failed.load()) {
    k->drain_status = PHOS_E_HIP;
    k->drain_error = d.error;
  }
}

static void restore_dma_main(phos_rst *r, std::vector<const uint8_t *> src, std::vector<uint8_t> pg,
                             uint64_t chunk_bytes) {
  phos_ctx *c = r->ctx;
  Slot &s = *r->slot;
  std::string why;
  auto failed = [r](const std::string &what) {
    r->dma_status = PHOS_E_HIP;
    r->dma_error = what;
  };
  auto since_begin = [r]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r->t_begin)
        .count();
  };
  const uint64_t pb = c->page_bytes, img_pages = c->image_bytes >> c->page_shift;
  const uint64_t cp = chunk_bytes >> c->page_shift;
  const uint64_t run_pages = std::max<uint64_t>(1, kDmaRunBytes / pb);
  std::vector<uint8_t> served(img_pages, 0);
  uint32_t scanned = 0;
  const uint32_t *want = c->h_want;  // pinned: kernels append with system-scope atomics
  DmaSignals sig[2];
  for (DmaSignals &d : sig)
    if (hsa_signal_create(0, 0, nullptr, &d.data) != HSA_STATUS_SUCCESS ||
        hsa_signal_create(0, 0, nullptr, &d.state) != HSA_STATUS_SUCCESS)
      return failed("hsa_signal_create failed");
  uint32_t slot = 0;
  hsa_signal_t first_data{0}, first_state{0};  // the first run's, for the timings
  auto note_first = [&]() {
    if (r->dma_first_copy_ms < 0 && first_data.handle && hsa_signal_load_scacquire(first_data) == 0)
      r->dma_first_copy_ms = since_begin();
    if (r->dma_first_ms < 0 && first_state.handle && hsa_signal_load_scacquire(first_state) == 0)
      r->dma_first_ms = since_begin();
  };
  // image pages [i0, i1): one piece, pool-contiguous
  auto copy_run = [&](uint64_t i0, uint64_t i1) -> bool {
    const uint64_t k = i0 / cp, n = i1 - i0, bytes = n * pb;
    if (bytes > kDmaRunBytes) {  // runs are cut at run_pages
      why = "DMA run too long";
      return false;
    }
    DmaSignals &d = sig[slot];
    note_first();
    if (d.used && !(wait_copy(d.data, &why) && wait_copy(d.state, &why))) return false;
    note_first();
    uint8_t *stage = c->h_bounce + slot * kDmaRunBytes;
    memcpy(stage, src[k] + (i0 - k * cp) * pb, bytes);
    const uint32_t p0 = c->h_img_pool[i0];
    hsa_signal_store_relaxed(d.data, 1);
    hsa_signal_store_relaxed(d.state, 1);
    if (hsa_amd_memory_async_copy(reinterpret_cast<void *>(c->pool_base + ((uint64_t)p0 << c->page_shift)),
                                  c->gpu_agent, stage, c->cpu_agent, bytes, 0, nullptr,
                                  d.data) != HSA_STATUS_SUCCESS ||
        hsa_amd_memory_async_copy(s.state + p0, c->gpu_agent, c->h_done, c->cpu_agent, 4 * n, 1,
                                  &d.data, d.state) != HSA_STATUS_SUCCESS) {
      why = "hsa_amd_memory_async_copy failed";
      return false;
    }
    if (!first_data.handle) {
      first_data = d.data;
      first_state = d.state;
      r->dma_first_issue_ms = since_begin();
    }
    d.used = true;
    slot ^= 1u;
    r->dma_pages += n;
    return true;
  };
  // the pages waiting launches asked for, each copied alone
  auto serve = [&]() -> bool {
    const uint32_t n = std::min<uint32_t>(__atomic_load_n(&want[0], __ATOMIC_ACQUIRE), kWantCap);
    for (; scanned < n; ++scanned) {
      const uint32_t p = __atomic_load_n(&want[1 + scanned], __ATOMIC_ACQUIRE);
      if (p == kNone) break;  // reserved, not written yet: next round
      if (p >= c->n_pages) continue;
      const uint32_t ip = c->h_img_page[p];
      if (ip == kNone || !pg[ip / cp] || served[ip]) continue;
      served[ip] = 1;
      ++r->asked_pages;
      if (!copy_run(ip, ip + 1)) return false;
    }
    return true;
  };
  bool ok = serve();
  uint64_t run = 0;
  for (uint64_t ip = 0; ok && ip <= img_pages; ++ip) {
    // a run breaks at the end, a served page, a piece boundary, a pool
    // discontinuity (buffer boundary) or run_pages
    bool take = ip < img_pages && pg[ip / cp] && !served[ip];
    const bool joins = take && ip > run && ip - run < run_pages && ip / cp == run / cp &&
                       c->h_img_pool[ip] == c->h_img_pool[ip - 1] + 1;
    if (ip > run && !joins) {
      for (uint64_t q = run; q < ip; ++q) served[q] = 1;
      ok = copy_run(run, ip) && serve();  // between runs, what launches wait for
      run = ip;
      take = take && !served[ip];  // it may have been one of them
    }
    if (!take) run = ip + 1;
  }
  for (DmaSignals &d : sig)
    if (ok && d.used) ok = wait_copy(d.data, &why) && wait_copy(d.state, &why);
  note_first();
  for (DmaSignals &d : sig) {
    if (d.data.handle) (void)hsa_signal_destroy(d.data);
    if (d.state.handle) (void)hsa_signal_destroy(d.state);
  }
  if (!ok) return failed(why);
  r->dma_ms = since_begin();
}

static phos_status restore_open(phos_ctx *c, uint32_t flags, const void *image,
                                const void *const *chunks, uint32_t nchunks, uint64_t chunk_bytes,
                                hipStream_t copy, phos_rst **out) {
  if (!c || !image || !out) return fail(PHOS_E_INVAL, "phos_restore_begin: NULL argument");
  *out = nullptr;
  if (flags & ~(PHOS_RST_DEFER_BACKGROUND | PHOS_RST_PREFETCH_SPEC))
    return fail(PHOS_E_INVAL, "unknown flags 0x%x", flags);
  if (((uintptr_t)image) & 15) return fail(PHOS_E_INVAL, "image must be 16-byte aligned");
  if (c->open_rst) return fail(PHOS_E_STATE, "a restore is already open");
  if (c->open_ckpt[1] || c->open_ckpt[2]) return fail(PHOS_E_STATE, "a checkpoint is open");
  DeviceGuard g(c->device);
  Slot &s = c->slots[0];
  TRY(ensure_slot(c, s, false));
  HIP_TRY(launch_fill_u32(s.state, c->n_pages, kFree, c->aux));
  HIP_TRY(launch_fill_u64(s.counters, kSlotCounters, 0, c->aux));
  HIP_TRY(hipStreamSynchronize(c->aux));
  phos_rst *r = new phos_rst;
  r->ctx = c;
  r->flags = flags;
  r->image = (const uint8_t *)image;
  r->copy = copy;
  r->slot = &s;
  if (!chunks) (void)device_readable(image, &r->host_image);
  bool any_pageable = false;
  std::function<void()> start_dma;
  if (chunks) {
    std::vector<unsigned long long> tab(nchunks);
    std::vector<uint8_t> pageable(nchunks, 0);
    for (uint32_t i = 0; i < nchunks; ++i) {
      bool in_host = false;
      pageable[i] = device_readable(chunks[i], &in_host) ? 0 : 1;
      r->host_image |= in_host;
      any_pageable |= pageable[i] != 0;
      // a pageable piece's address never reaches a kernel
      tab[i] = pageable[i] ? 0 : reinterpret_cast<uintptr_t>(chunks[i]);
    }
    r->chunk_pages = (uint32_t)(chunk_bytes >> c->page_shift);
    hipError_t e = hipMalloc((void **)&r->d_chunks, 8ull * nchunks);
    if (e == hipSuccess) e = hipMemcpy(r->d_chunks, tab.data(), 8ull * nchunks, hipMemcpyHostToDevice);
    if (e == hipSuccess && any_pageable) {
      const phos_status st = dma_engines_ready(c);
      if (st != PHOS_OK) {
        if (r->d_chunks) (void)hipFree(r->d_chunks);
        delete r;
        return st;
      }
      e = hipMalloc((void **)&r->d_pageable, nchunks);
      if (e == hipSuccess) e = hipMemcpy(r->d_pageable, pageable.data(), nchunks, hipMemcpyHostToDevice);
      r->want = true;
      c->h_want[0] = 0;  // no kernel of this context runs now (begin is a quiesce point)
      for (uint32_t i = 1; i <= kWantCap; ++i) c->h_want[i] = kNone;
      // hold the pageable pieces' pages for the host before any kernel can
      // claim them
      if (e == hipSuccess)
        e = launch_mark_pieces(c->d_img_page, s.state, c->n_pages, r->chunk_pages, r->d_pageable,
                               kHost, nullptr, c->aux);
      if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
    }
    if (e != hipSuccess) {
      if (r->d_chunks) (void)hipFree(r->d_chunks);
      if (r->d_pageable) (void)hipFree(r->d_pageable);
      delete r;
      return fail(PHOS_E_NOMEM, "restore piece table: %s", hipGetErrorString(e));
    }
    if (any_pageable) {
      // the DMA of the pageable pieces runs from its own host thread (a copy
      // from pageable memory can block the thread that issues it), started
      // once the background copy is enqueued
      std::vector<const uint8_t *> src(reinterpret_cast<const uint8_t *const *>(chunks),
                                       reinterpret_cast<const uint8_t *const *>(chunks) + nchunks);
      std::vector<uint8_t> pg(pageable);
      start_dma = [r, src, pg, chunk_bytes]() { restore_dma_main(r, src, pg, chunk_bytes); };
    }
  }
  if (!(flags & PHOS_RST_DEFER_BACKGROUND)) {
    phos_status st = start_background_args(c, s, rst_args(r, &s.counters[1], c->rst_deep_bg), copy,
                                           &r->bg, r->host_image);
    if (st != PHOS_OK) {
      delete r;
      return st;
    }
    r->bg_started = true;
  }
  r->t_begin = std::chrono::steady_clock::now();
  if (start_dma) r->dma_thread = std::thread(start_dma);
  c->open_rst = r;
  *out = r;
  return PHOS_OK;
}

extern "C" phos_status phos_restore_on_demand(phos_rst *r, phos_spec spec, const uint64_t *d_records,
                                              uint64_t n, hipStream_t app, uint64_t *d_faulted) {
  if (!r || (n && !d_records)) return fail(PHOS_E_INVAL, "phos_restore_on_demand: bad argument");
  if (((uintptr_t)d_records) & 7) return fail(PHOS_E_INVAL, "records must be 8-byte aligned");
  phos_ctx *c = r->ctx;
  HostSpec *h = get_spec(c, spec);
  if (!h) return fail(PHOS_E_INVAL, "phos_restore_on_demand: unknown spec %u", spec);
  DeviceGuard g(c->device);
  Slot &s = *r->slot;
  if (r->flags & PHOS_RST_PREFETCH_SPEC) {
    const PageRanges pr = page_ranges(c, *h, PHOS_R | PHOS_W);
    const VictimList none{nullptr, nullptr, 0, nullptr, 0, 0};
    HIP_TRY(launch_cow(rst_args(r, &s.counters[2]), pr, none, true, c->cow_grid, 0, app));
  }
  CopyArgs a = rst_args(r, &s.counters[2], c->rst_deep_demand);
  HIP_TRY(launch_demand(a, d_records, n, c->pool_base, (unsigned long long *)d_faulted, c->n_cu, app));
  return PHOS_OK;
}

extern "C" phos_status phos_restore_present(phos_rst *r, uint32_t *host, uint64_t nw) {
  if (!r || !host) return fail(PHOS_E_INVAL, "phos_restore_present: NULL argument");
  DeviceGuard g(r->ctx->device);
  return states_to_host(r->ctx, r->slot->state, host, nw);
}

extern "C" phos_status phos_restore_end(phos_rst *r, hipStream_t app, phos_rst_stats *stats) {
  if (!r) return fail(PHOS_E_INVAL, "phos_restore_end: NULL restore");
  phos_ctx *c = r->ctx;
  DeviceGuard g(c->device);
  Slot &s = *r->slot;
  hipEvent_t e;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(e, app));
  HIP_TRY(hipStreamWaitEvent(r->copy, e, 0));
  HIP_TRY(hipEventDestroy(e));
  if (!r->bg_started) {
    TRY(start_background_args(c, s, rst_args(r, &s.counters[1], c->rst_deep_bg), r->copy,
                              &r->bg, r->host_image));
    r->bg_started = true;
  }
  HIP_TRY(hipStreamWaitEvent(r->copy, r->bg.done, 0));
  if (r->dma_thread.joinable()) r->dma_thread.join();
  HIP_TRY(hipMemcpyAsync(c->h_pinned, s.counters, 4 * 8, hipMemcpyDeviceToHost, r->copy));
  HIP_TRY(hipStreamSynchronize(r->copy));
  HIP_TRY(hipStreamSynchronize(app));
  if (stats) {
    stats->bg_pages = c->h_pinned[1];
    stats->demand_pages = c->h_pinned[2];
    stats->dma_pages = r->dma_pages;
    stats->asked_pages = r->asked_pages;
    stats->dma_ms = r->dma_ms;
    stats->dma_first_ms = r->dma_first_ms;
    stats->dma_first_issue_ms = r->dma_first_issue_ms;
    stats->dma_first_copy_ms = r->dma_first_copy_ms;
    stats->bg_ms = r->bg.ms();
  }
  bool timeout = false;
  TRY(read_err(c, r->copy, &timeout));
  c->open_rst = nullptr;
  if (r->d_chunks) (void)hipFree(r->d_chunks);
  if (r->d_pageable) (void)hipFree(r->d_pageable);
  const phos_status dma_status = r->dma_status;
  const std::string dma_error = r->dma_error;
  delete r;
  if (dma_status != PHOS_OK) return fail(dma_status, "restore DMA: %s", dma_error.c_str());
  if (timeout) return fail(PHOS_E_TIMEOUT, "a device-side wait expired; the pool is not valid");
  return PHOS_OK;
}
