// batch.cpp — batched copy of many requests' segments in one persistent,
// graph-captured launch, the plain per-request launch it is compared with,
// and the autotuner that picks the chunk size and grid shape.  No paper
// analog: the paper copies each buffer separately in 4 MB chunks (Section 5);
// here a device-resident work queue feeds one replayable HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "phos.h"
#include "util.h"

using namespace phos;

#define HIP_TRY(x)                                                                  \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return fail(PHOS_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
#define TRY(x)                    \
  do {                            \
    phos_status s_ = (x);         \
    if (s_ != PHOS_OK) return s_; \
  } while (0)

namespace {
// Device queue layout: [hdr 4 x u64][prefix (max_segs + 1) x u64][segs max_segs x 32 B]
size_t queue_bytes(uint64_t max_segs) { return 8 * (4 + max_segs + 1) + 32 * max_segs; }
size_t stage_bytes(uint64_t max_segs, uint32_t max_reqs) {
  return queue_bytes(max_segs) + 8ull * max_reqs;
}

uint32_t cu_count(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) == hipSuccess && p.multiProcessorCount > 0)
    return (uint32_t)p.multiProcessorCount;
  return 256;
}

bool cfg_ok(const phos_batch_cfg &c) {
  return c.chunk_bytes >= 4096 && c.chunk_bytes % 16 == 0 && c.wg_per_cu >= 1 &&
         c.wg_per_cu <= 16 && (c.threads == 256 || c.threads == 512 || c.threads == 1024);
}

phos_status check_segs(const phos_copy_seg *segs, uint64_t nseg, uint32_t max_reqs,
                       uint64_t *total, uint64_t *nreq) {
  uint64_t t = 0, r = 0;
  for (uint64_t i = 0; i < nseg; ++i) {
    const phos_copy_seg &g = segs[i];
    if ((g.src | g.dst | g.bytes) & 15)
      return fail(PHOS_E_INVAL, "segment %llu: addresses and size must be 16-byte multiples",
                  (unsigned long long)i);
    if (g.bytes && (!g.src || !g.dst))
      return fail(PHOS_E_INVAL, "segment %llu: NULL address", (unsigned long long)i);
    if (g.req >= max_reqs)
      return fail(PHOS_E_INVAL, "segment %llu: request %u >= %u", (unsigned long long)i, g.req,
                  max_reqs);
    t += g.bytes;
    r = std::max<uint64_t>(r, (uint64_t)g.req + 1);
  }
  *total = t;
  *nreq = r;
  return PHOS_OK;
}

// Host image of [hdr][prefix] for nseg segments.
void fill_header(const phos_copy_seg *segs, uint64_t nseg, uint64_t total, uint64_t nreq,
                 unsigned long long *dst) {
  dst[0] = nseg;
  dst[1] = total;
  dst[2] = nreq;
  dst[3] = 0;
  unsigned long long *pre = dst + 4;
  unsigned long long acc = 0;
  for (uint64_t i = 0; i < nseg; ++i) {
    pre[i] = acc;
    acc += segs[i].bytes;
  }
  pre[nseg] = acc;
}
}  // namespace

struct phos_batch {
  int device = 0;
  uint64_t max_segs = 0;
  uint32_t max_reqs = 0;
  uint32_t n_cu = 256;
  uint32_t loaded_reqs = 0;
  uint64_t loaded_total = 0;
  phos_batch_cfg cfg{};
  uint8_t *d_queue = nullptr;
  unsigned long long *d_cursor = nullptr, *d_done = nullptr;
  unsigned long long *d_req_total = nullptr, *d_req_time = nullptr;  // time: [0] start, [1 + r]
  double clock_khz = 100000.0;  // GPU wall clock
  uint8_t *h_stage = nullptr;
  hipEvent_t stage_evt = nullptr;
  bool stage_used = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  BatchQ q() const {
    BatchQ b;
    b.hdr = reinterpret_cast<const unsigned long long *>(d_queue);
    b.byte_prefix = b.hdr + 4;
    b.segs = reinterpret_cast<const phos_copy_seg *>(d_queue + 8 * (4 + max_segs + 1));
    b.cursor = d_cursor;
    b.done = d_done;
    b.req_total = d_req_total;
    b.req_time = d_req_time + 1;
    b.chunk_bytes = cfg.chunk_bytes;
    return b;
  }
};

struct phos_seglist {
  int device = 0;
  uint64_t nseg = 0, total = 0;
  uint8_t *d_queue = nullptr;  // same layout as the batch queue
  unsigned long long *d_done = nullptr, *d_cursor = nullptr;
};

static void drop_graph(phos_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static phos_status capture(phos_batch *b) {
  drop_graph(b);
  const BatchQ q = b->q();
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_batch_reset(q, b->cap);
  if (e == hipSuccess) e = launch_batch_copy(q, b->cfg.wg_per_cu * b->n_cu, b->cfg.threads, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(PHOS_E_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return PHOS_OK;
}

static phos_batch_cfg default_cfg() {
  phos_batch_cfg c;
  c.chunk_bytes = (uint64_t)env_u32("PHOS_BATCH_CHUNK", 1u << 20);
  c.wg_per_cu = env_u32("PHOS_BATCH_WG_PER_CU", 2);
  c.threads = env_u32("PHOS_BATCH_THREADS", 512);
  return c;
}

extern "C" phos_status phos_batch_destroy(phos_batch *b) {
  if (!b) return fail(PHOS_E_INVAL, "phos_batch_destroy: NULL");
  DeviceGuard g(b->device);
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_cursor) (void)hipFree(b->d_cursor);
  if (b->d_done) (void)hipFree(b->d_done);
  if (b->d_req_total) (void)hipFree(b->d_req_total);
  if (b->d_req_time) (void)hipHostFree(b->d_req_time);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->stage_evt) (void)hipEventDestroy(b->stage_evt);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return PHOS_OK;
}

extern "C" phos_status phos_batch_create(int device, uint64_t max_segs, uint32_t max_reqs,
                                         const phos_batch_cfg *cfg, phos_batch **out) {
  if (!out || !max_segs || !max_reqs) return fail(PHOS_E_INVAL, "phos_batch_create: bad argument");
  *out = nullptr;
  phos_batch_cfg c = cfg ? *cfg : default_cfg();
  if (!cfg_ok(c)) return fail(PHOS_E_INVAL, "bad batch configuration");
  DeviceGuard g(device);
  phos_batch *b = new phos_batch;
  b->device = device;
  b->max_segs = max_segs;
  b->max_reqs = max_reqs;
  b->n_cu = cu_count(device);
  b->cfg = c;
  const size_t qb = queue_bytes(max_segs);
  hipError_t e = hipMalloc((void **)&b->d_queue, qb);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_cursor, 8);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_done, 8ull * max_reqs);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_req_total, 8ull * max_reqs);
  // completion stamps live in pinned host memory: the host reads them in place
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&b->d_req_time, 8ull * (max_reqs + 1), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(b->d_req_total, 0xFF, 8ull * max_reqs);
  int khz = 0;
  if (e == hipSuccess && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) ==
                             hipSuccess && khz > 0)
    b->clock_khz = khz;
  if (e == hipSuccess) e = hipMemset(b->d_queue, 0, 8 * 4);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&b->h_stage, stage_bytes(max_segs, max_reqs), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_evt, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    phos_batch_destroy(b);
    return fail(PHOS_E_NOMEM, "phos_batch_create: %s", hipGetErrorString(e));
  }
  phos_status st = capture(b);
  if (st != PHOS_OK) {
    phos_batch_destroy(b);
    return st;
  }
  *out = b;
  return PHOS_OK;
}

extern "C" phos_status phos_batch_load(phos_batch *b, const phos_copy_seg *segs, uint64_t nseg,
                                       hipStream_t stream) {
  if (!b || (!segs && nseg)) return fail(PHOS_E_INVAL, "phos_batch_load: NULL argument");
  if (nseg > b->max_segs) return fail(PHOS_E_INVAL, "%llu segments > capacity %llu",
                                      (unsigned long long)nseg, (unsigned long long)b->max_segs);
  uint64_t total = 0, nreq = 0;
  TRY(check_segs(segs, nseg, b->max_reqs, &total, &nreq));
  DeviceGuard g(b->device);
  if (b->stage_used) HIP_TRY(hipEventSynchronize(b->stage_evt));
  unsigned long long *hp = reinterpret_cast<unsigned long long *>(b->h_stage);
  fill_header(segs, nseg, total, nreq, hp);
  const size_t seg_off = 8 * (4 + b->max_segs + 1);
  memcpy(b->h_stage + seg_off, segs, nseg * sizeof(phos_copy_seg));
  HIP_TRY(hipMemcpyAsync(b->d_queue, b->h_stage, 8 * (4 + nseg + 1), hipMemcpyHostToDevice, stream));
  if (nseg)
    HIP_TRY(hipMemcpyAsync(b->d_queue + seg_off, b->h_stage + seg_off, nseg * sizeof(phos_copy_seg),
                           hipMemcpyHostToDevice, stream));
  // per-request totals (for the completion stamps)
  unsigned long long *tot = reinterpret_cast<unsigned long long *>(b->h_stage + queue_bytes(b->max_segs));
  for (uint64_t r = 0; r < nreq; ++r) tot[r] = 0;
  for (uint64_t i = 0; i < nseg; ++i) tot[segs[i].req] += segs[i].bytes;
  if (nreq)
    HIP_TRY(hipMemcpyAsync(b->d_req_total, tot, 8 * nreq, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(b->stage_evt, stream));
  b->stage_used = true;
  b->loaded_reqs = (uint32_t)nreq;
  b->loaded_total = total;
  return PHOS_OK;
}

namespace phos {
phos_batch_cfg batch_default_cfg() { return default_cfg(); }
bool batch_cfg_ok(const phos_batch_cfg &c) { return cfg_ok(c); }
const volatile unsigned long long *batch_stamps(const phos_batch *b) { return b->d_req_time; }
double batch_clock_khz(const phos_batch *b) { return b->clock_khz; }
}  // namespace phos

extern "C" phos_status phos_batch_run_plain(phos_batch *b, hipStream_t stream) {
  if (!b) return fail(PHOS_E_INVAL, "phos_batch_run_plain: NULL");
  DeviceGuard g(b->device);
  const uint64_t nchunks = (b->loaded_total + b->cfg.chunk_bytes - 1) / b->cfg.chunk_bytes;
  if (nchunks > 0x7FFFFFFFull) return fail(PHOS_E_INVAL, "too many chunks");
  BatchQ q = b->q();
  HIP_TRY(launch_batch_reset(q, stream));
  HIP_TRY(launch_plain_copy(q, nchunks, b->cfg.threads, stream));
  return PHOS_OK;
}

extern "C" phos_status phos_batch_times(phos_batch *b, double *ms, uint32_t n) {
  if (!b || (!ms && n)) return fail(PHOS_E_INVAL, "phos_batch_times: NULL");
  if (n > b->loaded_reqs) return fail(PHOS_E_INVAL, "only %u requests loaded", b->loaded_reqs);
  DeviceGuard g(b->device);
  std::vector<unsigned long long> t(n + 1);
  HIP_TRY(hipDeviceSynchronize());
  for (uint32_t i = 0; i <= n; ++i) t[i] = b->d_req_time[i];  // pinned host memory
  for (uint32_t r = 0; r < n; ++r)
    ms[r] = t[r + 1] ? (double)(t[r + 1] - t[0]) / b->clock_khz : -1.0;
  return PHOS_OK;
}

extern "C" phos_status phos_batch_run(phos_batch *b, hipStream_t stream) {
  if (!b) return fail(PHOS_E_INVAL, "phos_batch_run: NULL");
  DeviceGuard g(b->device);
  HIP_TRY(hipGraphLaunch(b->exec, stream));
  return PHOS_OK;
}

extern "C" phos_status phos_batch_copy(phos_batch *b, const phos_copy_seg *segs, uint64_t nseg,
                                       hipStream_t stream) {
  TRY(phos_batch_load(b, segs, nseg, stream));
  return phos_batch_run(b, stream);
}

extern "C" phos_status phos_batch_done_bytes(phos_batch *b, uint64_t **d_done) {
  if (!b || !d_done) return fail(PHOS_E_INVAL, "phos_batch_done_bytes: NULL");
  *d_done = reinterpret_cast<uint64_t *>(b->d_done);
  return PHOS_OK;
}

extern "C" phos_status phos_batch_get_cfg(phos_batch *b, phos_batch_cfg *cfg) {
  if (!b || !cfg) return fail(PHOS_E_INVAL, "phos_batch_get_cfg: NULL");
  *cfg = b->cfg;
  return PHOS_OK;
}

extern "C" phos_status phos_batch_set_cfg(phos_batch *b, const phos_batch_cfg *cfg) {
  if (!b || !cfg || !cfg_ok(*cfg)) return fail(PHOS_E_INVAL, "phos_batch_set_cfg: bad argument");
  DeviceGuard g(b->device);
  HIP_TRY(hipDeviceSynchronize());
  b->cfg = *cfg;
  return capture(b);
}

// ------------------------------------------------------------- plain path
extern "C" phos_status phos_seglist_create(int device, const phos_copy_seg *segs, uint64_t nseg,
                                           phos_seglist **out) {
  if (!out || (!segs && nseg)) return fail(PHOS_E_INVAL, "phos_seglist_create: NULL argument");
  *out = nullptr;
  uint64_t total = 0, nreq = 0;
  TRY(check_segs(segs, nseg, 0xFFFFFFFFu, &total, &nreq));
  DeviceGuard g(device);
  phos_seglist *l = new phos_seglist;
  l->device = device;
  l->nseg = nseg;
  l->total = total;
  const size_t qb = queue_bytes(nseg);
  std::vector<unsigned long long> host(qb / 8 + 1);
  fill_header(segs, nseg, total, nreq, host.data());
  memcpy(reinterpret_cast<uint8_t *>(host.data()) + 8 * (4 + nseg + 1), segs,
         nseg * sizeof(phos_copy_seg));
  hipError_t e = hipMalloc((void **)&l->d_queue, qb);
  if (e == hipSuccess) e = hipMalloc((void **)&l->d_done, 8 * std::max<uint64_t>(nreq, 1));
  if (e == hipSuccess) e = hipMalloc((void **)&l->d_cursor, 8);
  if (e == hipSuccess) e = hipMemcpy(l->d_queue, host.data(), qb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(l->d_done, 0, 8 * std::max<uint64_t>(nreq, 1));
  if (e != hipSuccess) {
    if (l->d_queue) (void)hipFree(l->d_queue);
    if (l->d_done) (void)hipFree(l->d_done);
    if (l->d_cursor) (void)hipFree(l->d_cursor);
    delete l;
    return fail(PHOS_E_NOMEM, "phos_seglist_create: %s", hipGetErrorString(e));
  }
  *out = l;
  return PHOS_OK;
}

extern "C" phos_status phos_seglist_destroy(phos_seglist *l) {
  if (!l) return fail(PHOS_E_INVAL, "phos_seglist_destroy: NULL");
  DeviceGuard g(l->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(l->d_queue);
  (void)hipFree(l->d_done);
  (void)hipFree(l->d_cursor);
  delete l;
  return PHOS_OK;
}

extern "C" phos_status phos_copy_plain(const phos_seglist *l, uint64_t chunk_bytes,
                                       uint32_t threads, hipStream_t stream) {
  if (!l || chunk_bytes < 4096 || chunk_bytes % 16 ||
      (threads != 256 && threads != 512 && threads != 1024))
    return fail(PHOS_E_INVAL, "phos_copy_plain: bad argument");
  DeviceGuard g(l->device);
  BatchQ q;
  q.hdr = reinterpret_cast<const unsigned long long *>(l->d_queue);
  q.byte_prefix = q.hdr + 4;
  q.segs = reinterpret_cast<const phos_copy_seg *>(l->d_queue + 8 * (4 + l->nseg + 1));
  q.cursor = l->d_cursor;
  q.done = l->d_done;
  q.req_total = nullptr;
  q.req_time = nullptr;
  q.chunk_bytes = chunk_bytes;
  const uint64_t nchunks = (l->total + chunk_bytes - 1) / chunk_bytes;
  if (nchunks > 0x7FFFFFFFull) return fail(PHOS_E_INVAL, "too many chunks");
  HIP_TRY(launch_plain_copy(q, nchunks, threads, stream));
  return PHOS_OK;
}

// --------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::pair<phos_batch_cfg, double>> g_tune_cache;

std::string shape_key(const phos_copy_seg *segs, uint64_t nseg) {
  uint64_t total = 0;
  for (uint64_t i = 0; i < nseg; ++i) total += segs[i].bytes;
  auto lg = [](uint64_t v) { return v ? 63 - __builtin_clzll(v) : 0; };
  char buf[96];
  snprintf(buf, sizeof buf, "t%d_n%d_m%d", lg(total), lg(nseg), lg(nseg ? total / nseg : 0));
  return buf;
}

void load_cache(const char *path) {
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char key[96];
  unsigned long long chunk;
  unsigned wg, th;
  double ms;
  while (fscanf(f, "%95s %llu %u %u %lf", key, &chunk, &wg, &th, &ms) == 5) {
    phos_batch_cfg c{chunk, wg, th};
    if (cfg_ok(c)) g_tune_cache[key] = {c, ms};
  }
  fclose(f);
}

void save_cache(const char *path) {
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto &kv : g_tune_cache)
    fprintf(f, "%s %llu %u %u %.6f\n", kv.first.c_str(), (unsigned long long)kv.second.first.chunk_bytes,
            kv.second.first.wg_per_cu, kv.second.first.threads, kv.second.second);
  fclose(f);
  rename(tmp.c_str(), path);
}
}  // namespace

extern "C" phos_status phos_batch_tune(int device, const phos_copy_seg *segs, uint64_t nseg,
                                       const char *cache_path, phos_batch_cfg *best,
                                       double *best_ms) {
  if (!segs || !nseg || !best) return fail(PHOS_E_INVAL, "phos_batch_tune: bad argument");
  uint64_t total = 0, nreq = 0;
  TRY(check_segs(segs, nseg, 0xFFFFFFFFu, &total, &nreq));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string key = shape_key(segs, nseg);
  load_cache(cache_path);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end()) {
    *best = it->second.first;
    if (best_ms) *best_ms = it->second.second;
    return PHOS_OK;
  }
  DeviceGuard g(device);
  phos_batch *b = nullptr;
  phos_batch_cfg c0 = default_cfg();
  TRY(phos_batch_create(device, nseg, (uint32_t)nreq, &c0, &b));
  hipStream_t s;
  hipEvent_t e0, e1;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    phos_batch_destroy(b);
    return fail(PHOS_E_HIP, "stream");
  }
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  phos_status st = phos_batch_load(b, segs, nseg, s);
  const uint64_t chunks[] = {64ull << 10, 128ull << 10, 256ull << 10, 512ull << 10,
                             1ull << 20,  2ull << 20,   4ull << 20};
  const uint32_t wgs[] = {1, 2, 4, 8};
  const uint32_t ths[] = {256, 512, 1024};
  double bms = 1e30;
  phos_batch_cfg bc = c0;
  for (uint64_t ch : chunks)
    for (uint32_t wg : wgs)
      for (uint32_t th : ths) {
        if (st != PHOS_OK) break;
        phos_batch_cfg c{ch, wg, th};
        st = phos_batch_set_cfg(b, &c);
        if (st != PHOS_OK) break;
        std::vector<float> ts;
        for (int rep = 0; rep < 4 && st == PHOS_OK; ++rep) {
          if (hipEventRecord(e0, s) != hipSuccess || phos_batch_run(b, s) != PHOS_OK ||
              hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            st = fail(PHOS_E_HIP, "tuning run failed");
            break;
          }
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep) ts.push_back(ms);  // first run warms up
        }
        if (st != PHOS_OK) break;
        std::sort(ts.begin(), ts.end());
        const double med = ts[ts.size() / 2];
        if (med < bms) {
          bms = med;
          bc = c;
        }
      }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  phos_batch_destroy(b);
  if (st != PHOS_OK) return st;
  g_tune_cache[key] = {bc, bms};
  save_cache(cache_path);
  *best = bc;
  if (best_ms) *best_ms = bms;
  return PHOS_OK;
}
