// serve.cpp — the serving loop (no paper analog): checkpoint, restore and
// on-demand-restore requests arrive on the host clock, are admitted in
// arrival order against an HBM budget, and are served either one at a time
// (plain FIFO) or by continuous batching: every admitted bulk request gets a
// share of each iteration of the persistent graph-captured copy, requests
// that arrive meanwhile join the next iteration, two iterations stay in
// flight so the GPU never waits for the host, and fault bursts run at once on
// their own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <numeric>
#include <thread>
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
using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing, page aligned.
class Arena {
 public:
  Arena(uint64_t size, uint64_t align) : align_(align) { free_[0] = size / align * align; }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = (bytes + align_ - 1) / align_ * align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      *off = o;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = (bytes + align_ - 1) / align_ * align_;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  uint64_t align_;
  std::map<uint64_t, uint64_t> free_;
};

struct Bulk {        // an admitted checkpoint / restore with work left to issue
  uint32_t idx;
  uint64_t dst;      // device address of its destination
  uint32_t seg = 0;  // issue cursor
  uint64_t seg_off = 0;
  uint64_t left = 0; // bytes not yet issued
};

struct Iter {        // one iteration of the batched copy
  phos_batch *b = nullptr;
  hipEvent_t ev = nullptr;     // the iteration's copy finished
  hipEvent_t up = nullptr;     // its work queue is uploaded
  bool busy = false;
  std::vector<std::pair<uint32_t, uint32_t>> finishing;  // (request, id in the iteration)
};

class Server {
 public:
  Server(int device, const phos_serve_cfg &cfg, const phos_serve_req *reqs, uint32_t n,
         phos_serve_out *out)
      : dev_(device), cfg_(cfg), reqs_(reqs), n_(n), out_(out),
        arena_(cfg.budget_bytes, cfg.page_bytes) {}
  ~Server() { cleanup(); }

  phos_status run(phos_serve_stats *stats);

 private:
  phos_status setup();
  void cleanup();
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0_).count();
  }
  phos_status launch_burst(uint32_t i, uint64_t dst, hipStream_t s);
  phos_status run_plain();
  phos_status run_batched();
  // GPU wall-clock stamp -> host clock (ms since the run start)
  double stamp_ms(unsigned long long s, double khz) const {
    return host0_ms_ + ((double)s - (double)gpu0_) / khz;
  }
  void complete(uint32_t i, double done_ms = -1.0) {
    out_[i].done_ms = done_ms >= 0 ? done_ms : now_ms();
    out_[i].latency_ms = out_[i].done_ms - reqs_[i].arrival_s * 1e3;
    if (!cfg_.keep) arena_.release(out_[i].dst_off, reqs_[i].bytes);
    --active_;
    ++done_;
  }
  uint64_t seg_bytes(uint32_t i) const {
    uint64_t t = 0;
    for (uint32_t s = 0; s < reqs_[i].nseg; ++s) t += reqs_[i].segs[s].bytes;
    return t;
  }

  int dev_;
  phos_serve_cfg cfg_;
  const phos_serve_req *reqs_;
  uint32_t n_;
  phos_serve_out *out_;
  Arena arena_;
  Clock::time_point t0_;
  uint32_t done_ = 0, active_ = 0, max_active_ = 0;
  uint64_t bulk_bytes_ = 0, iterations_ = 0;
  uint32_t page_shift_ = 16;
  uint32_t n_cu_ = 256;
  unsigned long long gpu0_ = 0, *h_clock_ = nullptr;  // clock calibration
  double host0_ms_ = 0;

  hipStream_t bulk_ = nullptr, burst_ = nullptr, upload_ = nullptr;
  Iter iters_[2];
  phos_batch *plain_ = nullptr;
  uint32_t *d_identity_ = nullptr, *d_err_ = nullptr;
  unsigned long long *d_faulted_ = nullptr;
  std::vector<hipEvent_t> ev_pool_;
  std::vector<phos_copy_seg> segbuf_;
};

constexpr uint32_t kIterMaxReqs = 4096;
constexpr uint64_t kIterMaxSegs = 1u << 20;

phos_status Server::setup() {
  if (!cfg_.d_arena || !cfg_.budget_bytes || !cfg_.page_bytes ||
      (cfg_.page_bytes & (cfg_.page_bytes - 1)))
    return fail(PHOS_E_INVAL, "serve: bad configuration");
  page_shift_ = (uint32_t)__builtin_ctz(cfg_.page_bytes);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev_) == hipSuccess && prop.multiProcessorCount > 0)
      n_cu_ = (uint32_t)prop.multiProcessorCount;
  }
  uint64_t max_pages = 1, max_segs = 1;
  for (uint32_t i = 0; i < n_; ++i) {
    const phos_serve_req &r = reqs_[i];
    if (r.bytes > cfg_.budget_bytes) return fail(PHOS_E_INVAL, "request %u exceeds the budget", i);
    if (i && r.arrival_s < reqs_[i - 1].arrival_s)
      return fail(PHOS_E_INVAL, "requests must be sorted by arrival");
    if (r.type == PHOS_REQ_BURST) {
      if (!r.d_state || (!r.d_records && r.nrec) || !r.image || r.bytes % cfg_.page_bytes)
        return fail(PHOS_E_INVAL, "burst %u: bad arguments", i);
      max_pages = std::max<uint64_t>(max_pages, r.bytes >> page_shift_);
    } else if (r.type == PHOS_REQ_CKPT || r.type == PHOS_REQ_RESTORE) {
      if (r.nseg && !r.segs) return fail(PHOS_E_INVAL, "request %u: no segments", i);
      for (uint32_t s = 0; s < r.nseg; ++s)
        if (r.segs[s].dst + r.segs[s].bytes > r.bytes)
          return fail(PHOS_E_INVAL, "request %u: segment beyond its destination", i);
      max_segs = std::max<uint64_t>(max_segs, r.nseg);
    } else {
      return fail(PHOS_E_INVAL, "request %u: unknown type %u", i, r.type);
    }
  }
  HIP_TRY(hipStreamCreateWithFlags(&bulk_, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&burst_, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&upload_, hipStreamNonBlocking));
  std::vector<uint32_t> ident(max_pages);
  std::iota(ident.begin(), ident.end(), 0u);
  HIP_TRY(hipMalloc((void **)&d_identity_, 4 * max_pages));
  HIP_TRY(hipMemcpy(d_identity_, ident.data(), 4 * max_pages, hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc((void **)&d_err_, 4));
  HIP_TRY(hipHostMalloc((void **)&h_clock_, 8, hipHostMallocDefault));
  HIP_TRY(hipMalloc((void **)&d_faulted_, 8));
  HIP_TRY(hipMemset(d_err_, 0, 4));
  HIP_TRY(hipMemset(d_faulted_, 0, 8));
  if (cfg_.mode == PHOS_SERVE_BATCHED) {
    for (Iter &it : iters_) {
      TRY(phos_batch_create(dev_, kIterMaxSegs, kIterMaxReqs, &cfg_.cfg, &it.b));
      HIP_TRY(hipEventCreateWithFlags(&it.ev, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&it.up, hipEventDisableTiming));
    }
  } else {
    TRY(phos_batch_create(dev_, max_segs, 1, &cfg_.cfg, &plain_));
  }
  segbuf_.reserve(1 << 16);
  return PHOS_OK;
}

void Server::cleanup() {
  (void)hipDeviceSynchronize();
  for (Iter &it : iters_) {
    if (it.b) phos_batch_destroy(it.b);
    if (it.ev) (void)hipEventDestroy(it.ev);
    if (it.up) (void)hipEventDestroy(it.up);
    it.b = nullptr;
    it.ev = it.up = nullptr;
  }
  if (plain_) phos_batch_destroy(plain_);
  plain_ = nullptr;
  for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
  ev_pool_.clear();
  if (h_clock_) (void)hipHostFree(h_clock_);
  h_clock_ = nullptr;
  if (d_identity_) (void)hipFree(d_identity_);
  if (d_err_) (void)hipFree(d_err_);
  if (d_faulted_) (void)hipFree(d_faulted_);
  d_identity_ = d_err_ = nullptr;
  d_faulted_ = nullptr;
  if (bulk_) (void)hipStreamDestroy(bulk_);
  if (burst_) (void)hipStreamDestroy(burst_);
  if (upload_) (void)hipStreamDestroy(upload_);
  bulk_ = burst_ = upload_ = nullptr;
}

// Section 6 machinery on a request's own pages: its records are offsets into
// the destination; pages not present are claimed and copied from the image.
phos_status Server::launch_burst(uint32_t i, uint64_t dst, hipStream_t s) {
  const phos_serve_req &r = reqs_[i];
  CopyArgs c;
  c.pool = reinterpret_cast<uint8_t *>(dst);
  c.image = reinterpret_cast<uint8_t *>(r.image);
  c.state = r.d_state;
  c.img_page = d_identity_;
  c.stat = d_faulted_;
  c.err = d_err_;
  c.page_shift = page_shift_;
  c.n_pages = (uint32_t)(r.bytes >> page_shift_);
  c.to_image = 0;
  c.spin_limit = env_u32("PHOS_SPIN_LIMIT", 1u << 22);
  c.nt = 0;
  c.chunk_pages = 0;
  c.image_chunks = nullptr;  // the request's image is one piece
  HIP_TRY(launch_demand(c, r.d_records, r.nrec, 0, nullptr, n_cu_, s));
  return PHOS_OK;
}

void sleep_until_ms(Clock::time_point t0, double ms) {
  const auto target = t0 + std::chrono::duration_cast<Clock::duration>(
                               std::chrono::duration<double, std::milli>(ms));
  const auto now = Clock::now();
  if (target > now + std::chrono::microseconds(200))
    std::this_thread::sleep_until(target - std::chrono::microseconds(100));
  while (Clock::now() < target) std::this_thread::yield();
}

phos_status Server::run_plain() {
  for (uint32_t i = 0; i < n_; ++i) {
    const phos_serve_req &r = reqs_[i];
    sleep_until_ms(t0_, r.arrival_s * 1e3);  // no-op when it arrived while the previous ran
    uint64_t off = 0;
    if (!arena_.alloc(r.bytes, &off)) return fail(PHOS_E_NOMEM, "plain: budget exhausted");
    out_[i].dst_off = off;
    out_[i].admit_ms = now_ms();
    ++active_;
    max_active_ = std::max(max_active_, active_);
    const uint64_t dst = reinterpret_cast<uint64_t>(cfg_.d_arena) + off;
    if (r.type == PHOS_REQ_BURST) {
      TRY(launch_burst(i, dst, bulk_));
    } else {
      segbuf_.assign(r.segs, r.segs + r.nseg);
      for (phos_copy_seg &g : segbuf_) {
        g.dst += dst;
        g.req = 0;
      }
      TRY(phos_batch_load(plain_, segbuf_.data(), segbuf_.size(), bulk_));
      TRY(phos_batch_run_plain(plain_, bulk_));
      bulk_bytes_ += seg_bytes(i);
    }
    HIP_TRY(hipStreamSynchronize(bulk_));
    const unsigned long long st = r.type != PHOS_REQ_BURST ? batch_stamps(plain_)[1] : 0;
    complete(i, st ? stamp_ms(st, batch_clock_khz(plain_)) : -1.0);
  }
  return PHOS_OK;
}

phos_status Server::run_batched() {
  uint32_t next = 0;
  std::deque<uint32_t> pending;   // arrived, not admitted
  std::deque<Bulk> bulk;          // admitted, bytes left to issue
  std::vector<std::pair<uint32_t, hipEvent_t>> bursts;
  while (done_ < n_) {
    bool progress = false;
    const double t = now_ms();
    while (next < n_ && reqs_[next].arrival_s * 1e3 <= t) pending.push_back(next++);
    // admission in arrival order while the destination fits the budget
    while (!pending.empty()) {
      const uint32_t i = pending.front();
      uint64_t off = 0;
      if (!arena_.alloc(reqs_[i].bytes, &off)) break;
      pending.pop_front();
      out_[i].dst_off = off;
      out_[i].admit_ms = now_ms();
      ++active_;
      max_active_ = std::max(max_active_, active_);
      const uint64_t dst = reinterpret_cast<uint64_t>(cfg_.d_arena) + off;
      if (reqs_[i].type == PHOS_REQ_BURST) {
        TRY(launch_burst(i, dst, burst_));
        hipEvent_t e;
        if (ev_pool_.empty()) {
          HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        } else {
          e = ev_pool_.back();
          ev_pool_.pop_back();
        }
        HIP_TRY(hipEventRecord(e, burst_));
        bursts.emplace_back(i, e);
      } else {
        Bulk b;
        b.idx = i;
        b.dst = dst;
        b.left = seg_bytes(i);
        bulk_bytes_ += b.left;
        if (b.left) bulk.push_back(b);
        else complete(i);
      }
      progress = true;
    }
    // completions
    for (Iter &it : iters_) {
      if (!it.busy) continue;
      const hipError_t q = hipEventQuery(it.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return fail(PHOS_E_HIP, "iteration: %s", hipGetErrorString(q));
      it.busy = false;
      const volatile unsigned long long *st = batch_stamps(it.b);
      for (auto &f : it.finishing) {
        const unsigned long long s = st[1 + f.second];
        complete(f.first, s ? stamp_ms(s, batch_clock_khz(it.b)) : -1.0);
      }
      it.finishing.clear();
      progress = true;
    }
    for (size_t k = 0; k < bursts.size();) {
      const hipError_t q = hipEventQuery(bursts[k].second);
      if (q == hipErrorNotReady) {
        ++k;
        continue;
      }
      if (q != hipSuccess) return fail(PHOS_E_HIP, "burst: %s", hipGetErrorString(q));
      complete(bursts[k].first);
      ev_pool_.push_back(bursts[k].second);
      bursts[k] = bursts.back();
      bursts.pop_back();
      progress = true;
    }
    // issue iterations into free slots, at most quantum bytes per request:
    // small requests (at most small_bytes left) first, shortest first, so
    // they never wait behind a large one; the large ones in arrival order,
    // so they are not starved by a stream of medium ones
    for (Iter &it : iters_) {
      if (it.busy || bulk.empty()) continue;
      const uint64_t small = cfg_.small_bytes;
      std::stable_sort(bulk.begin(), bulk.end(), [small](const Bulk &x, const Bulk &y) {
        const bool xs = x.left <= small, ys = y.left <= small;
        if (xs != ys) return xs;
        return xs ? x.left < y.left : x.idx < y.idx;
      });
      segbuf_.clear();
      uint64_t budget = cfg_.iter_bytes;
      uint32_t nreq = 0;
      for (auto b = bulk.begin(); b != bulk.end() && budget && nreq < kIterMaxReqs; ++b) {
        uint64_t take = std::min(std::min(cfg_.quantum_bytes, b->left), budget);
        const phos_serve_req &r = reqs_[b->idx];
        const uint32_t rid = nreq++;
        budget -= take;
        b->left -= take;
        while (take) {
          const phos_copy_seg &g = r.segs[b->seg];
          const uint64_t len = std::min(take, g.bytes - b->seg_off);
          if (len) {
            phos_copy_seg piece;
            piece.src = g.src + b->seg_off;
            piece.dst = b->dst + g.dst + b->seg_off;
            piece.bytes = len;
            piece.req = rid;
            piece._p = 0;
            segbuf_.push_back(piece);
          }
          take -= len;
          b->seg_off += len;
          if (b->seg_off == g.bytes) {
            ++b->seg;
            b->seg_off = 0;
          }
        }
        if (!b->left) it.finishing.emplace_back(b->idx, rid);
        if (segbuf_.size() + 4096 > kIterMaxSegs) break;
      }
      while (!bulk.empty() && !bulk.front().left) bulk.pop_front();
      bulk.erase(std::remove_if(bulk.begin(), bulk.end(), [](const Bulk &b) { return !b.left; }),
                 bulk.end());
      if (segbuf_.empty()) continue;
      // the work queue goes up on its own stream while the previous
      // iteration still copies; the copy stream only waits for the upload
      TRY(phos_batch_load(it.b, segbuf_.data(), segbuf_.size(), upload_));
      HIP_TRY(hipEventRecord(it.up, upload_));
      HIP_TRY(hipStreamWaitEvent(bulk_, it.up, 0));
      TRY(phos_batch_run(it.b, bulk_));
      HIP_TRY(hipEventRecord(it.ev, bulk_));
      it.busy = true;
      ++iterations_;
      progress = true;
    }
    if (!progress) {
      // nothing to do right now: wait for the next arrival or a completion
      const bool inflight = iters_[0].busy || iters_[1].busy || !bursts.empty();
      if (!inflight && next < n_ && pending.empty()) sleep_until_ms(t0_, reqs_[next].arrival_s * 1e3);
      else std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
  }
  return PHOS_OK;
}

phos_status Server::run(phos_serve_stats *stats) {
  TRY(setup());
  for (uint32_t i = 0; i < n_; ++i) out_[i] = phos_serve_out{-1.0, -1.0, -1.0, 0};
  HIP_TRY(hipDeviceSynchronize());
  t0_ = Clock::now();
  {  // map the GPU wall clock onto the host clock
    const double a = now_ms();
    HIP_TRY(launch_read_clock(h_clock_, bulk_));
    HIP_TRY(hipStreamSynchronize(bulk_));
    const double b = now_ms();
    gpu0_ = *(volatile unsigned long long *)h_clock_;
    host0_ms_ = 0.5 * (a + b);
  }
  phos_status st = cfg_.mode == PHOS_SERVE_BATCHED ? run_batched() : run_plain();
  HIP_TRY(hipDeviceSynchronize());
  const double wall = now_ms() - (n_ ? reqs_[0].arrival_s * 1e3 : 0.0);
  if (st != PHOS_OK) return st;
  uint32_t err = 0;
  unsigned long long faulted = 0;
  HIP_TRY(hipMemcpy(&err, d_err_, 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(&faulted, d_faulted_, 8, hipMemcpyDeviceToHost));
  if (stats) {
    stats->wall_ms = wall;
    stats->bytes = bulk_bytes_ + (faulted << page_shift_);
    stats->iterations = iterations_;
    stats->max_active = max_active_;
  }
  if (err) return fail(PHOS_E_TIMEOUT, "a device-side wait expired");
  return PHOS_OK;
}
}  // namespace

extern "C" phos_status phos_serve_run(int device, const phos_serve_cfg *cfg,
                                      const phos_serve_req *reqs, uint32_t n, phos_serve_out *out,
                                      phos_serve_stats *stats) {
  if (!cfg || (!reqs && n) || (!out && n)) return fail(PHOS_E_INVAL, "phos_serve_run: NULL");
  if (cfg->mode != PHOS_SERVE_PLAIN && cfg->mode != PHOS_SERVE_BATCHED)
    return fail(PHOS_E_INVAL, "unknown serving mode %u", cfg->mode);
  if (cfg->mode == PHOS_SERVE_BATCHED && (!cfg->quantum_bytes || !cfg->iter_bytes))
    return fail(PHOS_E_INVAL, "batched serving needs quantum and iteration sizes");
  DeviceGuard g(device);
  Server s(device, *cfg, reqs, n, out);
  return s.run(stats);
}
