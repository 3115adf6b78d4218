// kernels.hip — gfx950 kernels of the validated-speculation checkpoint/restore
// hot path (PhoenixOS, arXiv 2405.12079), written for CDNA4: wave64 ballots,
// LDS-staged interval tables and dirty bitmaps, 16-byte vector loads/stores.
//
//   validate_kernel   Section 4.1 runtime validation + Section 4.3 dirty tracking
//   vscan / vscatter  ordered compaction of the violation reports
//   cow_kernel        Section 4.2 pre-launch copy of pages about to be written
//   background_kernel Section 4.2/4.3/6 concurrent bulk copy under per-page claims
//   pagelist/gather   Section 4.3 recopy of dirty and victim pages
//   precopy_kernel    Sections 4.3/7 pre-copy round of a recopy checkpoint
//   demand_kernel     Section 6 on-demand restore of the pages a launch touches
//   batch_copy        persistent copy of many requests' segments (no paper analog)
//   twin_kernel       Section 4.1 instrumented twin of an application kernel
#include <hip/hip_runtime.h>
#include <type_traits>
#include <mutex>

#include "internal.h"
#include "util.h"

#define GLOBAL_AS __attribute__((address_space(1)))
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace phos {
namespace {

__device__ __forceinline__ uint32_t ld_acquire(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// The claim (free -> claimed) publishes nothing and the claimer reads
// nothing another block produced under it, so it needs no ordering: a
// relaxed compare-and-swap (an acquire-release one would write back the
// whole L2 before every claim).  Data is ordered by the "done" store.
__device__ __forceinline__ bool cas_u32(uint32_t *p, uint32_t &expected, uint32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup barrier that orders LDS only: it does not wait for the block's
// outstanding global stores (a __syncthreads would drain them).  The signal
// fences keep the compiler from moving any memory access across it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Block-cooperative 16-byte copy, U loads in flight per thread (8; 16 when
// the source sits across PCIe, where latency, not HBM, sets the rate);
// NT: non-temporal (streaming) loads and stores.
template <bool NT, int U>
__device__ __forceinline__ void block_copy16_t(const uint4 *__restrict__ src_,
                                               uint4 *__restrict__ dst_, uint64_t n16,
                                               uint32_t tid, uint32_t nthreads) {
  const u32x4 *__restrict__ src = reinterpret_cast<const u32x4 *>(src_);
  u32x4 *__restrict__ dst = reinterpret_cast<u32x4 *>(dst_);
  const uint64_t T = nthreads;
  uint64_t i = tid;
  for (; i + (U - 1) * T < n16; i += U * T) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = NT ? __builtin_nontemporal_load(src + i + u * T) : src[i + u * T];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NT) __builtin_nontemporal_store(v[u], dst + i + u * T);
      else dst[i + u * T] = v[u];
    }
  }
  for (; i < n16; i += T) dst[i] = src[i];
}
// tid / nthreads: this thread among the threads sharing the copy (default:
// the whole block); deep: 16 loads in flight per thread
__device__ __forceinline__ void block_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                             uint64_t n16, bool nt = false,
                                             uint32_t tid = ~0u, uint32_t nthreads = 0,
                                             bool deep = false) {
  if (tid == ~0u) {
    tid = threadIdx.x;
    nthreads = blockDim.x;
  }
  if (deep) {
    if (nt) block_copy16_t<true, 16>(src, dst, n16, tid, nthreads);
    else block_copy16_t<false, 16>(src, dst, n16, tid, nthreads);
  } else {
    if (nt) block_copy16_t<true, 8>(src, dst, n16, tid, nthreads);
    else block_copy16_t<false, 8>(src, dst, n16, tid, nthreads);
  }
}

// 32 consecutive bytes of a byte map (one per page) as a 32-bit mask.
__device__ __forceinline__ uint32_t bytes_to_mask(const uint8_t *p) {
  const uint4 a = *reinterpret_cast<const uint4 *>(p);
  const uint4 b = *reinterpret_cast<const uint4 *>(p + 16);
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) m |= ((w[i] >> (8 * j)) & 0xFFu) ? (1u << (4 * i + j)) : 0u;
  }
  return m;
}

// ============================================================ validation
// Interval bounds in scalar registers: an access at a is inside interval j
// iff lo[j] <= a <= hi8[j] (hi8 = hi - 8); empty intervals get lo = ~0,
// hi8 = 0.  Mode bits are wave-uniform, so the mode folding is scalar logic.
struct IvRegs {
  uint64_t lo[8], hi8[8];
  uint32_t mode[8];
};

// 0 = valid; 1 = in no interval; 2 = inside but the mode bit is missing.
template <int NIV>
__device__ __forceinline__ uint32_t classify_n(const IvRegs &R, uint64_t a, uint32_t w) {
  bool any = false, okr = false, okw = false;
#pragma unroll
  for (int j = 0; j < NIV; ++j) {
    const bool in = (a >= R.lo[j]) & (a <= R.hi8[j]);
    any |= in;
    if (R.mode[j] & PHOS_R) okr |= in;
    if (R.mode[j] & PHOS_W) okw |= in;
  }
  return (w ? okw : okr) ? 0u : (any ? 2u : 1u);
}

// Any number of intervals, from the LDS table.
__device__ __forceinline__ uint32_t classify_lds(const DevSpec &S, uint32_t niv, uint64_t a,
                                                 uint32_t w) {
  bool any = false, ok = false;
  for (uint32_t j = 0; j < niv; ++j) {
    const DevIv iv = S.iv[j];
    const bool in = (a - iv.lo) <= iv.span;
    any |= in;
    ok |= in & (((iv.mode >> w) & 1u) != 0);
  }
  return ok ? 0u : (any ? 2u : 1u);
}

struct VShared {
  DevSpec spec;
  uint32_t list[kVWaves][kWcap];
  uint32_t vpend[kVWaves][kVPend];  // pool pages of failing writes, marked at the tile's end
  uint32_t wcnt[kVWaves];
  uint32_t win_fw;   // first global dirty-map word of the LDS window
  uint32_t win_nw;   // window words in use, or kNone (write pages straight to the map)
  // the window words holding write-interval pages (window-relative, repeats
  // allowed) and each one's write-interval bits, or niw = kNone (more than 64)
  uint32_t niw;
  uint32_t iw[64];
  uint32_t imask[64];
  VLaunch L;
  uint32_t seq;  // sequence number of the tile's launch
  unsigned long long off;
};

// The block's LDS dirty window in the form the scan uses: a validated write
// at a marks bit ((a - lo) >> page_shift) & 31 of word (a - lo) >> word_shift
// when a - lo < bytes (the window lies inside the pool).  direct: no window
// (the write intervals span too much of the pool): marks go straight to the
// dirty map.
struct TrackWin {
  uint64_t lo, bytes;
  uint32_t word_shift;
  bool direct;
};

// Section 4.3 tracking of one record, without branches: a validated write
// marks its page in the LDS window; every other lane ORs 0 into a pad word of
// its own (kTrackWords + lane), so the wave issues one LDS atomic and no
// divergent code.  Without a window (DIRECT) the page goes straight to the
// dirty map.
template <bool DIRECT>
__device__ __forceinline__ void track_write(const VArgs &A, const TrackWin &W, uint32_t *s_track,
                                            uint64_t a, bool marks, uint32_t lane) {
  if (DIRECT) {
    const uint64_t off = a - A.pool_base;
    if (marks && off < A.pool_bytes) A.dirty[off >> A.page_shift] = 1;
    return;
  }
  const uint64_t d = a - W.lo;
  const bool in = marks && d < W.bytes;
  const uint32_t word = in ? (uint32_t)(d >> W.word_shift) : kTrackWords + lane;
  const uint32_t bit = in ? 1u << ((uint32_t)(d >> A.page_shift) & 31u) : 0u;
  atomicOr(&s_track[word], bit);  // result unused: no return
}

// A failing write at pool page `page` of launch number `seq`: inside a
// buffer, the page is a victim (Section 4.3).
__device__ __forceinline__ void track_victim(const VArgs &A, uint32_t seq, uint32_t page) {
  // the page's buffer, its victim mark and launch numbers, looked up together
  const uint32_t buf = A.page_buf[page];
  const uint8_t marked = A.victim[page];
  const uint32_t last = A.victim_seq[page], first = A.victim_first[page];
  if (buf == kNone) return;
  // the latest launch that writes here out of its speculation, and the
  // earliest (its copy-on-write copies the page).  Both only ever move one
  // way, so a value read that already covers seq (even a stale one) makes
  // the atomic unnecessary.
  if (last < seq) atomicMax(&A.victim_seq[page], seq);
  if (first > seq) atomicMin(&A.victim_first[page], seq);
  if (marked == 0) {
    // newly marked victim page (a stale read only adds a duplicate)
    A.victim[page] = 1;
    const uint32_t i = atomicAdd(&A.vmeta[0], 1u);
    if (i < A.vlist_cap) A.vlist[i] = page;
    else A.vmeta[3] = 1;
  }
}

// Keep the step's failing writes inside the pool (two records per lane,
// their pool pages) in the wave's LDS list; past its end they are marked at
// once.
__device__ __forceinline__ void rank_victims(const VArgs &A, VShared &S, uint32_t wave,
                                             uint64_t lt, bool f0, uint64_t a0, bool f1,
                                             uint64_t a1, uint32_t &vcnt) {
  const uint64_t m0 = __ballot(f0), m1 = __ballot(f1);
  if (__builtin_expect((m0 | m1) != 0, 0)) {
    const uint64_t o0 = a0 - A.pool_base, o1 = a1 - A.pool_base;
    f0 = f0 && o0 < A.pool_bytes;
    f1 = f1 && o1 < A.pool_bytes;
    const uint64_t n0 = __ballot(f0), n1 = __ballot(f1);
    const uint32_t rk = vcnt + __popcll(n0 & lt) + __popcll(n1 & lt);
    const uint32_t p0 = (uint32_t)(o0 >> A.page_shift), p1 = (uint32_t)(o1 >> A.page_shift);
    if (f0) {
      if (rk < kVPend) S.vpend[wave][rk] = p0;
      else track_victim(A, S.seq, p0);
    }
    const uint32_t rk1 = rk + (f0 ? 1u : 0u);
    if (f1) {
      if (rk1 < kVPend) S.vpend[wave][rk1] = p1;
      else track_victim(A, S.seq, p1);
    }
    vcnt += __popcll(n0) + __popcll(n1);
  }
}

// Rank the step's violating records inside the wave (two records per lane,
// interleaved in index order) and keep their local indices in LDS.
__device__ __forceinline__ void rank_violations(VShared &S, uint32_t wave, uint64_t lt, bool b0,
                                                bool b1, uint32_t local, uint32_t &wcnt) {
  const uint64_t m0 = __ballot(b0), m1 = __ballot(b1);
  if (__builtin_expect((m0 | m1) != 0, 0)) {
    const uint32_t rk = wcnt + __popcll(m0 & lt) + __popcll(m1 & lt);
    if (b0 && rk < kWcap) S.list[wave][rk] = local;
    const uint32_t rk1 = rk + (b0 ? 1u : 0u);
    if (b1 && rk1 < kWcap) S.list[wave][rk1] = local + 1;
    wcnt += __popcll(m0) + __popcll(m1);
  }
}

// One wave's range [wbase, wend) of records; NIV < 0: intervals from LDS.
// TRACK: 0 none, 1 the LDS window, 2 straight to the dirty map.  With TRACK
// 1 and `check`, every other step the wave looks at the window words that
// hold write-interval pages (lane i: word iw_lane); once all those pages are
// marked, the rest of the range only looks for failing writes (the same
// software pipeline, a second copy of the step without the marks).
template <int NIV, int TRACK>
__device__ __forceinline__ uint32_t scan_range(const VArgs &A, VShared &S, uint32_t *s_track,
                                               const TrackWin &TW, uint32_t niv,
                                               const GLOBAL_AS uint64_t *rec8, bool al16,
                                               uint64_t wbase, uint64_t wend, uint32_t wave,
                                               uint32_t lane, uint32_t &vcnt, uint32_t iw_lane,
                                               bool check) {
  // this specialization's bounds, from LDS into registers (uniform values;
  // kept in VGPRs: scalar registers are needed for the comparison masks)
  IvRegs R;
#pragma unroll
  for (int j = 0; j < (NIV > 0 ? NIV : 0); ++j) {
    const DevIv iv = S.spec.iv[j];
    R.lo[j] = iv.lo;
    R.hi8[j] = iv.lo == ~0ull ? 0ull : iv.lo + iv.span;
    R.mode[j] = rfl(iv.mode);
  }
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t wcnt = 0;
  uint64_t c = wbase;
  // MARK: validated writes mark their pages (fw: a failing write, its victim
  // marks taken by rank_victims)
  auto one = [&](auto MARK, uint64_t r, bool valid, bool &fw) -> bool {
    const uint64_t a = r & ~7ull;
    const uint32_t w = (uint32_t)(r & 1u);
    const uint32_t reason = NIV >= 0 ? classify_n<(NIV >= 0 ? NIV : 0)>(R, a, w)
                                     : classify_lds(S.spec, niv, a, w);
    fw = false;
    if (TRACK) {
      if constexpr (decltype(MARK)::value)
        track_write<TRACK == 2>(A, TW, s_track, a, valid && w && reason == 0, lane);
      fw = valid && w && reason != 0;
    }
    return valid && reason != 0 && ((A.flags >> w) & 1u);
  };
  // main body: whole steps only, software pipelined: the next step's four
  // 16-byte loads are in flight while this step is classified (the last
  // step reloads itself instead of branching)
  constexpr uint32_t U = kVUnroll;
  constexpr uint64_t kS = (uint64_t)kVStep * kVUnroll;
  bool full = false;  // wave-uniform
  if (al16 && c + kS <= wend) {
    const GLOBAL_AS u32x4 *__restrict__ rec4 = (const GLOBAL_AS u32x4 *)rec8;
    u32x4 q[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) q[u] = rec4[((c + u * kVStep) >> 1) + lane];
    auto step = [&](auto MARK) {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint64_t r0 = ((uint64_t)q[u].y << 32) | q[u].x, r1 = ((uint64_t)q[u].w << 32) | q[u].z;
        bool f0, f1;
        const bool b0 = one(MARK, r0, true, f0);
        const bool b1 = one(MARK, r1, true, f1);
        rank_violations(S, wave, lt, b0, b1, (uint32_t)(c - wbase) + u * kVStep + 2 * lane, wcnt);
        if (TRACK) rank_victims(A, S, wave, lt, f0, r0 & ~7ull, f1, r1 & ~7ull, vcnt);
      }
    };
    uint32_t it = 0;
    for (;;) {
      const bool more = c + 2 * kS <= wend;
      const uint64_t cn = more ? c + kS : c;
      u32x4 nq[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) nq[u] = rec4[((cn + u * kVStep) >> 1) + lane];
      if (TRACK == 1 && full) step(std::false_type{});
      else step(std::true_type{});
      c += kS;
      if (!more) break;
      if (TRACK == 1 && check && !full && (++it & 1u) == 0) {
        const uint32_t v = iw_lane != kNone ? s_track[iw_lane] : ~0u;
        full = __ballot(v != ~0u) == 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) q[u] = nq[u];
    }
  }
  // tail (and 8-byte-aligned arrays): 128 records per step, guarded loads
  for (; c < wend; c += kVStep) {
    const uint64_t i0 = c + 2 * lane;
    const bool v0 = i0 < wend, v1 = i0 + 1 < wend;
    const uint64_t r0 = v0 ? rec8[i0] : 0, r1 = v1 ? rec8[i0 + 1] : 0;
    bool f0, f1;
    const bool b0 = one(std::true_type{}, r0, v0, f0);
    const bool b1 = one(std::true_type{}, r1, v1, f1);
    rank_violations(S, wave, lt, b0, b1, (uint32_t)(i0 - wbase), wcnt);
    if (TRACK) rank_victims(A, S, wave, lt, f0, r0 & ~7ull, f1, r1 & ~7ull, vcnt);
  }
  return wcnt;
}

__device__ __forceinline__ void emit_violation(const VArgs &A, const VShared &S, uint32_t niv,
                                               uint64_t idx, uint64_t r, unsigned long long pos) {
  if (pos >= A.scratch_cap) return;
  const uint64_t a = r & ~7ull;
  const uint32_t w = (uint32_t)(r & 1u);
  const uint64_t off = a - A.pool_base;
  const uint32_t b = off < A.pool_bytes ? A.page_buf[off >> A.page_shift] : kNone;
  phos_violation v;
  v.index = idx;
  v.addr = a;
  v.launch_id = S.L.launch_id;
  v.is_write = (uint8_t)w;
  v.reason = (uint8_t)classify_lds(S.spec, niv, a, w);
  v._p = 0;
  v.victim = (int32_t)b;
  v._q = 0;
  A.scratch[pos] = v;
}

template <bool BATCH, bool TRACK>
__global__ void __launch_bounds__(kVThreads) validate_kernel(VArgs A, DevSpec single) {
  __shared__ VShared S;
  __shared__ uint32_t s_track[TRACK ? kTrackWords + 64 : 1];  // the window, then 64 pad words
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t tile = blockIdx.x;

  if (tid == 0) {
    const uint32_t pos = BATCH ? A.tile_launch[tile] : 0u;
    S.L = BATCH ? A.launches[pos] : A.single;
    S.seq = A.seq0 + pos;
  }
  __syncthreads();
  const uint32_t niv = rfl(BATCH ? S.L.niv : single.niv);
  for (uint32_t j = tid; j < niv; j += kVThreads)
    S.spec.iv[j] = BATCH ? A.ivs[S.L.iv_off + j] : single.iv[j];
  __syncthreads();

  if (TRACK) {
    // The window, built by wave 0 with a lane per interval (at most kMaxIv =
    // 64): one LDS window of whole dirty-map words spanning every write
    // interval, and the window words holding write-interval pages, if at
    // most 64 (with them the scan can tell when every such page is marked).
    static_assert(kMaxIv <= 64, "one lane per interval");
    if (wave == 0) {
      const uint64_t pool_end = A.pool_base + A.pool_bytes;
      uint32_t f = kNone, l = 0, p0 = 1u, p1 = 0u;  // this lane's words and pages (p0 > p1: none)
      if (lane < niv) {
        const DevIv iv = S.spec.iv[lane];
        const uint64_t hi = iv.lo + iv.span + 8;
        const uint64_t lo_c = iv.lo > A.pool_base ? iv.lo : A.pool_base;
        const uint64_t hi_c = hi < pool_end ? hi : pool_end;
        if ((iv.mode & PHOS_W) && iv.lo != ~0ull && hi_c > lo_c) {
          p0 = (uint32_t)((lo_c - A.pool_base) >> A.page_shift);
          p1 = (uint32_t)((hi_c - 1 - A.pool_base) >> A.page_shift);
          f = p0 >> 5;
          l = p1 >> 5;
        }
      }
      uint32_t fw = f, lw = l;
      for (uint32_t d = 32; d; d >>= 1) {
        const uint32_t of = __shfl_xor(fw, (int)d, 64), ol = __shfl_xor(lw, (int)d, 64);
        fw = of < fw ? of : fw;
        lw = ol > lw ? ol : lw;
      }
      const uint32_t nw =
          (fw != kNone && lw - fw + 1 <= kTrackWords) ? lw - fw + 1 : (fw == kNone ? 0u : kNone);
      // the list: each interval's words at its exclusive prefix of word counts
      const uint32_t c = f != kNone ? l - f + 1 : 0u;
      uint32_t incl = c;
      for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t x = __shfl_up(incl, d, 64);
        if (lane >= d) incl += x;
      }
      const uint32_t total = __shfl(incl, 63, 64);
      const uint32_t niw = (nw == kNone || nw == 0 || total > 64u) ? kNone : total;
      if (lane == 0) {
        S.win_fw = fw;
        S.win_nw = nw;
        S.niw = niw;
      }
      // Lane i takes list entry i: the word of the interval whose words
      // cover position i.  Pages of the listed words outside the write
      // intervals start marked, so the words are all ones once every
      // write-interval page is (the flush masks those pages off again); a
      // word listed twice stores the same value twice.
      if (niw != kNone) {
        uint32_t gw = 0;
        for (uint32_t j = 0; j < niv; ++j) {
          const uint32_t qs = __shfl(incl - c, (int)j, 64), qc = __shfl(c, (int)j, 64);
          const uint32_t qf = __shfl(f, (int)j, 64);
          if (lane >= qs && lane < qs + qc) gw = qf + (lane - qs);
        }
        const uint32_t base = gw * 32u;
        uint32_t m = 0;
        for (uint32_t j = 0; j < niv; ++j) {
          const uint32_t q0 = __shfl(p0, (int)j, 64), q1 = __shfl(p1, (int)j, 64);
          if (q0 > q1 || q1 < base || q0 > base + 31u) continue;
          const uint32_t x = q0 > base ? q0 - base : 0u, y = q1 < base + 31u ? q1 - base : 31u;
          m |= (y == 31u ? ~0u : (2u << y) - 1u) & ~((1u << x) - 1u);
        }
        if (lane < niw) {
          S.iw[lane] = gw - fw;
          S.imask[lane] = m;
          s_track[gw - fw] = ~m;
        }
      }
    }
    __syncthreads();
    // Without the word list the whole window starts clear.
    if (S.niw == kNone && S.win_nw != kNone)
      for (uint32_t j = tid; j < S.win_nw; j += kVThreads) s_track[j] = 0;
    __syncthreads();
  }

  const uint64_t n = S.L.n;
  const uint64_t *rec = S.L.rec;
  // the record pointer came through LDS: restate that it is global memory so
  // the loads are global (not flat) loads
  const GLOBAL_AS uint64_t *__restrict__ rec8 = (const GLOBAL_AS uint64_t *)rec;
  const uint32_t Q = A.tile_recs / kVWaves;
  const uint64_t wbase = (uint64_t)(tile - S.L.tile0) * A.tile_recs + (uint64_t)wave * Q;
  const uint64_t wend = wbase + Q < n ? wbase + Q : n;
  const bool al16 = (((uintptr_t)rec) & 15u) == 0;
  uint32_t wcnt = 0, vcnt = 0;
  // the window, read once into (wave-uniform) registers
  TrackWin TW{0, 0, 0, true};
  if (TRACK) {
    const uint32_t wfw = rfl(S.win_fw), wnw = rfl(S.win_nw);
    TW.direct = wnw == kNone;
    TW.word_shift = A.page_shift + 5;
    TW.lo = A.pool_base + (TW.direct || wnw == 0 ? 0ull : (uint64_t)wfw << TW.word_shift);
    TW.bytes = TW.direct ? 0ull : (uint64_t)wnw << TW.word_shift;
  }
  // the window words this lane watches for the early stop
  uint32_t iw_lane = kNone;
  bool check = false;
  if (TRACK && !TW.direct) {
    const uint32_t niw = rfl(S.niw);
    check = niw != kNone && niw != 0;
    if (check && lane < niw) iw_lane = S.iw[lane];
  }
#define PHOS_SCAN(N)                                                                          \
  wcnt = scan_range<N, TRACK ? 1 : 0>(A, S, s_track, TW, niv, rec8, al16, wbase, wend, wave, lane, \
                                      vcnt, iw_lane, check)
  if (TRACK && TW.direct)
    wcnt = scan_range<-1, 2>(A, S, s_track, TW, niv, rec8, al16, wbase, wend, wave, lane, vcnt,
                             kNone, false);
  else switch (niv) {
    case 0: PHOS_SCAN(0); break;
    case 1: PHOS_SCAN(1); break;
    case 2: PHOS_SCAN(2); break;
    case 3: PHOS_SCAN(3); break;
    case 4: PHOS_SCAN(4); break;
    case 5: PHOS_SCAN(5); break;
    case 6: PHOS_SCAN(6); break;
    case 7: PHOS_SCAN(7); break;
    case 8: PHOS_SCAN(8); break;
    default: PHOS_SCAN(-1); break;
  }
#undef PHOS_SCAN

  if (lane == 0) S.wcnt[wave] = wcnt;
  __syncthreads();

  if (TRACK) {  // the failing writes this wave kept
    const uint32_t nv = vcnt < kVPend ? vcnt : kVPend;
    for (uint32_t j = lane; j < nv; j += 64) track_victim(A, S.seq, S.vpend[wave][j]);
  }
  if (TRACK && S.win_nw != kNone && S.win_nw) {
    // Flush the window, one word (32 pages) per thread: a plain byte store
    // per marked page, without reading the map first (the page maps need no
    // atomics, byte stores from different L2s never clobber each other, and
    // storing a mark again changes nothing).
    // With the word list only its words can hold marks (and their pages
    // outside the write intervals were set at the start).
    const uint32_t niw = S.niw;
    const uint32_t nf = niw != kNone ? niw : S.win_nw;
    for (uint32_t i = tid; i < nf; i += kVThreads) {
      const uint32_t lw = niw != kNone ? S.iw[i] : i;
      const uint32_t bits = s_track[lw] & (niw != kNone ? S.imask[i] : ~0u);
      if (!bits) continue;
      uint8_t *d = A.dirty + 32ull * (S.win_fw + lw);
      if (bits == ~0u) {
        const uint4 ones = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
        reinterpret_cast<uint4 *>(d)[0] = ones;
        reinterpret_cast<uint4 *>(d)[1] = ones;
      } else {
        for (uint32_t m = bits; m; m &= m - 1) d[__ffs(m) - 1] = 1;
      }
    }
  }

  if (tid == 0) {
    uint32_t total = 0;
    for (uint32_t w = 0; w < kVWaves; ++w) total += S.wcnt[w];
    A.tile_count[tile] = total;
    unsigned long long off = 0;
    if (total) {
      off = atomicAdd(A.cursor, (unsigned long long)total);
      A.tile_off[tile] = off;
      atomicAdd(&A.seg_sum[tile / kSeg], (unsigned long long)total);
    }
    S.off = off;
  }
  __syncthreads();
  unsigned long long start = S.off;
  for (uint32_t w = 0; w < wave; ++w) start += S.wcnt[w];
  if (wcnt == 0) {
  } else if (wcnt <= kWcap) {
    for (uint32_t j = lane; j < wcnt; j += 64) {
      const uint64_t i = wbase + S.list[wave][j];
      emit_violation(A, S, niv, i, rec8[i], start + j);
    }
  } else {
    // More violations than the LDS list holds: rescan this wave's range in
    // order and write each one at its rank (rare: degenerate launches).
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t cnt = 0;
    for (uint64_t cc = wbase; cc < wend; cc += kVStep) {
      const uint64_t i0 = cc + 2 * lane;
      const uint64_t r0 = i0 < wend ? rec8[i0] : 0, r1 = i0 + 1 < wend ? rec8[i0 + 1] : 0;
      const bool b0 = i0 < wend && classify_lds(S.spec, niv, r0 & ~7ull, (uint32_t)(r0 & 1u)) &&
                      ((A.flags >> (r0 & 1u)) & 1u);
      const bool b1 = i0 + 1 < wend && classify_lds(S.spec, niv, r1 & ~7ull, (uint32_t)(r1 & 1u)) &&
                      ((A.flags >> (r1 & 1u)) & 1u);
      const uint64_t m0 = __ballot(b0), m1 = __ballot(b1);
      const uint32_t rk = cnt + __popcll(m0 & lt) + __popcll(m1 & lt);
      if (b0) emit_violation(A, S, niv, i0, r0, start + rk);
      if (b1) emit_violation(A, S, niv, i0 + 1, r1, start + rk + (b0 ? 1u : 0u));
      cnt += __popcll(m0) + __popcll(m1);
    }
  }
}

// Calls of at most kFuseTiles tiles, in one kernel: every workgroup scans
// the tile counts itself (at most kFuseTiles of them, from L2) and keeps each
// tile's destination in LDS; then each wave moves whole tiles (tile i by
// wave i % (waves of the grid)), its lanes one violation each.  Workgroup 0
// also writes the total and resets the workspace counters (nothing here
// reads them).
__global__ void __launch_bounds__(1024)
    vfinish_kernel(const uint32_t *tile_count, const unsigned long long *tile_off, uint32_t ntiles,
                   const phos_violation *scratch, uint64_t scratch_cap, phos_violation *out,
                   uint64_t cap, uint64_t *n_out, unsigned long long *cursor,
                   unsigned long long *seg_sum, uint32_t *overflow) {
  __shared__ unsigned long long s[1024];
  __shared__ unsigned long long s_dst[kFuseTiles];
  const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
  const uint32_t per = (ntiles + 1023) / 1024;
  const uint32_t t0 = t * per < ntiles ? t * per : ntiles;
  const uint32_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  unsigned long long sum = 0;
  for (uint32_t i = t0; i < t1; ++i) sum += tile_count[i];
  s[t] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    const unsigned long long x = t >= d ? s[t - d] : 0ull;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  unsigned long long dst = s[t] - sum;
  for (uint32_t i = t0; i < t1; ++i) {
    s_dst[i] = dst;
    dst += tile_count[i];
  }
  __syncthreads();
  const uint32_t waves = gridDim.x * (blockDim.x / 64u);
  for (uint32_t i = blockIdx.x * (blockDim.x / 64u) + wave; i < ntiles; i += waves) {
    const uint32_t c = tile_count[i];
    if (!c) continue;
    const unsigned long long src = tile_off[i], d0 = s_dst[i];
    for (uint32_t j = lane; j < c; j += 64) {
      if (d0 + j >= cap || src + j >= scratch_cap) continue;
      const u32x4 *from = reinterpret_cast<const u32x4 *>(scratch + src + j);
      u32x4 *to = reinterpret_cast<u32x4 *>(out + d0 + j);
      const u32x4 a0 = from[0], a1 = from[1];
      to[0] = a0;
      to[1] = a1;
    }
  }
  if (blockIdx.x == 0) {
    if (t == 1023) {
      *n_out = s[1023];
      *cursor = 0;
      if (overflow && s[1023] > cap) atomicOr(overflow, 1u);  // sticky until read
    }
    for (uint32_t i = t; i < (ntiles + kSeg - 1) / kSeg; i += 1024) seg_sum[i] = 0;
  }
}

// Exclusive scan of per-segment violation counts (one block of 1024).
__global__ void __launch_bounds__(1024)
    vscan_kernel(unsigned long long *seg_sum, uint32_t nseg, unsigned long long *seg_prefix,
                 uint64_t *n_out, unsigned long long *cursor, uint64_t cap, uint32_t *overflow) {
  __shared__ unsigned long long s[1024];
  const uint32_t t = threadIdx.x;
  unsigned long long carry = 0;
  for (uint32_t base = 0; base < nseg; base += 1024) {
    const unsigned long long v = base + t < nseg ? seg_sum[base + t] : 0ull;
    s[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      const unsigned long long x = t >= d ? s[t - d] : 0ull;
      __syncthreads();
      s[t] += x;
      __syncthreads();
    }
    if (base + t < nseg) {
      seg_prefix[base + t] = carry + s[t] - v;
      seg_sum[base + t] = 0;
    }
    carry += s[1023];
    __syncthreads();
  }
  if (t == 0) {
    *n_out = carry;
    *cursor = 0;
    if (overflow && carry > cap) atomicOr(overflow, 1u);  // sticky until read
  }
}

// Move each tile's violations from scratch to their ordered place.  One
// block per kScatTiles tiles (a call of 30,000 tiles fills the GPU instead of
// 30 CUs): the block adds up the counts of its segment's tiles before its
// own, scans its own counts in one wave, and its four waves move the tiles,
// one violation per lane as two 16-byte loads and stores.
constexpr uint32_t kScatTiles = 16;  // a scatter block's tiles: four per wave
static_assert(kSeg % kScatTiles == 0, "a scatter block's tiles lie in one segment");

__global__ void __launch_bounds__(256)
    vscatter_kernel(const uint32_t *tile_count, const unsigned long long *tile_off, uint32_t ntiles,
                    const unsigned long long *seg_prefix, const phos_violation *scratch,
                    uint64_t scratch_cap, phos_violation *out, uint64_t cap) {
  __shared__ unsigned long long s_red[4];
  __shared__ uint32_t s_cnt[kScatTiles];
  __shared__ unsigned long long s_dst[kScatTiles];
  const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
  const uint32_t tile0 = blockIdx.x * kScatTiles;
  const uint32_t seg0 = tile0 / kSeg * kSeg;
  unsigned long long before = 0;  // this segment's violations before tile0
  for (uint32_t k = seg0 + t; k < tile0; k += 256) before += tile_count[k];
  for (uint32_t d = 32; d; d >>= 1) before += __shfl_xor(before, (int)d, 64);
  if (lane == 0) s_red[wave] = before;
  __syncthreads();
  if (wave == 0) {
    const uint32_t tk = tile0 + lane;
    const uint32_t c = lane < kScatTiles && tk < ntiles ? tile_count[tk] : 0u;
    uint32_t incl = c;
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint32_t x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    if (lane < kScatTiles) {
      s_cnt[lane] = c;
      s_dst[lane] = seg_prefix[tile0 / kSeg] + s_red[0] + s_red[1] + s_red[2] + s_red[3] + (incl - c);
    }
  }
  __syncthreads();
  for (uint32_t k = wave; k < kScatTiles; k += 4) {
    const uint32_t tk = tile0 + k;
    if (tk >= ntiles) break;
    const uint32_t ck = s_cnt[k];
    if (!ck) continue;
    const unsigned long long dst = s_dst[k], src = tile_off[tk];
    for (uint32_t i = lane; i < ck; i += 64) {
      if (dst + i >= cap || src + i >= scratch_cap) continue;
      const u32x4 *from = reinterpret_cast<const u32x4 *>(scratch + src + i);
      u32x4 *to = reinterpret_cast<u32x4 *>(out + dst + i);
      const u32x4 a0 = from[0], a1 = from[1];
      to[0] = a0;
      to[1] = a1;
    }
  }
}

// ============================================================ page copies
// Pool page p <-> image page ip.
// DEEP: 16 loads in flight per thread (kernel instances for images across
// PCIe; the others keep the smaller register footprint)
template <bool DEEP = false>
__device__ __forceinline__ void copy_page(const CopyArgs &C, uint32_t p, uint32_t ip,
                                          uint32_t tid = ~0u, uint32_t nthreads = 0) {
  const uint64_t pb = 1ull << C.page_shift;
  uint8_t *pool_p = C.pool + ((uint64_t)p << C.page_shift);
  uint8_t *img_p;
  if (C.image_chunks) {  // image in pieces of chunk_pages pages
    const uint32_t c = ip / C.chunk_pages;
    img_p = reinterpret_cast<uint8_t *>(C.image_chunks[c]) +
            ((uint64_t)(ip - c * C.chunk_pages) << C.page_shift);
  } else {
    img_p = C.image + ((uint64_t)ip << C.page_shift);
  }
  const uint4 *src = reinterpret_cast<const uint4 *>(C.to_image ? pool_p : img_p);
  uint4 *dst = reinterpret_cast<uint4 *>(C.to_image ? img_p : pool_p);
  block_copy16(src, dst, pb >> 4, C.nt != 0, tid, nthreads, DEEP);
}

// A bounded wait gives up after C.spin_limit polls, or as soon as any other
// wait of the same context has given up (the error word is read every 64
// polls): one lost publication then ends every waiter promptly, and the call
// reports PHOS_E_TIMEOUT, instead of each waiter spending its whole budget.
__device__ __forceinline__ bool wait_expired(const CopyArgs &C, uint32_t it) {
  if (it > C.spin_limit || ((it & 63u) == 0 && ld_relaxed(C.err) != 0u)) {
    atomicOr(C.err, 1u);
    return true;
  }
  return false;
}

// Blocking staging: slot `slot` (ring position pos) may be written once the
// drain of its previous occupant, slot - stage_cap, is published.  With
// WAIT, one thread of the block waits (bounded; false: the wait gave up);
// without, it only looks once.
template <bool WAIT>
__device__ __forceinline__ bool stage_room(const CopyArgs &C, unsigned long long slot, uint32_t pos) {
  if (slot < C.stage_cap) return true;
  const uint32_t need = (uint32_t)(slot - C.stage_cap + 1);
  uint32_t it = 0;
  // the copy engine writes free_seq in memory: read it at system scope
  while ((int32_t)(__hip_atomic_load(&C.free_seq[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) -
                   need) < 0) {
    if (!WAIT) return false;
    __builtin_amdgcn_s_sleep(8);
    if (wait_expired(C, ++it)) return false;
  }
  return true;
}

// Blocking staging, block-collective: publish the slots of won pages
// [j0, j1) to the host's drain (all but those marked kNone in won_ip, whose
// wait gave up).  Each slot's word packs its sequence number + 1 (high half)
// with its pool page (low half), so one store publishes both.  Every wave's slot
// stores have completed into the L2 before the barrier, and one
// system-scope release then writes the L2 back, so the copy engine that
// drains a published slot reads the page, not what the slot held before.
__device__ __forceinline__ void stage_publish(const CopyArgs &C, unsigned long long slot0,
                                              uint32_t j0, uint32_t j1, const uint32_t *won,
                                              const uint32_t *won_ip) {
  if (j0 >= j1) return;  // block-uniform
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    for (uint32_t j = j0; j < j1; ++j) {
      if (won_ip[j] == kNone) continue;  // not staged (its wait gave up)
      const unsigned long long slot = slot0 + j;
      const uint64_t v = ((uint64_t)(uint32_t)(slot + 1) << 32) | won[j];
      __hip_atomic_store(&C.fill[slot % C.stage_cap], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Block-collective: every thread offers at most one candidate page.  Pages
// still free are claimed (one winner per page across the whole GPU), copied
// by this block, then published as done; with WAIT, a thread whose page is
// claimed by someone else waits until it is done.  Every claimer publishes
// before it waits, so no wait can form a cycle.
template <bool WAIT, bool DEEP = false>
__device__ void claim_copy(uint32_t cand, const CopyArgs &C, unsigned long long *extra) {
  __shared__ uint32_t s_won[kCThreads], s_won_ip[kCThreads];
  __shared__ uint32_t s_nwon;
  if (threadIdx.x == 0) s_nwon = 0;
  __syncthreads();
  bool wait = false;
  const uint32_t ip = cand != kNone ? C.img_page[cand] : kNone;
  if (ip != kNone) {
    // A plain (possibly L2-stale) read can only lag behind: kDone is final
    // until the next quiesce, so "done" is trusted and anything else goes
    // through the compare-and-swap.
    uint32_t st = C.state[cand];
    if (st != kFree && st != kDone) st = ld_relaxed(&C.state[cand]);
    if (st == kHost || st == kWanted) {
      // held by the host's DMA: the first waiter asks the host for it
      uint32_t exp = kHost;
      if (st == kHost && C.want && cas_u32(&C.state[cand], exp, kWanted)) {
        const uint32_t i =
            __hip_atomic_fetch_add(&C.want[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (i < C.want_cap) {  // past the cap the bulk DMA brings it
          __hip_atomic_store(&C.want[1 + i], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          // push it out now: this wave is about to spin, and a store left
          // in a write buffer would reach the host only when the kernel ends
          __threadfence_system();
        }
      }
      st = kWanted;
    } else if (st == kFree) {
      uint32_t exp = kFree;
      if (cas_u32(&C.state[cand], exp, kClaimed)) {
        const uint32_t slot = atomicAdd(&s_nwon, 1u);
        s_won[slot] = cand;
        s_won_ip[slot] = ip;  // image page read once, here
        st = kDone;  // ours: published below
      } else {
        st = exp;
      }
    }
    wait = (st == kClaimed || st == kWanted);
  }
  __syncthreads();
  const uint32_t nwon = s_nwon;
  // Section 6: a launch is waiting for these pages: hold the background copy
  // back while they move (this block waits for nobody until it lets go)
  const bool priority = nwon && C.demand && !C.to_image;
  if (priority && threadIdx.x == 0) atomicAdd(C.demand, 1ull);
  if (C.stage && C.to_image) {
    // copy-on-write into a host image: the first pages go to the device
    // staging area at HBM speed (moved to the image when the checkpoint
    // ends), the rest straight to the host once the area is full; under the
    // blocking policy every page takes a slot of the ring, waiting for one
    // the host's drain has freed
    __shared__ unsigned long long s_slot0;
    __shared__ uint32_t s_room;
    if (threadIdx.x == 0) s_slot0 = nwon ? atomicAdd(C.stage_head, (unsigned long long)nwon) : 0;
    __syncthreads();
    const unsigned long long slot0 = s_slot0;
    const uint64_t pb = 1ull << C.page_shift;
    uint32_t pend = 0;  // blocking policy: won pages [pend, i) are staged, not yet published
    for (uint32_t i = 0; i < nwon; ++i) {
      const unsigned long long slot = slot0 + i;
      if (C.stage_block) {
        const uint32_t pos = (uint32_t)(slot % C.stage_cap);
        if (threadIdx.x == 0) s_room = stage_room<false>(C, slot, pos);
        __syncthreads();
        if (!s_room) {
          // about to wait: what this block has staged goes to the drain
          // first (with a short ring the slot waited for may be behind it)
          stage_publish(C, slot0, pend, i, s_won, s_won_ip);
          pend = i;
          __syncthreads();
          if (threadIdx.x == 0) s_room = stage_room<true>(C, slot, pos);
          __syncthreads();
        }
        const bool room = s_room != 0;
        if (room)
          block_copy16(reinterpret_cast<const uint4 *>(C.pool + ((uint64_t)s_won[i] << C.page_shift)),
                       reinterpret_cast<uint4 *>(C.stage + (uint64_t)pos * pb), pb >> 4, C.nt != 0);
        else
          copy_page<DEEP>(C, s_won[i], s_won_ip[i]);
        __syncthreads();  // every wave has read s_room and s_won_ip[i]
        // a page whose wait gave up went straight to the image; its slot
        // still holds an undrained page and is not published (the
        // checkpoint reports the timeout)
        if (threadIdx.x == 0 && !room) s_won_ip[i] = kNone;
      } else if (slot < C.stage_cap) {
        block_copy16(reinterpret_cast<const uint4 *>(C.pool + ((uint64_t)s_won[i] << C.page_shift)),
                     reinterpret_cast<uint4 *>(C.stage + slot * pb), pb >> 4, C.nt != 0);
        if (threadIdx.x == 0) C.stage_page[slot] = s_won[i];
      } else {
        copy_page<DEEP>(C, s_won[i], s_won_ip[i]);
      }
    }
    if (C.stage_block) {
      __syncthreads();  // the last hole mark is visible
      stage_publish(C, slot0, pend, nwon, s_won, s_won_ip);
    }
  } else {
    for (uint32_t i = 0; i < nwon; ++i) copy_page<DEEP>(C, s_won[i], s_won_ip[i]);
  }
  // Publishing "done".  Checkpoint direction: a waiter only needs this
  // block's reads of the pool to have returned (the image is read after the
  // kernel ends), so waiting for every outstanding access is enough.
  // Restore direction: the pool writes must reach memory before anyone on
  // another XCD reads them, which takes a device-scope release.
  if (nwon) {
    if (C.to_image) __builtin_amdgcn_s_waitcnt(0);
    else __threadfence();
  }
  __syncthreads();
  if (threadIdx.x < nwon) {
    if (C.to_image)
      __hip_atomic_store(&C.state[s_won[threadIdx.x]], kDone, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    else
      st_release(&C.state[s_won[threadIdx.x]], kDone);
  }
  if (threadIdx.x == 0 && nwon) {
    atomicAdd(C.stat, (unsigned long long)nwon);
    if (extra) atomicAdd(extra, (unsigned long long)nwon);
    if (priority) atomicAdd(C.demand, ~0ull);  // -1
  }
  if (WAIT && wait) {
    uint32_t it = 0;
    while (ld_acquire(&C.state[cand]) != kDone) {
      __builtin_amdgcn_s_sleep(8);
      if (wait_expired(C, ++it)) break;
    }
  }
  __syncthreads();
}

// Section 4.2: work units of kUnitPages pages of the write intervals, then
// units of kVictimUnit victim pages (pages hit by failing writes inside buffers);
// a persistent grid strides over them and skips units already copied.
static_assert(kUnitPages <= kCThreads && kVictimUnit <= kCThreads, "one candidate per thread");
__device__ __forceinline__ bool unit_needed(const CopyArgs &C, uint32_t cand) {
  return __syncthreads_or(cand != kNone && C.img_page[cand] != kNone && C.state[cand] != kDone);
}

template <bool DEEP>
__global__ void __launch_bounds__(kCThreads)
    cow_kernel(CopyArgs C, PageRanges R, VictimList V, uint32_t wait) {
  const uint32_t t = threadIdx.x;
  const uint32_t range_units = R.units_prefix[R.n];
  // victim pages marked since the previous call: entries [start, end)
  uint32_t start = 0, end = 0, map_units = 0;
  const uint32_t *vlist = V.list;
  const uint32_t all_map_units = (V.map_words + kCThreads / 4 - 1) / (kCThreads / 4);
  if (V.meta && V.scan_map) {
    map_units = all_map_units;
  } else if (V.meta && V.bucket) {
    vlist = V.bucket;
    start = *V.bstart;
    end = *V.bend;
    if (V.meta[3]) map_units = all_map_units;  // the list overflowed
  } else if (V.meta) {
    start = V.meta[1];
    end = V.meta[0] < V.cap ? V.meta[0] : V.cap;
    if (V.meta[3]) map_units = all_map_units;  // the list overflowed
  }
  const uint32_t list_units = end > start ? (end - start + kVictimUnit - 1) / kVictimUnit : 0;
  uint32_t units = range_units + list_units + map_units;
  // The background copy has finished, and the copy-on-write calls come from
  // one stream (the earlier ones are complete): every page is done already,
  // so there is nothing to scan.  The block still takes part in the victim
  // cursor update below.
  __shared__ uint32_t s_skip;  // one decision for the whole block
  if (t == 0)
    s_skip = C.skip_when_finished && C.bg_exit &&
             __hip_atomic_load(&C.bg_exit[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  if (s_skip) units = 0;
  for (uint32_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    if (unit < range_units) {
      uint32_t j = 0;
      while (j + 1 < R.n && R.units_prefix[j + 1] <= unit) ++j;
      const uint32_t first = (unit - R.units_prefix[j]) * kUnitPages;
      const uint32_t cand = (t < kUnitPages && first + t < R.np[j]) ? R.p0[j] + first + t : kNone;
      if (!unit_needed(C, cand)) continue;
      if (wait) claim_copy<true, DEEP>(cand, C, nullptr);
      else claim_copy<false, DEEP>(cand, C, nullptr);
      continue;
    }
    if (unit < range_units + list_units) {
      const uint32_t e = start + (unit - range_units) * kVictimUnit + t;
      uint32_t cand = (t < kVictimUnit && e < end) ? vlist[e] : kNone;
      if (cand >= C.n_pages) cand = kNone;
      if (!unit_needed(C, cand)) continue;
      if (wait) claim_copy<true, DEEP>(cand, C, nullptr);
      else claim_copy<false, DEEP>(cand, C, nullptr);
      continue;
    }
    // list overflowed: scan the victim page map, 64 words of 32 pages per unit
    const uint32_t w = (unit - range_units - list_units) * (kCThreads / 4) + t;
    uint32_t bits = (t < kCThreads / 4 && w < V.map_words) ? bytes_to_mask(V.map + 32ull * w) : 0u;
    for (uint32_t b = bits; b; b &= b - 1) {
      const uint32_t p = w * 32 + (__ffs(b) - 1);
      if (p >= C.n_pages || C.state[p] == kDone) bits &= ~(1u << (__ffs(b) - 1));
    }
    while (__syncthreads_or(bits != 0u)) {
      uint32_t cand = kNone;
      if (bits) {
        cand = w * 32 + (__ffs(bits) - 1);
        bits &= bits - 1;
      }
      if (wait) claim_copy<true, DEEP>(cand, C, nullptr);
      else claim_copy<false, DEEP>(cand, C, nullptr);
    }
  }
  // the last block out moves the list cursor past the entries handled here
  if (V.meta && !V.scan_map && !V.bucket) {
    __syncthreads();
    if (t == 0 && atomicAdd(&V.meta[2], 1u) == gridDim.x - 1) {
      V.meta[1] = end;
      V.meta[2] = 0;
    }
  }
}

// Background copy.  Persistent blocks walk the pool in groups of `grab`
// pages (64 KiB per group): block b copies groups b, b + grid, b + 2 grid, ...
// so the whole grid streams through one narrow window of the pool (the
// measured HBM copy rate falls as the active window widens).  Waves 0..7 copy
// batch i (`batch` groups) while wave 8 claims batch i + 1, so the claim
// round trips (image page, page maps, state, compare-and-swap) never stall
// the copy.
constexpr uint32_t kBgMaxBatch = 256;  // candidate pages per batch

__device__ __forceinline__ bool bg_live(uint64_t i, uint32_t batch, uint32_t grab, uint32_t n_pages) {
  return ((i * batch) * gridDim.x + blockIdx.x) * (uint64_t)grab < n_pages;
}

// Claimer wave: claim the candidate pages of batch i into (s_p, s_ip, *s_n).
__device__ __forceinline__ void bg_claim_batch(const CopyArgs &C, uint64_t i, uint32_t batch,
                                               uint32_t grab, uint32_t *s_p, uint32_t *s_ip,
                                               uint32_t *s_n) {
  const uint32_t lane = threadIdx.x - kBgCopyThreads;
  if (lane == 0) *s_n = 0;  // same wave as every append below: ordered
  const uint32_t nb = batch * grab;
  for (uint32_t k = lane; k < nb; k += 64) {
    const uint64_t g = (i * batch + k / grab) * gridDim.x + blockIdx.x;
    const uint64_t p = g * grab + k % grab;
    const bool in = p < C.n_pages;
    const uint64_t q = in ? p : 0;
    // the independent reads first, so their round trips overlap
    const uint32_t ip = C.img_page[q];
    uint32_t st = C.state[q];  // a plain read can only lag: "done" is final
    // Section 4.3: a page already traced as written is copied by the recopy
    // anyway; copying it now would be wasted (a stale 0 only means a
    // redundant copy)
    const uint32_t traced = C.skip_dirty ? (C.skip_dirty[q] | C.skip_victim[q]) : 0u;
    if (!in || ip == kNone || traced) continue;
    if (st == kClaimed) st = ld_relaxed(&C.state[p]);
    if (st != kFree) continue;
    uint32_t exp = kFree;
    if (!cas_u32(&C.state[p], exp, kClaimed)) continue;
    const uint32_t slot = atomicAdd(s_n, 1u);
    s_p[slot] = (uint32_t)p;
    s_ip[slot] = ip;
  }
}

template <bool DEEP>
__global__ void __launch_bounds__(kBgThreads)
    background_kernel(CopyArgs C, uint32_t grab, uint32_t batch) {
  __shared__ uint32_t s_p[2][kBgMaxBatch], s_ip[2][kBgMaxBatch], s_n[2], s_arrive;
  const uint32_t t = threadIdx.x;
  const bool claimer = t >= kBgCopyThreads;
  if (t == 0) s_arrive = 0;
  if (claimer) bg_claim_batch(C, 0, batch, grab, s_p[0], s_ip[0], &s_n[0]);
  __syncthreads();
  uint32_t cur = 0, copied = 0;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  for (uint64_t i = 0; bg_live(i, batch, grab, C.n_pages); ++i) {
    if (claimer) {
      // Section 6: on-demand copies go first: claim nothing new while a
      // launch's pages are moving (bounded: this is a policy, not a
      // correctness wait; the pages already claimed are still copied and
      // published by the copying waves below, which do not wait for this).
      // With hold_ticks the policy lasts that long after the start only:
      // the first launches get the link, then the whole image streams.
      if (C.demand &&
          (C.hold_ticks == 0 || __builtin_amdgcn_s_memrealtime() - t_start < C.hold_ticks)) {
        uint32_t it = 0;
        while (__hip_atomic_load(C.demand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 &&
               ++it < C.pause_limit)
          __builtin_amdgcn_s_sleep(16);
      }
      bg_claim_batch(C, i + 1, batch, grab, s_p[cur ^ 1], s_ip[cur ^ 1], &s_n[cur ^ 1]);
    } else {
      const uint32_t n = s_n[cur];
      for (uint32_t m = 0; m < n; ++m) copy_page<DEEP>(C, s_p[cur][m], s_ip[cur][m], t, kBgCopyThreads);
      // Stores that must land before "done":
      //  - towards the pool (restore): other XCDs read the page right after;
      //  - into a recopy image (skip_dirty set): a pre-copy round on the
      //    application's stream may overwrite a page this copy published,
      //    from another XCD; if this copy's stores could still sit in this
      //    XCD's L2, their write-back could land after the round's fresh
      //    page and leave a stale one in the image.
      // Each wave makes its stores visible at device scope before it
      // arrives, and the publisher releases "done".  Into a copy-on-write
      // image no store needs to land first: the host reads the image after
      // the kernel, nothing else writes a page this copy claimed, and a
      // copy-on-write waiter only needs this block's reads of the pool to
      // have returned, which every wave's stores depended on before it
      // arrived.
      const bool ordered = !C.to_image || C.skip_dirty != nullptr;
      if (ordered && n) __threadfence();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      uint32_t order = 0;
      if ((t & 63u) == 0) order = atomicAdd(&s_arrive, 1u);
      order = rfl(order);
      if (order == kBgCopyThreads / 64 - 1) {
        for (uint32_t m = t & 63u; m < n; m += 64) {
          if (ordered) st_release(&C.state[s_p[cur][m]], kDone);
          else __hip_atomic_store(&C.state[s_p[cur][m]], kDone, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        }
        if ((t & 63u) == 0) s_arrive = 0;
      }
      copied += n;
    }
    lds_barrier();  // list `cur` is free for the claim after next; s_arrive is 0
    cur ^= 1;
  }
  if (t == 0 && copied) atomicAdd(C.stat, (unsigned long long)copied);
  if (C.bg_exit && t == 0) {
    // every block's pages are claimed and published by now (its own, or by
    // a copy-on-write that claimed them first): the last block out says so
    __threadfence();
    if (atomicAdd(&C.bg_exit[0], 1ull) == gridDim.x - 1)
      __hip_atomic_store(&C.bg_exit[1], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Shared background pass of a copy-on-write and a recopy checkpoint open
// together (Sections 4.2 and 4.3 in one window): the two images hold the same
// bytes for every page not yet written, so one pass reads each pool page once
// and stores it to both, instead of two passes reading the pool twice.  Each
// page is still claimed in each image on its own (C.state: copy-on-write,
// every page; C.state2: recopy, pages not yet traced as written), exactly as
// two separate passes would claim it, so copy-on-write, pre-copy rounds and
// the recopy interleave with it as they do with one pass per image.

// Claimer wave: claim batch i's candidate pages in both images; won bit 0 =
// the copy-on-write image, bit 1 = the recopy image.
__device__ __forceinline__ void bg_claim_pair(const CopyArgs &C, uint64_t i, uint32_t batch,
                                              uint32_t grab, uint32_t *s_p, uint32_t *s_ip,
                                              uint32_t *s_m, uint32_t *s_n, uint32_t &n1,
                                              uint32_t &n2, uint32_t &nr) {
  const uint32_t lane = threadIdx.x - kBgCopyThreads;
  if (lane == 0) *s_n = 0;  // same wave as every append below: ordered
  const uint32_t nb = batch * grab;
  for (uint32_t k = lane; k < nb; k += 64) {
    const uint64_t g = (i * batch + k / grab) * gridDim.x + blockIdx.x;
    const uint64_t p = g * grab + k % grab;
    const bool in = p < C.n_pages;
    const uint64_t q = in ? p : 0;
    // the independent reads first, so their round trips overlap
    const uint32_t ip = C.img_page[q];
    uint32_t st1 = C.state[q], st2 = C.state2[q];  // plain reads only lag: "done" is final
    const uint32_t traced = C.skip_dirty[q] | C.skip_victim[q];
    if (!in || ip == kNone) continue;
    uint32_t won = 0, exp;
    if (st1 == kClaimed) st1 = ld_relaxed(&C.state[p]);
    exp = kFree;
    if (st1 == kFree && cas_u32(&C.state[p], exp, kClaimed)) won |= 1u;
    if (!traced) {
      if (st2 == kClaimed) st2 = ld_relaxed(&C.state2[p]);
      exp = kFree;
      if (st2 == kFree && cas_u32(&C.state2[p], exp, kClaimed)) won |= 2u;
    }
    if (!won) continue;
    n1 += won & 1u;
    n2 += won >> 1;
    ++nr;
    const uint32_t slot = atomicAdd(s_n, 1u);
    s_p[slot] = (uint32_t)p;
    s_ip[slot] = ip;
    s_m[slot] = won;
  }
}

// One page from the pool to one or both images (won: as above, uniform over
// the block), U 16-byte loads in flight per thread, each stored once per image.
template <bool NT, int U>
__device__ __forceinline__ void copy_page_pair_t(const u32x4 *__restrict__ src,
                                                 u32x4 *__restrict__ d1, u32x4 *__restrict__ d2,
                                                 uint64_t n16, uint32_t tid, uint32_t nthreads) {
  const uint64_t T = nthreads;
  uint64_t i = tid;
  for (; i + (U - 1) * T < n16; i += U * T) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = NT ? __builtin_nontemporal_load(src + i + u * T) : src[i + u * T];
    if (d1) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (NT) __builtin_nontemporal_store(v[u], d1 + i + u * T);
        else d1[i + u * T] = v[u];
      }
    }
    if (d2) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (NT) __builtin_nontemporal_store(v[u], d2 + i + u * T);
        else d2[i + u * T] = v[u];
      }
    }
  }
  for (; i < n16; i += T) {
    const u32x4 v = src[i];
    if (d1) d1[i] = v;
    if (d2) d2[i] = v;
  }
}

__device__ __forceinline__ void copy_page_pair(const CopyArgs &C, uint32_t p, uint32_t ip,
                                               uint32_t won, uint32_t tid, uint32_t nthreads) {
  const uint64_t pb = 1ull << C.page_shift;
  const u32x4 *src = reinterpret_cast<const u32x4 *>(C.pool + ((uint64_t)p << C.page_shift));
  u32x4 *d1 = (won & 1u) ? reinterpret_cast<u32x4 *>(C.image + ((uint64_t)ip << C.page_shift))
                         : nullptr;
  u32x4 *d2 = (won & 2u) ? reinterpret_cast<u32x4 *>(C.image2 + ((uint64_t)ip << C.page_shift))
                         : nullptr;
  if (C.nt) copy_page_pair_t<true, 8>(src, d1, d2, pb >> 4, tid, nthreads);
  else copy_page_pair_t<false, 8>(src, d1, d2, pb >> 4, tid, nthreads);
}

// Same shape as background_kernel: waves 0..7 copy batch i while wave 8
// claims batch i + 1.
__global__ void __launch_bounds__(kBgThreads)
    background_pair_kernel(CopyArgs C, uint32_t grab, uint32_t batch) {
  __shared__ uint32_t s_p[2][kBgMaxBatch], s_ip[2][kBgMaxBatch], s_m[2][kBgMaxBatch], s_n[2],
      s_arrive;
  const uint32_t t = threadIdx.x;
  const bool claimer = t >= kBgCopyThreads;
  uint32_t n1 = 0, n2 = 0, nr = 0;  // pages this claimer won, per image, and in either
  if (t == 0) s_arrive = 0;
  if (claimer) bg_claim_pair(C, 0, batch, grab, s_p[0], s_ip[0], s_m[0], &s_n[0], n1, n2, nr);
  __syncthreads();
  uint32_t cur = 0;
  for (uint64_t i = 0; bg_live(i, batch, grab, C.n_pages); ++i) {
    if (claimer) {
      bg_claim_pair(C, i + 1, batch, grab, s_p[cur ^ 1], s_ip[cur ^ 1], s_m[cur ^ 1],
                    &s_n[cur ^ 1], n1, n2, nr);
    } else {
      const uint32_t n = s_n[cur];
      for (uint32_t m = 0; m < n; ++m)
        copy_page_pair(C, s_p[cur][m], s_ip[cur][m], s_m[cur][m], t, kBgCopyThreads);
      // The recopy image's stores must be visible at device scope before its
      // "done" (a pre-copy round may overwrite the page from another XCD
      // right after; see background_kernel), so each wave fences before it
      // arrives and the publisher releases; the copy-on-write image's "done"
      // needs no ordering of stores.
      if (n) __threadfence();
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      uint32_t order = 0;
      if ((t & 63u) == 0) order = atomicAdd(&s_arrive, 1u);
      order = rfl(order);
      if (order == kBgCopyThreads / 64 - 1) {
        for (uint32_t m = t & 63u; m < n; m += 64) {
          const uint32_t won = s_m[cur][m], pg = s_p[cur][m];
          if (won & 1u)
            __hip_atomic_store(&C.state[pg], kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (won & 2u) st_release(&C.state2[pg], kDone);
        }
        if ((t & 63u) == 0) s_arrive = 0;
      }
    }
    lds_barrier();  // list `cur` is free for the claim after next; s_arrive is 0
    cur ^= 1;
  }
  if (claimer) {
    for (uint32_t d = 32; d; d >>= 1) {
      n1 += __shfl_down(n1, d, 64);
      n2 += __shfl_down(n2, d, 64);
      nr += __shfl_down(nr, d, 64);
    }
    if (t == kBgCopyThreads) {
      if (n1) atomicAdd(C.stat, (unsigned long long)n1);
      if (n2) atomicAdd(C.stat2, (unsigned long long)n2);
      if (nr && C.stat_read) atomicAdd(C.stat_read, (unsigned long long)nr);
    }
  }
  if (C.bg_exit && t == 0) {
    // the copy-on-write image's completion, as background_kernel reports it
    __threadfence();
    if (atomicAdd(&C.bg_exit[0], 1ull) == gridDim.x - 1)
      __hip_atomic_store(&C.bg_exit[1], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Set the state of every pool page whose image page lies in a flagged image
// piece (pieces the kernels cannot read, moved by DMA instead); count them.
__global__ void __launch_bounds__(256)
    mark_pieces_kernel(const uint32_t *img_page, uint32_t *state, uint32_t n_pages,
                       uint32_t chunk_pages, const uint8_t *flag, uint32_t value,
                       unsigned long long *count) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  if (p < n_pages) {
    const uint32_t ip = img_page[p];
    if (ip != kNone && flag[ip / chunk_pages]) {
      state[p] = value;
      hit = true;
    }
  }
  const uint64_t m = __ballot(hit);
  if (count && (threadIdx.x & 63u) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

// Pre-copy round of a recopy checkpoint (iterative recopy, Sections 4.3 and
// 7): every listed page (marked dirty so far; its writers have all run) is
// unmarked and copied into the image now; a page written again later is
// marked again and copied at the re-quiesce.  The claims keep the concurrent
// background copy of the same image from landing a stale copy afterwards: a
// free page is claimed and published, a page the background holds is waited
// for and then overwritten, a done page is overwritten.
__global__ void __launch_bounds__(kBgCopyThreads)
    precopy_kernel(CopyArgs C, const uint32_t *list, const unsigned int *count, uint8_t *dirty) {
  __shared__ uint32_t s_own;
  const uint32_t cnt = *count;
  uint32_t nw = 0;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const uint32_t p = list[i];
    const uint32_t ip = p < C.n_pages ? C.img_page[p] : kNone;
    if (ip == kNone) continue;  // the same page for the whole block
    if (threadIdx.x == 0) {
      dirty[p] = 0;
      uint32_t own = 0, st = ld_relaxed(&C.state[p]);
      if (st == kFree) {
        uint32_t exp = kFree;
        if (cas_u32(&C.state[p], exp, kClaimed)) own = 1;
        else st = exp;
      }
      if (!own && st == kClaimed) {
        uint32_t it = 0;
        while (ld_acquire(&C.state[p]) != kDone) {
          __builtin_amdgcn_s_sleep(8);
          if (wait_expired(C, ++it)) break;
        }
      }
      s_own = own;
    }
    __syncthreads();
    copy_page(C, p, ip);
    __syncthreads();  // every wave's copy issued (its loads returned)
    if (threadIdx.x == 0 && s_own)
      __hip_atomic_store(&C.state[p], kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++nw;
    __syncthreads();  // s_own is rewritten for the next page
  }
  if (threadIdx.x == 0 && nw) atomicAdd(C.stat, (unsigned long long)nw);
}

// Staged copy-on-write pages -> their places in the host image (at the end
// of the checkpoint, after every copy that could stage one).
__global__ void __launch_bounds__(kBgCopyThreads) unstage_kernel(CopyArgs C) {
  const unsigned long long head = *C.stage_head;
  const uint64_t n = head < C.stage_cap ? head : C.stage_cap;
  const uint64_t pb = 1ull << C.page_shift;
  for (uint64_t slot = blockIdx.x; slot < n; slot += gridDim.x) {
    const uint32_t p = C.stage_page[slot];
    const uint32_t ip = p < C.n_pages ? C.img_page[p] : kNone;
    if (ip == kNone) continue;
    block_copy16(reinterpret_cast<const uint4 *>(C.stage + slot * pb),
                 reinterpret_cast<uint4 *>(C.image + ((uint64_t)ip << C.page_shift)), pb >> 4,
                 false);
  }
}

// Section 4.2, victim pages by launch.  A validation call numbers its
// launches s0 .. s0 + n - 1; every page it newly marks as a victim is
// appended to the victim list once, and its earliest failing write belongs to
// one of these launches.  The appended pages are sorted into one bucket per
// launch (counting sort: count, exclusive scan, scatter), so that launch's
// copy-on-write copies exactly the victim pages it is the first to write.
// Bucket k's bounds are interleaved: bse[2k] its start, bse[2k + 1] its end
// (during the sort: its count, then its fill pointer).
__global__ void __launch_bounds__(256)
    vb_snap_kernel(const uint32_t *vmeta, uint32_t cap, uint32_t *seg0, uint32_t *bse, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bse[2 * i + 1] = 0;
  if (i == 0) *seg0 = vmeta[0] < cap ? vmeta[0] : cap;
}

constexpr uint32_t kVbLdsBuckets = 8192;  // block histograms in LDS up to this many launches

__device__ __forceinline__ uint32_t vb_bucket_of(const uint32_t *vlist, const uint32_t *victim_first,
                                                 uint32_t e, uint32_t b, uint32_t n_pages,
                                                 uint32_t s0, uint32_t n, uint32_t &p) {
  p = kNone;
  if (e >= b) return n;
  p = vlist[e];
  // a page first marked by an earlier call (a repeated append) has its
  // bucket already
  return p < n_pages ? victim_first[p] - s0 : n;
}

// COUNT: bucket sizes into the ends; otherwise place each page at its
// bucket's fill pointer (the end, advanced from the bucket's start).  With
// few launches each block sums its entries per bucket in LDS first and adds
// one total per bucket it saw; otherwise each wave adds once per distinct
// bucket among its 64 entries (neighbouring entries mostly share one).
template <bool COUNT>
__global__ void __launch_bounds__(256)
    vb_pass_kernel(const uint32_t *vlist, const uint32_t *vmeta, uint32_t cap, const uint32_t *seg0,
                   const uint32_t *victim_first, uint32_t n_pages, uint32_t s0, uint32_t n,
                   uint32_t *bse, uint32_t *bucket, uint32_t bucket_cap) {
  extern __shared__ uint32_t s_hist[];  // n counters when n <= kVbLdsBuckets
  const uint32_t a = *seg0, b = vmeta[0] < cap ? vmeta[0] : cap;
  const uint32_t t = threadIdx.x, stride = gridDim.x * blockDim.x;
  if (n <= kVbLdsBuckets) {
    for (uint32_t k = t; k < n; k += blockDim.x) s_hist[k] = 0;
    __syncthreads();
    for (uint32_t e = a + blockIdx.x * blockDim.x + t; e < b; e += stride) {
      uint32_t p;
      const uint32_t k = vb_bucket_of(vlist, victim_first, e, b, n_pages, s0, n, p);
      if (k < n) atomicAdd(&s_hist[k], 1u);
    }
    __syncthreads();
    for (uint32_t k = t; k < n; k += blockDim.x) {
      const uint32_t c = s_hist[k];
      if (!c) continue;
      const uint32_t base = atomicAdd(&bse[2 * k + 1], c);
      if (!COUNT) s_hist[k] = base;  // this block's slots start here
    }
    if (COUNT) return;
    __syncthreads();
    for (uint32_t e = a + blockIdx.x * blockDim.x + t; e < b; e += stride) {
      uint32_t p;
      const uint32_t k = vb_bucket_of(vlist, victim_first, e, b, n_pages, s0, n, p);
      if (k < n) {
        const uint32_t pos = atomicAdd(&s_hist[k], 1u);
        if (pos < bucket_cap) bucket[pos] = p;
      }
    }
    return;
  }
  const uint32_t lane = t & 63;
  const uint64_t below = (1ull << lane) - 1;
  // wave-uniform loop: every lane takes part in the ballots
  for (uint32_t e0 = a + blockIdx.x * blockDim.x + (t & ~63u); e0 < b; e0 += stride) {
    uint32_t p;
    const uint32_t k = vb_bucket_of(vlist, victim_first, e0 + lane, b, n_pages, s0, n, p);
    uint64_t pending = __ballot(k < n);
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const uint32_t lk = __shfl(k, leader);
      const uint64_t same = __ballot(k == lk) & pending;
      uint32_t base = 0;
      if ((int)lane == leader) base = atomicAdd(&bse[2 * lk + 1], (uint32_t)__popcll(same));
      base = __shfl(base, leader);
      if (!COUNT && ((same >> lane) & 1)) {
        const uint32_t pos = base + (uint32_t)__popcll(same & below);
        if (pos < bucket_cap) bucket[pos] = p;
      }
      pending &= ~same;
    }
  }
}

// One workgroup: start[k] = *cursor + (sizes of buckets before k), end[k] =
// start[k] (the scatter's fill pointer); the cursor moves past them all.
__global__ void __launch_bounds__(1024) vb_scan_kernel(uint32_t *bse, uint32_t n, uint32_t *cursor) {
  __shared__ uint32_t s_part[1024];
  const uint32_t t = threadIdx.x, per = (n + 1023) / 1024;
  const uint32_t k0 = t * per, k1 = k0 + per < n ? k0 + per : n;
  uint32_t sum = 0;
  for (uint32_t k = k0; k < k1; ++k) sum += bse[2 * k + 1];
  s_part[t] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {  // inclusive scan of the parts
    const uint32_t v = t >= off ? s_part[t - off] : 0u;
    __syncthreads();
    s_part[t] += v;
    __syncthreads();
  }
  const uint32_t base = *cursor;
  uint32_t run = base + s_part[t] - sum;
  for (uint32_t k = k0; k < k1; ++k) {
    const uint32_t c = bse[2 * k + 1];
    bse[2 * k] = run;
    bse[2 * k + 1] = run;
    run += c;
  }
  __syncthreads();
  if (t == 1023) *cursor = base + s_part[1023];
}

// Section 4.3: (dirty | victim) page maps -> page list, wave64 prefix-sum compaction.
__global__ void __launch_bounds__(256)
    pagelist_kernel(const uint8_t *a, const uint8_t *b, const uint32_t *exclude, uint32_t nwords,
                    uint32_t n_pages, uint32_t *list, unsigned int *count) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t bits = 0;
  if (w < nwords) {
    bits = bytes_to_mask(a + 32ull * w) | (b ? bytes_to_mask(b + 32ull * w) : 0u);
    if (exclude) bits &= ~exclude[w];
    const uint64_t last = (uint64_t)w * 32 + 32;
    if (last > n_pages) bits &= (n_pages - w * 32 >= 32) ? ~0u : ((1u << (n_pages - w * 32)) - 1u);
  }
  const uint32_t c = __popc(bits);
  uint32_t incl = c;
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t x = __shfl_up(incl, d, 64);
    if (lane >= d) incl += x;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (lane == 0 && total) base = atomicAdd(count, total);
  base = __shfl(base, 0, 64);
  uint32_t pos = base + incl - c;
  while (bits) {
    const uint32_t bit = __ffs(bits) - 1;
    list[pos++] = w * 32 + bit;
    bits &= bits - 1;
  }
}

// Final pages of a pre-copy round (see launch_finallist): one 32-page word
// per thread, listed in word order like pagelist_kernel.
__global__ void __launch_bounds__(256)
    finallist_kernel(const uint8_t *dirty, uint8_t *victim, const uint32_t *victim_seq,
                     uint32_t thr, const uint32_t *exclude, uint32_t nwords, uint32_t n_pages,
                     uint32_t *list, unsigned int *count) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t bits = 0;
  if (w < nwords) {
    uint32_t v = bytes_to_mask(victim + 32ull * w);
    for (uint32_t m = v; m; m &= m - 1) {
      const uint32_t b = __ffs(m) - 1;
      const uint32_t q = victim_seq[32ull * w + b];
      if (q == 0 || q > thr) v &= ~(1u << b);  // a failing write still to come (or unknown)
    }
    bits = (bytes_to_mask(dirty + 32ull * w) | v) & ~exclude[w];
    const uint64_t last = (uint64_t)w * 32 + 32;
    if (last > n_pages) bits &= (n_pages - w * 32 >= 32) ? ~0u : ((1u << (n_pages - w * 32)) - 1u);
    for (uint32_t m = v & bits; m; m &= m - 1) victim[32ull * w + __ffs(m) - 1] = 0;
  }
  const uint32_t c = __popc(bits);
  uint32_t incl = c;
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t x = __shfl_up(incl, d, 64);
    if (lane >= d) incl += x;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (lane == 0 && total) base = atomicAdd(count, total);
  base = __shfl(base, 0, 64);
  uint32_t pos = base + incl - c;
  while (bits) {
    const uint32_t bit = __ffs(bits) - 1;
    list[pos++] = w * 32 + bit;
    bits &= bits - 1;
  }
}

// Copy the listed pages (no claims: the application is quiesced).
__global__ void __launch_bounds__(kBgCopyThreads)
    gather_pages_kernel(CopyArgs C, const uint32_t *list, const unsigned int *count) {
  const uint32_t cnt = *count;
  uint32_t nw = 0;
  // the next page's list entry and image page are read before this page's copy
  uint32_t p = blockIdx.x < cnt ? list[blockIdx.x] : kNone;
  uint32_t ip = p < C.n_pages ? C.img_page[p] : kNone;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const uint32_t pn = i + gridDim.x < cnt ? list[i + gridDim.x] : kNone;
    const uint32_t ipn = pn < C.n_pages ? C.img_page[pn] : kNone;
    if (ip != kNone) {
      copy_page(C, p, ip);
      ++nw;
    }
    p = pn;
    ip = ipn;
  }
  if (threadIdx.x == 0 && nw) atomicAdd(C.stat, (unsigned long long)nw);
}

// Section 6: bring in every not-yet-present page (inside a buffer) that the
// launch's records touch, before the launch runs.
// A persistent grid of at most one block per CU walks the records in chunks:
// its blocks may wait (for pages another block or the host is bringing in),
// and waiting blocks must never fill the GPU, or the kernel that publishes
// those pages could find no room to run.
constexpr uint32_t kDemandPerThread = 4;
template <bool DEEP>
__global__ void __launch_bounds__(kCThreads)
    demand_kernel(CopyArgs C, const uint64_t *rec, uint64_t n, uint64_t pool_base,
                  unsigned long long *faulted) {
  const uint64_t per = (uint64_t)kCThreads * kDemandPerThread;
  const uint64_t nchunks = (n + per - 1) / per;
  const uint64_t pool_bytes = (uint64_t)C.n_pages << C.page_shift;
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    for (uint32_t u = 0; u < kDemandPerThread; ++u) {
      const uint64_t i = ch * per + (uint64_t)u * kCThreads + threadIdx.x;
      uint32_t cand = kNone;
      if (i < n) {
        const uint64_t off = (rec[i] & ~7ull) - pool_base;
        if (off < pool_bytes) {
          const uint32_t p = (uint32_t)(off >> C.page_shift);
          if (C.img_page[p] != kNone && C.state[p] != kDone) cand = p;
        }
      }
      claim_copy<true, DEEP>(cand, C, faulted);
    }
  }
}

__global__ void states_to_bits_kernel(const uint32_t *state, uint32_t n_pages, uint32_t *bits) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if ((uint64_t)w * 32 >= n_pages) return;
  uint32_t v = 0;
  for (uint32_t b = 0; b < 32; ++b) {
    const uint64_t p = (uint64_t)w * 32 + b;
    if (p < n_pages && state[p] == kDone) v |= 1u << b;
  }
  bits[w] = v;
}

__global__ void bytes_to_bits_kernel(const uint8_t *bytes, uint32_t nwords, uint32_t *bits) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nwords) bits[w] = bytes_to_mask(bytes + 32ull * w);
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n, unsigned long long v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ============================================================ twin kernel
// Section 4.1, the instrumented twin of an application kernel: the kernel's
// own global accesses are checked in place against the launch's speculated
// intervals (wave-uniform; in registers for up to 8 intervals).  A failed
// check is reported (unordered: one reservation per wave and check); with
// tracking, a validated write marks its page dirty and a failing write
// inside a buffer marks its page a victim (Section 4.3).  The access itself
// is made either way, as the paper's instrumented kernel does: what to do
// about a failure is the caller's protocol.
template <int NIV>
__device__ __forceinline__ uint32_t twin_classify(const IvRegs &R, const DevSpec &S, uint64_t a,
                                                  uint32_t w) {
  if constexpr (NIV >= 0) return classify_n<NIV>(R, a, w);
  else return classify_lds(S, S.niv, a, w);
}

__device__ __forceinline__ void twin_report(const TwinArgs &A, bool bad, uint64_t i, uint64_t a,
                                            uint32_t w, uint32_t reason) {
  const uint64_t m = __ballot(bad);
  if (!m) return;
  const uint32_t lane = threadIdx.x & 63u, lead = (uint32_t)__ffsll((unsigned long long)m) - 1u;
  unsigned long long base = 0;
  if (lane == lead) {
    base = atomicAdd(A.count, (unsigned long long)__popcll(m));
    if (A.overflow && base + (unsigned long long)__popcll(m) > A.cap) atomicOr(A.overflow, 1u);
  }
  base = __shfl(base, (int)lead, 64);
  if (!bad) return;
  const unsigned long long pos = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
  if (pos >= A.cap) return;
  const uint64_t off = a - A.pool_base;
  phos_violation v;
  v.index = i;
  v.addr = a;
  v.launch_id = A.launch_id;
  v.is_write = (uint8_t)w;
  v.reason = (uint8_t)reason;
  v._p = 0;
  v.victim = (int32_t)(off < A.pool_bytes ? A.page_buf[off >> A.page_shift] : kNone);
  v._q = 0;
  A.out[pos] = v;
}

// Every lane of the wave calls this (act: the lane has an element).
__device__ __forceinline__ void twin_track(const TwinArgs &A, bool act, uint64_t a, uint32_t reason) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t off = a - A.pool_base;
  const bool in = act && off < A.pool_bytes;
  const uint32_t page = in ? (uint32_t)(off >> A.page_shift) : kNone;
  // validated writes: one store per run of lanes on the same page
  const uint32_t dp = reason == 0 ? page : kNone;
  const uint32_t prev = __shfl_up(dp, 1, 64);
  if (dp != kNone && (lane == 0 || prev != dp)) A.dirty[dp] = 1;
  if (reason != 0 && in && A.page_buf[page] != kNone) {
    atomicMax(&A.victim_seq[page], A.seq);
    if (A.victim[page] == 0) {
      A.victim[page] = 1;  // newly marked (a stale read only adds a duplicate)
      const uint32_t k = atomicAdd(&A.vmeta[0], 1u);
      if (k < A.vlist_cap) A.vlist[k] = page;
      else A.vmeta[3] = 1;
    }
  }
}

// Section 4.2 with the validator inside the kernel: the write has already
// been made when its check fails, so if it lands on a page that the open
// copy-on-write checkpoint has not copied yet, that image can no longer be
// the state at t1 (the caller must fall back to a stop-the-world copy).
__device__ __forceinline__ void twin_misspec(const TwinArgs &A, bool bad_write, uint64_t a) {
  const uint64_t off = a - A.pool_base;
  if (!bad_write || off >= A.pool_bytes) return;
  const uint32_t page = (uint32_t)(off >> A.page_shift);
  if (A.page_buf[page] != kNone && ld_relaxed(const_cast<uint32_t *>(&A.cow_state[page])) != kDone)
    atomicOr(A.misspec, 1u);
}

// Each thread takes kTwinU elements per pass (stride: the grid): all their
// loads are issued first, then the stores, then the checks, so a wave keeps
// kTwinU elements' loads in flight and the checks' ALU work overlaps the
// memory traffic of other waves instead of adding to it.
constexpr int kTwinU = 4;

template <bool CHECK, int NIV>
__global__ void __launch_bounds__(256) twin_kernel(TwinArgs A, DevSpec S) {
  IvRegs R;
#pragma unroll
  for (int j = 0; j < (NIV > 0 ? NIV : 0); ++j) {
    R.lo[j] = S.iv[j].lo;
    R.hi8[j] = S.iv[j].lo == ~0ull ? 0ull : S.iv[j].lo + S.iv[j].span;
    R.mode[j] = S.iv[j].mode;
  }
  const bool rd = CHECK && (A.flags & PHOS_V_READS), wr = CHECK && (A.flags & PHOS_V_WRITES);
  const bool tr = CHECK && (A.flags & PHOS_V_TRACK);
  const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
  // lanes leave the loop in lane order (i0 grows with the lane), so the
  // lanes still in it are a prefix of the wave
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < A.n; i0 += kTwinU * T) {
    bool act[kTwinU];
    int64_t j[kTwinU];
    uint64_t xv[kTwinU], yv[kTwinU];
#pragma unroll
    for (int k = 0; k < kTwinU; ++k) {
      act[k] = i0 + k * T < A.n;
      j[k] = act[k] ? (A.idx ? A.idx[i0 + k * T] : (int64_t)(i0 + k * T)) : 0;
    }
#pragma unroll
    for (int k = 0; k < kTwinU; ++k) {
      xv[k] = act[k] ? A.x[i0 + k * T] : 0;
      yv[k] = act[k] ? A.y[j[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < kTwinU; ++k)
      if (act[k]) A.y[j[k]] = 3 * yv[k] + xv[k];
    if (CHECK) {
#pragma unroll
      for (int k = 0; k < kTwinU; ++k) {
        const uint64_t i = i0 + k * T;
        const uint64_t xa = (uint64_t)(A.x + i), ya = (uint64_t)(A.y + j[k]);
        if (rd) {
          const uint32_t r0 = twin_classify<NIV>(R, S, xa, 0);
          twin_report(A, act[k] && r0 != 0, i, xa, 0, r0);
          if (A.idx) {
            const uint64_t ia = (uint64_t)(A.idx + i);
            const uint32_t r1 = twin_classify<NIV>(R, S, ia, 0);
            twin_report(A, act[k] && r1 != 0, i, ia, 0, r1);
          }
          const uint32_t r2 = twin_classify<NIV>(R, S, ya, 0);
          twin_report(A, act[k] && r2 != 0, i, ya, 0, r2);
        }
        if (wr || tr) {
          const uint32_t r3 = twin_classify<NIV>(R, S, ya, 1);
          if (wr) twin_report(A, act[k] && r3 != 0, i, ya, 1, r3);
          if (tr) twin_track(A, act[k], ya, r3);
          if (A.cow_state) twin_misspec(A, act[k] && r3 != 0, ya);
        }
      }
    }
  }
}

// ============================================================ batched copy
// Copy bytes [b0, b1) of the concatenated segment stream.
__device__ void copy_stream_range(const BatchQ &Q, uint64_t nseg, uint64_t b0, uint64_t b1) {
  __shared__ uint32_t s_seg;
  if (threadIdx.x == 0) {
    uint64_t lo = 0, hi = nseg;  // last segment with prefix <= b0
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (Q.byte_prefix[mid] <= b0) lo = mid; else hi = mid;
    }
    s_seg = (uint32_t)lo;
  }
  __syncthreads();
  uint64_t s = s_seg;
  __syncthreads();
  uint64_t pos = b0;
  while (pos < b1 && s < nseg) {
    const uint64_t seg_lo = Q.byte_prefix[s], seg_hi = Q.byte_prefix[s + 1];
    const uint64_t lo = pos > seg_lo ? pos : seg_lo;
    const uint64_t hi = b1 < seg_hi ? b1 : seg_hi;
    if (hi > lo) {
      const phos_copy_seg g = Q.segs[s];
      block_copy16(reinterpret_cast<const uint4 *>(g.src + (lo - seg_lo)),
                   reinterpret_cast<uint4 *>(g.dst + (lo - seg_lo)), (hi - lo) >> 4);
      if (threadIdx.x == 0 && Q.done) {
        const unsigned long long old = atomicAdd(&Q.done[g.req], (unsigned long long)(hi - lo));
        // the request's last piece: stamp its completion on the GPU wall clock
        if (Q.req_total && old + (hi - lo) == Q.req_total[g.req])
          Q.req_time[g.req] = __builtin_amdgcn_s_memrealtime();
      }
      pos = hi;
    }
    ++s;
  }
}

// Segments handed over in device memory: one workgroup checks them and
// writes the byte stream's header and exclusive prefix, then resets the chunk
// cursor.  A segment that is not 16-byte aligned or has a NULL address makes
// the whole call copy nothing (total 0) and raises the bad-segment word.
__global__ void __launch_bounds__(1024)
    segs_prefix_kernel(const phos_copy_seg *segs, uint64_t nseg, unsigned long long *hdr,
                       unsigned long long *prefix, unsigned long long *cursor, uint32_t *bad) {
  __shared__ unsigned long long s[1024];
  __shared__ uint32_t s_bad;
  const uint32_t t = threadIdx.x;
  if (t == 0) s_bad = 0;
  __syncthreads();
  unsigned long long carry = 0;
  for (uint64_t b0 = 0; b0 < nseg; b0 += 1024) {
    const uint64_t i = b0 + t;
    unsigned long long v = 0;
    if (i < nseg) {
      const phos_copy_seg g = segs[i];
      v = g.bytes;
      if (((g.src | g.dst | g.bytes) & 15u) || (g.bytes && (!g.src || !g.dst))) s_bad = 1;
    }
    s[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      const unsigned long long x = t >= d ? s[t - d] : 0ull;
      __syncthreads();
      s[t] += x;
      __syncthreads();
    }
    if (i < nseg) prefix[i] = carry + s[t] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (t == 0) {
    prefix[nseg] = carry;
    hdr[0] = nseg;
    hdr[1] = s_bad ? 0ull : carry;
    hdr[2] = 0;
    hdr[3] = 0;
    *cursor = 0;
    if (s_bad && bad) atomicOr(bad, 1u);
  }
}

// Reset the chunk cursor and the per-request completed-byte counters.
__global__ void batch_reset_kernel(const unsigned long long *hdr, unsigned long long *cursor,
                                   unsigned long long *done, unsigned long long *req_time) {
  const uint64_t nreq = hdr[2];
  for (uint64_t i = threadIdx.x; i < nreq; i += blockDim.x) {
    done[i] = 0;
    if (req_time) req_time[i + 1] = 0;
  }
  if (threadIdx.x == 0) {
    *cursor = 0;
    if (req_time) req_time[0] = __builtin_amdgcn_s_memrealtime();  // start stamp
  }
}

// Persistent: resident blocks claim chunk_bytes pieces of the stream in order.
__global__ void batch_copy_kernel(BatchQ Q) {
  __shared__ unsigned long long s_chunk;
  const uint64_t nseg = Q.hdr[0], total = Q.hdr[1];
  const uint64_t nchunks = (total + Q.chunk_bytes - 1) / Q.chunk_bytes;
  for (;;) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(Q.cursor, 1ull);
    __syncthreads();
    const uint64_t c = s_chunk;
    __syncthreads();
    if (c >= nchunks) break;
    const uint64_t b0 = c * Q.chunk_bytes;
    copy_stream_range(Q, nseg, b0, b0 + Q.chunk_bytes < total ? b0 + Q.chunk_bytes : total);
  }
}

// Plain: one block per chunk, no persistence.
__global__ void plain_copy_kernel(BatchQ Q) {
  const uint64_t nseg = Q.hdr[0], total = Q.hdr[1];
  const uint64_t b0 = (uint64_t)blockIdx.x * Q.chunk_bytes;
  if (b0 >= total) return;
  copy_stream_range(Q, nseg, b0, b0 + Q.chunk_bytes < total ? b0 + Q.chunk_bytes : total);
}

__global__ void clock_kernel(unsigned long long *out) { *out = __builtin_amdgcn_s_memrealtime(); }

unsigned grid_cap(uint64_t n, unsigned block, unsigned cap) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ============================================================ launchers
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_cap(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_cap(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_validate(const VArgs &a, const DevSpec *single, bool track, hipStream_t s) {
  if (!a.ntiles) return hipSuccess;
  const DevSpec &sp = *single;
  const dim3 g(a.ntiles), b(kVThreads);
  if (a.launches) {
    if (track) hipLaunchKernelGGL((validate_kernel<true, true>), g, b, 0, s, a, sp);
    else hipLaunchKernelGGL((validate_kernel<true, false>), g, b, 0, s, a, sp);
  } else {
    if (track) hipLaunchKernelGGL((validate_kernel<false, true>), g, b, 0, s, a, sp);
    else hipLaunchKernelGGL((validate_kernel<false, false>), g, b, 0, s, a, sp);
  }
  return hipGetLastError();
}

hipError_t launch_vscan(unsigned long long *seg_sum, uint32_t nseg, unsigned long long *seg_prefix,
                        uint64_t *n_out, unsigned long long *cursor, uint64_t cap,
                        uint32_t *overflow, hipStream_t s) {
  hipLaunchKernelGGL(vscan_kernel, dim3(1), dim3(1024), 0, s, seg_sum, nseg, seg_prefix, n_out,
                     cursor, cap, overflow);
  return hipGetLastError();
}

hipError_t launch_vfinish(const uint32_t *tile_count, const unsigned long long *tile_off,
                          uint32_t ntiles, const phos_violation *scratch, uint64_t scratch_cap,
                          phos_violation *out, uint64_t cap, uint64_t *n_out,
                          unsigned long long *cursor, unsigned long long *seg_sum,
                          uint32_t *overflow, hipStream_t s) {
  if (ntiles > kFuseTiles) return hipErrorInvalidValue;
  // a wave per tile, up to 64 workgroups of 16 waves
  uint32_t blocks = (ntiles + 15u) / 16u;
  blocks = blocks < 1u ? 1u : (blocks > 64u ? 64u : blocks);
  hipLaunchKernelGGL(vfinish_kernel, dim3(blocks), dim3(1024), 0, s, tile_count, tile_off, ntiles,
                     scratch, scratch_cap, out, cap, n_out, cursor, seg_sum, overflow);
  return hipGetLastError();
}

hipError_t launch_vscatter(const uint32_t *tile_count, const unsigned long long *tile_off,
                           uint32_t ntiles, const unsigned long long *seg_prefix,
                           const phos_violation *scratch, uint64_t scratch_cap,
                           phos_violation *out, uint64_t cap, hipStream_t s) {
  if (!ntiles) return hipSuccess;
  hipLaunchKernelGGL(vscatter_kernel, dim3((ntiles + kScatTiles - 1) / kScatTiles), dim3(256), 0, s,
                     tile_count, tile_off, ntiles, seg_prefix, scratch, scratch_cap, out, cap);
  return hipGetLastError();
}

hipError_t launch_cow(const CopyArgs &c, const PageRanges &r, const VictimList &v, bool wait,
                      uint32_t max_grid, uint32_t victim_blocks, hipStream_t s) {
  // the victim entries are only known on the device: extra blocks stride
  // over them (the whole grid when the caller knows some may be new)
  uint32_t units = r.units_prefix[r.n] + (v.meta ? victim_blocks : 0);
  if (!units) return hipSuccess;
  const dim3 g(units < max_grid ? units : max_grid);
  if (c.deep)
    hipLaunchKernelGGL(cow_kernel<true>, g, dim3(kCThreads), 0, s, c, r, v, wait ? 1u : 0u);
  else
    hipLaunchKernelGGL(cow_kernel<false>, g, dim3(kCThreads), 0, s, c, r, v, wait ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_background(const CopyArgs &c, uint32_t grab, uint32_t batch, uint32_t grid,
                             hipStream_t s) {
  if (!c.n_pages || !grid) return hipSuccess;
  if (grab == 0 || grab > kBgMaxBatch) return hipErrorInvalidValue;
  if (batch == 0) batch = 1;
  if (batch * grab > kBgMaxBatch) batch = kBgMaxBatch / grab;
  if (c.deep)
    hipLaunchKernelGGL(background_kernel<true>, dim3(grid), dim3(kBgThreads), 0, s, c, grab, batch);
  else
    hipLaunchKernelGGL(background_kernel<false>, dim3(grid), dim3(kBgThreads), 0, s, c, grab, batch);
  return hipGetLastError();
}

hipError_t launch_background_pair(const CopyArgs &c, uint32_t grab, uint32_t batch, uint32_t grid,
                                  hipStream_t s) {
  if (!c.n_pages || !grid) return hipSuccess;
  if (grab == 0 || grab > kBgMaxBatch || !c.image || !c.image2 || !c.state || !c.state2 ||
      !c.stat || !c.stat2 || !c.skip_dirty || !c.skip_victim || !c.to_image || c.image_chunks)
    return hipErrorInvalidValue;
  if (batch == 0) batch = 1;
  if (batch * grab > kBgMaxBatch) batch = kBgMaxBatch / grab;
  hipLaunchKernelGGL(background_pair_kernel, dim3(grid), dim3(kBgThreads), 0, s, c, grab, batch);
  return hipGetLastError();
}

hipError_t launch_mark_pieces(const uint32_t *img_page, uint32_t *state, uint32_t n_pages,
                              uint32_t chunk_pages, const uint8_t *flag, uint32_t value,
                              unsigned long long *count, hipStream_t s) {
  if (!n_pages) return hipSuccess;
  hipLaunchKernelGGL(mark_pieces_kernel, dim3((n_pages + 255) / 256), dim3(256), 0, s, img_page,
                     state, n_pages, chunk_pages, flag, value, count);
  return hipGetLastError();
}

hipError_t launch_finallist(const uint8_t *dirty, uint8_t *victim, const uint32_t *victim_seq,
                            uint32_t thr, const uint32_t *exclude, uint32_t nwords,
                            uint32_t n_pages, uint32_t *list, unsigned int *count, hipStream_t s) {
  if (!nwords) return hipSuccess;
  hipLaunchKernelGGL(finallist_kernel, dim3((nwords + 255) / 256), dim3(256), 0, s, dirty, victim,
                     victim_seq, thr, exclude, nwords, n_pages, list, count);
  return hipGetLastError();
}

hipError_t launch_vb_snap(const uint32_t *vmeta, uint32_t cap, uint32_t *seg0, uint32_t *bse,
                          uint32_t n, hipStream_t s) {
  const uint32_t blocks = n ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(vb_snap_kernel, dim3(blocks), dim3(256), 0, s, vmeta, cap, seg0, bse, n);
  return hipGetLastError();
}

hipError_t launch_vb_build(const uint32_t *vlist, const uint32_t *vmeta, uint32_t cap,
                           const uint32_t *seg0, const uint32_t *victim_first, uint32_t n_pages,
                           uint32_t s0, uint32_t n, uint32_t *bse, uint32_t *cursor,
                           uint32_t *bucket, uint32_t bucket_cap, hipStream_t s) {
  if (!n) return hipSuccess;
  const dim3 grid(256), block(256);
  const size_t lds = n <= kVbLdsBuckets ? 4ull * n : 0;
  hipLaunchKernelGGL(vb_pass_kernel<true>, grid, block, lds, s, vlist, vmeta, cap, seg0,
                     victim_first, n_pages, s0, n, bse, bucket, bucket_cap);
  hipLaunchKernelGGL(vb_scan_kernel, dim3(1), dim3(1024), 0, s, bse, n, cursor);
  hipLaunchKernelGGL(vb_pass_kernel<false>, grid, block, lds, s, vlist, vmeta, cap, seg0,
                     victim_first, n_pages, s0, n, bse, bucket, bucket_cap);
  return hipGetLastError();
}

hipError_t launch_pagelist(const uint8_t *a, const uint8_t *b, uint32_t nwords, uint32_t n_pages,
                           uint32_t *list, unsigned int *count, hipStream_t s,
                           const uint32_t *exclude) {
  if (!nwords) return hipSuccess;
  hipLaunchKernelGGL(pagelist_kernel, dim3((nwords + 255) / 256), dim3(256), 0, s, a, b, exclude,
                     nwords, n_pages, list, count);
  return hipGetLastError();
}

hipError_t launch_unstage(const CopyArgs &c, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(unstage_kernel, dim3(grid), dim3(kBgCopyThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_precopy(const CopyArgs &c, const uint32_t *list, const unsigned int *count,
                          uint8_t *dirty, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(precopy_kernel, dim3(grid), dim3(kBgCopyThreads), 0, s, c, list, count, dirty);
  return hipGetLastError();
}

hipError_t launch_gather_pages(const CopyArgs &c, const uint32_t *list, const unsigned int *count,
                               uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(gather_pages_kernel, dim3(grid), dim3(kBgCopyThreads), 0, s, c, list, count);
  return hipGetLastError();
}

hipError_t launch_demand(const CopyArgs &c, const uint64_t *rec, uint64_t n, uint64_t pool_base,
                         unsigned long long *faulted, uint32_t max_grid, hipStream_t s) {
  if (!n) return hipSuccess;
  const uint64_t per = (uint64_t)kCThreads * kDemandPerThread;
  const uint64_t chunks = (n + per - 1) / per;
  const uint32_t grid = (uint32_t)(chunks < max_grid ? chunks : (max_grid ? max_grid : 1));
  if (c.deep)
    hipLaunchKernelGGL(demand_kernel<true>, dim3(grid), dim3(kCThreads), 0, s, c, rec, n, pool_base,
                       faulted);
  else
    hipLaunchKernelGGL(demand_kernel<false>, dim3(grid), dim3(kCThreads), 0, s, c, rec, n, pool_base,
                       faulted);
  return hipGetLastError();
}

hipError_t launch_states_to_bits(const uint32_t *state, uint32_t n_pages, uint32_t *bits,
                                 hipStream_t s) {
  const uint32_t nw = (n_pages + 31) / 32;
  if (!nw) return hipSuccess;
  hipLaunchKernelGGL(states_to_bits_kernel, dim3((nw + 255) / 256), dim3(256), 0, s, state, n_pages,
                     bits);
  return hipGetLastError();
}

hipError_t launch_bytes_to_bits(const uint8_t *bytes, uint32_t nwords, uint32_t *bits,
                                hipStream_t s) {
  if (!nwords) return hipSuccess;
  hipLaunchKernelGGL(bytes_to_bits_kernel, dim3((nwords + 255) / 256), dim3(256), 0, s, bytes,
                     nwords, bits);
  return hipGetLastError();
}

hipError_t launch_read_clock(unsigned long long *out, hipStream_t s) {
  hipLaunchKernelGGL(clock_kernel, dim3(1), dim3(1), 0, s, out);
  return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchQ &q, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, s, q.hdr, q.cursor, q.done,
                     q.req_time ? q.req_time - 1 : nullptr);
  return hipGetLastError();
}

hipError_t launch_segs_prefix(const phos_copy_seg *segs, uint64_t nseg, unsigned long long *hdr,
                              unsigned long long *prefix, unsigned long long *cursor,
                              uint32_t *bad, hipStream_t s) {
  hipLaunchKernelGGL(segs_prefix_kernel, dim3(1), dim3(1024), 0, s, segs, nseg, hdr, prefix, cursor,
                     bad);
  return hipGetLastError();
}

hipError_t launch_batch_copy(const BatchQ &q, uint32_t grid, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(batch_copy_kernel, dim3(grid), dim3(threads), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_plain_copy(const BatchQ &q, uint64_t nchunks, uint32_t threads, hipStream_t s) {
  if (!nchunks) return hipSuccess;
  hipLaunchKernelGGL(plain_copy_kernel, dim3((unsigned)nchunks), dim3(threads), 0, s, q);
  return hipGetLastError();
}

// One resident round of blocks: each block's share of the elements is fixed
// (grid stride), so blocks beyond what fits at once would run as a second,
// partial round.  Measured on 3 x 2 GiB arrays: 4 blocks (16 waves) per CU
// keep enough loads in flight without crowding HBM; the tracking twin does
// more work per element between its loads and is fastest with 5.
template <bool C, int N>
static hipError_t launch_twin_t(const TwinArgs &a, const DevSpec &spec, uint64_t blocks,
                                uint32_t n_cu, hipStream_t s) {
  static int per_cu = 0;  // per kernel instance; a racing first call computes the same value
  if (!per_cu) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, twin_kernel<C, N>, 256, 0) != hipSuccess ||
        v < 1)
      v = 1;
    per_cu = v;
  }
  const uint32_t want = env_u32("PHOS_TWIN_BLOCKS_PER_CU", (a.flags & PHOS_V_TRACK) ? 5 : 4);
  const uint64_t cap = (uint64_t)(want && (int)want < per_cu ? (int)want : per_cu) * (n_cu ? n_cu : 1);
  const uint32_t grid = (uint32_t)(blocks < cap ? (blocks ? blocks : 1) : cap);
  hipLaunchKernelGGL((twin_kernel<C, N>), dim3(grid), dim3(256), 0, s, a, spec);
  return hipGetLastError();
}

hipError_t launch_twin(const TwinArgs &a, const DevSpec &spec, uint64_t blocks, uint32_t n_cu,
                       hipStream_t s) {
  if (!a.n) return hipSuccess;
  if (!a.flags) return launch_twin_t<false, 0>(a, spec, blocks, n_cu, s);
  switch (spec.niv) {
    case 0: return launch_twin_t<true, 0>(a, spec, blocks, n_cu, s);
    case 1: return launch_twin_t<true, 1>(a, spec, blocks, n_cu, s);
    case 2: return launch_twin_t<true, 2>(a, spec, blocks, n_cu, s);
    case 3: return launch_twin_t<true, 3>(a, spec, blocks, n_cu, s);
    case 4: return launch_twin_t<true, 4>(a, spec, blocks, n_cu, s);
    case 5: return launch_twin_t<true, 5>(a, spec, blocks, n_cu, s);
    case 6: return launch_twin_t<true, 6>(a, spec, blocks, n_cu, s);
    case 7: return launch_twin_t<true, 7>(a, spec, blocks, n_cu, s);
    case 8: return launch_twin_t<true, 8>(a, spec, blocks, n_cu, s);
    default: return launch_twin_t<true, -1>(a, spec, blocks, n_cu, s);
  }
}

}  // namespace phos

// ============================================== fixed validation workspace
// The workspace of phos_validate_noalloc (layout in internal.h): every GPU
// the library runs on holds its own copy until the process ends.  In host
// code the array's name denotes a host-side stand-in, not device memory, so
// its only host use is the address lookup below; kernels get the looked-up
// address.
static __device__ __align__(256) uint8_t scratch[phos::kNaBytes];

namespace phos {

hipError_t noalloc_workspace(int device, uint8_t **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static uint8_t *addr[kMaxDevices] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<uint8_t *>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace phos
