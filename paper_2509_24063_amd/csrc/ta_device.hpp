// ta_device.hpp -- device-side building blocks shared by the exchange kernels:
// wave64 collectives, a 256-thread block scan, the single-pass decoupled
// look-back prefix used by every device-wide scan, and small search helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ta {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / WAVE;

constexpr uint32_t TAM1_MAGIC = 0x314D4154u;  // "TAM1"
constexpr uint32_t TAD1_MAGIC = 0x31444154u;  // "TAD1"

// bits of the device status word
enum : uint32_t { ERR_INVALID = 1, ERR_CAPACITY = 2, ERR_CORRUPT = 3, ERR_REF = 4, ERR_INTERNAL = 5 };
constexpr uint32_t ANY_ERR = (1u << ERR_INVALID) | (1u << ERR_CAPACITY) | (1u << ERR_CORRUPT) | (1u << ERR_REF) |
                             (1u << ERR_INTERNAL);

__device__ inline void fail(uint32_t* status, uint32_t code) { atomicOr(status, 1u << code); }
__device__ inline uint32_t status_of(const uint32_t* status) {
  return __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int lane_id() { return (int)__lane_id(); }

// Orders the LDS accesses of the lanes of one wave (LDS written by some lanes
// and then read by others).  Wavefront scope: it keeps the compiler from
// moving LDS accesses across it and waits for this wave's LDS operations, but
// not for its global loads and stores, which stay in flight.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The wave's index in its block, as a wave-uniform (scalar) value, so that
// indices derived from it stay in scalar registers and their loads can be
// scalar loads.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)); }

__device__ inline uint64_t lanemask_le(int l) { return l >= 63 ? ~0ull : ((2ull << l) - 1); }
__device__ inline uint64_t lanemask_lt(int l) { return l == 0 ? 0ull : (l >= 64 ? ~0ull : ((1ull << l) - 1)); }

__device__ inline uint64_t wave_incl_scan(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t t = __shfl_up(v, d, WAVE);
    if (l >= d) v += t;
  }
  return v;
}
// Inclusive scan of a 32-bit value over the 64 lanes with DPP row shifts
// (within rows of 16 lanes) and row broadcasts (15 -> rows 1 and 3, then
// 31 -> rows 2 and 3): six adds, no LDS traffic.  All lanes must call it.
__device__ inline uint32_t wave_incl_scan32(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return (uint32_t)x;
}

// The same scan on 64-bit values: each DPP move carries both halves from the
// same source lane, then one 64-bit add.  All lanes must call it.
__device__ inline uint64_t wave_incl_scan64(uint64_t v) {
  auto step = [&](auto dpp) {
    const uint32_t lo = dpp((uint32_t)v), hi = dpp((uint32_t)(v >> 32));
    v += ((uint64_t)hi << 32) | lo;
  };
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true); });
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true); });
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true); });
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true); });
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); });
  step([](uint32_t x) { return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); });
  return v;
}
__device__ inline uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int d = WAVE / 2; d; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}
__device__ inline uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int d = WAVE / 2; d; d >>= 1) v |= __shfl_xor(v, d, WAVE);
  return v;
}
__device__ inline uint64_t wave_xor(uint64_t v) {
#pragma unroll
  for (int d = WAVE / 2; d; d >>= 1) v ^= __shfl_xor(v, d, WAVE);
  return v;
}
__device__ inline uint32_t uniform32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ inline uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive prefix of v over the 256 threads of the block; *total = block sum.
// s_wave: __shared__ uint64_t[WAVES].  Contains two block barriers.
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t* s_wave, uint64_t* total) {
  const uint64_t incl = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) s_wave[wave_id()] = incl;
  __syncthreads();
  uint64_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    const uint64_t x = s_wave[i];
    off += (i < wave_id()) ? x : 0;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back (single-pass chained scan).  Tiles are handed out in
// order through an atomic ticket, so a tile only ever waits for tiles that
// were handed out earlier and are therefore already running; tile 0 never
// waits.  Each tile publishes its aggregate, sums predecessors' values back to
// the nearest inclusive prefix, and publishes its own inclusive prefix.  A
// status word per tile packs a 2-bit flag and a 62-bit value so one 64-bit
// atomic store publishes both.  The flag array and the ticket must be zero
// before the kernel starts; every look-back kernel clears the array and
// ticket that the next one will use (see LookBack::clear_*).
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INCL = 2ull << 62;
constexpr uint64_t LB_VALUE = (1ull << 62) - 1;
constexpr uint32_t LB_SPIN_LIMIT = 1u << 20;

struct LookBack {
  uint64_t* flags;        // per tile status words (zero on entry)
  uint32_t* ticket;       // tile ticket (zero on entry)
  uint64_t* clear_flags;  // array the next look-back kernel uses: zeroed here
  uint32_t* clear_ticket;
  int64_t clear_n;
  uint32_t* status;
};

__device__ inline void lb_clear_next(const LookBack& lb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lb.clear_n; i += stride) lb.clear_flags[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && lb.clear_ticket) *lb.clear_ticket = 0;
}

__device__ inline uint32_t lb_take_ticket(const LookBack& lb, uint32_t* s_ticket) {
  if (threadIdx.x == 0) *s_ticket = atomicAdd(lb.ticket, 1u);
  __syncthreads();
  const uint32_t t = uniform32(*s_ticket);  // the same in every lane: a scalar value
  __syncthreads();
  return t;
}

// The two halves of a tile's part in the look-back, for kernels that do
// other work between them: lb_publish makes the tile's aggregate visible
// (tile 0's is already its inclusive prefix); lb_lookback, called by all 64
// lanes of one wave, sums predecessors back to the nearest inclusive prefix,
// publishes the tile's own and returns its exclusive prefix.  Predecessors
// only need to have published their aggregates.
__device__ inline void lb_publish(const LookBack& lb, uint32_t t, uint64_t agg) {
  __hip_atomic_store(lb.flags + t, (t == 0 ? LB_INCL : LB_AGG) | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t lb_lookback(const LookBack& lb, uint32_t t, uint64_t agg) {
  const int l = lane_id();
  if (t == 0) return 0;
  uint64_t excl = 0;
  int64_t hi = (int64_t)t - 1;
  uint32_t spins = 0;
  for (;;) {
    const int64_t k = hi - l;
    const uint64_t f =
        k >= 0 ? __hip_atomic_load(lb.flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_INCL;
    const uint64_t incl = __ballot((f >> 62) == 2);
    const uint64_t none = __ballot((f >> 62) == 0);
    const int first = incl ? (__ffsll((unsigned long long)incl) - 1) : WAVE;
    const uint64_t need = first >= WAVE - 1 ? ~0ull : ((2ull << first) - 1);
    if (none & need) {
      if (++spins > LB_SPIN_LIMIT) {  // never reached when every tile publishes; keeps the wave finite
        if (l == 0) fail(lb.status, ERR_INTERNAL);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum(l <= first ? (f & LB_VALUE) : 0);
    if (first < WAVE) break;
    hi -= WAVE;
  }
  if (l == 0) __hip_atomic_store(lb.flags + t, LB_INCL | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}
// Both halves at once; called by all 64 lanes of one wave, returns the
// exclusive prefix of tile t.
__device__ inline uint64_t lb_exclusive(const LookBack& lb, uint32_t t, uint64_t agg) {
  if (lane_id() == 0) lb_publish(lb, t, agg);
  return lb_lookback(lb, t, agg);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of n values given by a functor (value(i) for
// i < n, uint64_t).  out[i] = sum of values before i, out[n] = total.  n is
// read from device memory so the launch needs only a host bound.  A tile is
// SCAN_WAVES waves x SCAN_ROUNDS rounds of 64 consecutive items: every load and store
// instruction of a wave touches 64 consecutive items, each round is one wave
// scan, and one look-back per tile joins the tiles.
#ifndef TA_SCAN_ROUNDS
#define TA_SCAN_ROUNDS 8
#endif
#ifndef TA_SCAN_BLOCK
#define TA_SCAN_BLOCK 512
#endif
constexpr int SCAN_ROUNDS = TA_SCAN_ROUNDS;
constexpr int SCAN_BLOCK = TA_SCAN_BLOCK;  // threads of a scan block (a tile is SCAN_BLOCK x rounds items)
constexpr int SCAN_WAVES = SCAN_BLOCK / WAVE;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ROUNDS;
// Rounds per thread of a functor's scan: SCAN_ROUNDS, or the functor's
// static ROUNDS (4, 8 or 16) where measurement favours another tile: larger
// tiles for dense scans over many items (fewer tiles to look back over),
// smaller ones for short scans (more tiles in flight).  Look-back flag
// arrays are sized for the smallest tile.
constexpr int SCAN_ROUNDS_MIN = 4;
constexpr int SCAN_TILE_MIN = SCAN_BLOCK * SCAN_ROUNDS_MIN;
template <class In, class = void>
struct scan_rounds : std::integral_constant<int, SCAN_ROUNDS> {};
template <class In>
struct scan_rounds<In, std::void_t<decltype(In::ROUNDS)>> : std::integral_constant<int, In::ROUNDS> {};
template <class In>
constexpr int scan_tile() {
  static_assert(scan_rounds<In>::value >= SCAN_ROUNDS_MIN, "flag arrays are sized for SCAN_TILE_MIN");
  return SCAN_BLOCK * scan_rounds<In>::value;
}

// A functor gives the value of item i with operator()(i).  It may define
// wave_begin(first, last), called by all 64 lanes of a wave before it reads
// items first..last (consecutive), e.g. to bound a segment search once per
// wave instead of once per item.  A functor whose value takes dependent
// loads may instead define values(wbase, n, v): the values of the wave's
// SCAN_ROUNDS items wbase + 64 r + lane (0 for items >= n), loaded in stages
// (every item's first loads, then every item's second loads, ...), so that
// a wave waits once per stage rather than once per stage and item.  Lanes
// past n may call operator() with index n - 1 (side effects of a functor
// must be idempotent), so that no load sits behind a branch.  A functor may
// also define emit(i, excl, v), called for every item i < n after out[i] is
// stored, with the item's exclusive prefix and value (e.g. to list the items
// of a kind by their rank).
template <class T, class = void>
struct has_wave_begin : std::false_type {};
template <class T, class = void>
struct has_emit : std::false_type {};
template <class T>
struct has_emit<T, std::void_t<decltype(&T::emit)>> : std::true_type {};
template <class T>
struct has_wave_begin<T, std::void_t<decltype(&T::wave_begin)>> : std::true_type {};
template <class T, class = void>
struct has_values : std::false_type {};
template <class T>
struct has_values<T, std::void_t<decltype(&T::template values<SCAN_ROUNDS>)>> : std::true_type {};

template <class In>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan(In in, const int64_t* n_dev, int64_t n_cap, uint64_t* out,
                                                     LookBack lb) {
  __shared__ uint64_t s_wave[SCAN_WAVES];
  __shared__ uint32_t s_ticket;
  __shared__ uint64_t s_prefix;
  constexpr int R = scan_rounds<In>::value;
  constexpr int64_t TILE = (int64_t)SCAN_BLOCK * R;
  lb_clear_next(lb);
  int64_t n = *n_dev;
  if (n > n_cap) {  // more items than the arrays hold: nothing is scanned
    if (blockIdx.x == 0 && threadIdx.x == 0) fail(lb.status, ERR_CAPACITY);
    n = 0;
  }
  if (n <= 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    return;
  }
  const int64_t ntiles = (n + TILE - 1) / TILE;
  // blocks beyond the tile count leave before taking a ticket: each ticket is
  // an atomic on one address, and they serialize
  if ((int64_t)blockIdx.x >= ntiles) return;
  const int l = lane_id(), wv = wave_id();
  for (;;) {
    const uint32_t t = lb_take_ticket(lb, &s_ticket);
    if ((int64_t)t >= ntiles) break;
    const int64_t wbase = (int64_t)t * TILE + (int64_t)wv * (WAVE * R);
    In fn = in;
    if constexpr (has_wave_begin<In>::value) {
      const int64_t last = wbase + WAVE * R - 1 < n ? wbase + WAVE * R - 1 : n - 1;
      fn.wave_begin(wbase < n ? wbase : n - 1, last);
    }
    uint64_t v[R];
    if constexpr (has_values<In>::value) {
      fn.template values<R>(wbase, n, v);
    } else if (wbase + WAVE * R <= n) {  // uniform: every item of the wave exists
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = fn(wbase + r * WAVE + l);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = wbase + r * WAVE + l;
        const uint64_t x = fn(i < n ? i : n - 1);
        v[r] = i < n ? x : 0;
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // every item's loads before the first scan
    uint64_t ex[R];
    uint64_t carry = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t incl = wave_incl_scan64(v[r]);
      ex[r] = carry + incl - v[r];
      carry += readlane64(incl, WAVE - 1);
    }
    if (l == 0) s_wave[wv] = carry;
    __syncthreads();
    uint64_t woff = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_WAVES; ++i) {
      woff += (i < wv) ? s_wave[i] : 0;
      tot += s_wave[i];
    }
    if (threadIdx.x < WAVE) {
      const uint64_t e = lb_exclusive(lb, t, tot);
      if (threadIdx.x == 0) s_prefix = e;
    }
    __syncthreads();
    const uint64_t base = s_prefix + woff;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      if (i < n) {
        out[i] = base + ex[r];
        if constexpr (has_emit<In>::value) fn.emit(i, base + ex[r], v[r]);
      }
    }
    if ((int64_t)t == ntiles - 1 && threadIdx.x == 0) out[n] = s_prefix + tot;
    __syncthreads();
  }
}

// Largest i in [lo, hi) with a[i] <= x (a non-decreasing); lo if none.
template <class T>
__device__ inline int64_t last_le(const T* a, int64_t lo, int64_t hi, T x) {
  int64_t l = lo, h = hi;  // invariant: answer in [l, h)
  while (h - l > 1) {
    const int64_t m = l + (h - l) / 2;
    if (a[m] <= x) l = m;
    else h = m;
  }
  return l;
}

// The same search done by a whole wave: 64 probes per round (each round
// shrinks the range 64-fold), result uniform across the wave.  All 64 lanes
// must call it.
template <class T>
__device__ inline int64_t wave_last_le(const T* a, int64_t lo, int64_t hi, T x) {
  const int l = lane_id();
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + WAVE - 1) / WAVE;
    const int64_t p = lo + (int64_t)l * step;
    const bool ok = p < hi && a[p] <= x;
    const uint64_t m = __ballot(ok);
    const int last = m ? 63 - __clzll((long long)m) : 0;
    lo = lo + (int64_t)last * step;
    hi = (lo + step < hi) ? lo + step : hi;
  }
  return lo;
}

// Same, comparing only the bits of a[] selected by mask (a[] & mask must be
// non-decreasing).
__device__ inline int64_t wave_last_le_masked(const uint64_t* a, int64_t lo, int64_t hi, uint64_t x, uint64_t mask) {
  const int l = lane_id();
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + WAVE - 1) / WAVE;
    const int64_t p = lo + (int64_t)l * step;
    const bool ok = p < hi && (a[p] & mask) <= x;
    const uint64_t m = __ballot(ok);
    const int last = m ? 63 - __clzll((long long)m) : 0;
    lo = lo + (int64_t)last * step;
    hi = (lo + step < hi) ? lo + step : hi;
  }
  return lo;
}
__device__ inline int64_t last_le_masked(const uint64_t* a, int64_t lo, int64_t hi, uint64_t x, uint64_t mask) {
  int64_t l = lo, h = hi;
  while (h - l > 1) {
    const int64_t m = l + (h - l) / 2;
    if ((a[m] & mask) <= x) l = m;
    else h = m;
  }
  return l;
}

// Segment of item g (pre: per-segment prefix, nseg+1 entries) when the wave
// works on the consecutive items [first, last]: two wave searches bound the
// segments of the wave, then each lane searches only that small range.
__device__ inline int64_t wave_seg(const uint64_t* pre, int64_t nseg, uint64_t g, uint64_t first, uint64_t last) {
  const int64_t lo = wave_last_le<uint64_t>(pre, 0, nseg, first);
  const int64_t hi = wave_last_le<uint64_t>(pre, lo, nseg, last);
  return last_le<uint64_t>(pre, lo, hi + 1, g);
}

// Exclusive scans of up to 8 columns of n per-segment values, one block of
// 1024 threads per column: out[c][i] = sum of in[c][0..i), out[c][n] = the
// column total (also stored to meta[meta_idx[c]] when meta_idx[c] >= 0).
// Chunks of COL_CHUNK values are staged in LDS with coalesced loads and
// stores; each thread scans 8 consecutive values, one block scan joins them.
constexpr int COL_CHUNK = 8192;
constexpr int COL_MAX = 8;
struct ColScan {
  const uint64_t* in[COL_MAX];
  uint64_t* out[COL_MAX];
  uint64_t cap[COL_MAX];  // a total above cap[c] is a capacity error
  int8_t meta_idx[COL_MAX];
  int64_t* meta;
  uint32_t* status;
  int64_t n;
};

// Column c of a ColScan, by one block of 1024 threads (s_v: COL_CHUNK
// values, s_w: 16 words of LDS).  Ends with a block barrier.
__device__ inline void scan_column(const ColScan& a, int c, uint64_t* s_v, uint64_t* s_w) {
  const uint64_t* in = a.in[c];
  uint64_t* out = a.out[c];
  const int t = threadIdx.x;
  uint64_t carry = 0;
  for (int64_t base = 0; base < a.n; base += COL_CHUNK) {
    const int64_t m = a.n - base < COL_CHUNK ? a.n - base : COL_CHUNK;
    for (int i = t; i < COL_CHUNK; i += 1024) s_v[i] = i < m ? in[base + i] : 0;
    __syncthreads();
    uint64_t v[8], sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = sum;
      sum += s_v[8 * t + k];
    }
    const uint64_t incl = wave_incl_scan(sum);
    if (lane_id() == 63) s_w[t / 64] = incl;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      pre += (i < t / 64) ? s_w[i] : 0;
      tot += s_w[i];
    }
    const uint64_t e = carry + pre + incl - sum;
#pragma unroll
    for (int k = 0; k < 8; ++k) s_v[8 * t + k] = e + v[k];
    __syncthreads();
    for (int i = t; i < m; i += 1024) out[base + i] = s_v[i];
    carry += tot;
    __syncthreads();
  }
  if (t == 0) {
    out[a.n] = carry;
    if (a.meta && a.meta_idx[c] >= 0) a.meta[a.meta_idx[c]] = (int64_t)carry;
    if (carry > a.cap[c] && a.status) fail(a.status, ERR_CAPACITY);
  }
  __syncthreads();
}

// One block of 1024 threads per column.
[[maybe_unused]] static __global__ __launch_bounds__(1024) void k_scan_cols(ColScan a) {
  __shared__ uint64_t s_v[COL_CHUNK];
  __shared__ uint64_t s_w[16];
  scan_column(a, blockIdx.x, s_v, s_w);
}

// Segment counts up to which a call's per-segment passes and their column
// scans run as one block of 1024 threads in one launch (fewer launches; above
// it, one thread per segment over many blocks is faster).
constexpr int64_t FUSE_NSEG = 127;

// All columns of a ColScan with n <= FUSE_NSEG (so n + 1 values fit 128
// threads) at once, column c by threads [128 c, 128 c + 128) of a block of
// 1024: one load per value, a wave scan, the two waves of a column joined
// through s_w (16 words of LDS).  Ends with a block barrier.
__device__ inline void scan_columns_small(const ColScan& a, int ncols, uint64_t* s_w) {
  const int t = threadIdx.x, c = t / 128, i = t % 128;
  const bool on = c < ncols;
  const uint64_t v = on && i < a.n ? a.in[c][i] : 0;
  const uint64_t incl = wave_incl_scan64(v);
  if (lane_id() == WAVE - 1) s_w[t / WAVE] = incl;
  __syncthreads();
  const uint64_t lo = (t / WAVE) & 1 ? s_w[t / WAVE - 1] : 0;  // the column's first wave
  if (on && i <= a.n) a.out[c][i] = lo + incl - v;            // (i = n: the total)
  if (on && i == 0) {
    const uint64_t tot = s_w[2 * c] + s_w[2 * c + 1];
    if (a.meta && a.meta_idx[c] >= 0) a.meta[a.meta_idx[c]] = (int64_t)tot;
    if (tot > a.cap[c] && a.status) fail(a.status, ERR_CAPACITY);
  }
  __syncthreads();
}

__device__ inline uint64_t ld64(const uint8_t* p) { return *reinterpret_cast<const uint64_t*>(p); }
__device__ inline uint32_t ld32(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }

}  // namespace ta
