// ta_mutate.hip -- growth of records used in place, and compaction back to
// canonical messages (Sec. 2.2.1, "Mutability").
//
// A record read and changed in place through a view may need more room than
// it has (a behaviour is added).  The paper gives up the old block and takes
// a new one outside the buffer.  Here the new blocks come from an arena that
// follows the last message in the same buffer; offsets count words from the
// message's record area, so a redirected offset simply points past it.
//
// ta_view_grow:    k_grow_check (every listed record checked, its block
//                  located), k_scan (arena positions), k_grow_move (blocks
//                  copied, zero words added, header size and offset updated)
// ta_view_compact: k_cmp_setup (headers), k_scan_cols (record prefix),
//                  k_scan<CRecIn> (record sizes, every block checked),
//                  k_cmp_sizes, k_scan_cols (message offsets), k_cmp_heads,
//                  k_cmp_write (offset entries and record words)
#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

constexpr int64_t GROW_CAP_MAX = int64_t(1) << 35;  // offsets into the arena stay 32-bit

struct GrowScratch {
  uint64_t* pos;   // [n] byte position of the block in use
  uint64_t* w;     // [n] its words
  uint64_t* recs;  // [n] byte position of the message's record area
  uint64_t* ent;   // [n] byte position of the record's offset entry
  uint64_t* scan;  // [n+1] words before record k in the arena
  int64_t* meta;   // [0] records listed, [1] arena bytes in use
};

// Every listed record: ascending (message, record), inside its message, its
// block in use below the arena's free part, new size not smaller.
__global__ __launch_bounds__(BLOCK) void k_grow_check(const uint8_t* msgs, int64_t cap, const int64_t* msg_off,
                                                      int64_t nseg, const int32_t* seg, const uint32_t* rec,
                                                      const uint32_t* words, int64_t n, const int64_t* arena_used,
                                                      GrowScratch g, ClearFirst cf, uint32_t* status) {
  do_clear_first(cf);
  const int64_t a0 = msg_off[nseg], used = *arena_used;
  const bool base_ok = a0 >= 0 && a0 <= cap && !(a0 & 7) && used >= 0 && !(used & 7) && a0 + used <= cap;
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (int64_t)gridDim.x * BLOCK;
  if (tid == 0) {
    g.meta[0] = base_ok ? n : 0;
    g.meta[1] = used;
    if (!base_ok) fail(status, ERR_INVALID);
  }
  if (!base_ok) return;
  const int64_t limit = a0 + used;
  for (int64_t k = tid; k < n; k += stride) {
    const int64_t s = seg[k];
    bool ok = s >= 0 && s < nseg;
    if (ok && k > 0) ok = seg[k - 1] < s || (seg[k - 1] == s && rec[k - 1] < rec[k]);
    int64_t a = 0, b = 0;
    if (ok) {
      a = msg_off[s];
      b = msg_off[s + 1];
      ok = a >= 0 && b >= a && b <= a0 && !(a & 7);
    }
    uint32_t nn = 0;
    uint64_t rw = 0;
    if (ok) ok = tam1_header(msgs + a, b - a, &nn, &rw) && rec[k] < nn;
    uint64_t p = 0, w = 0, recs = 0;
    if (ok) {
      recs = (uint64_t)a + 32 + 8 * (((uint64_t)nn + 1) / 2);
      p = recs + 8 * (uint64_t)ld32(msgs + a + 32 + 4 * (uint64_t)rec[k]);
      ok = p + 16 <= (uint64_t)limit;
    }
    if (ok) {
      w = ld64(msgs + p + 8) >> 32;
      ok = w >= 2 && p + 8 * w <= (uint64_t)limit && (uint64_t)words[k] >= w;
    }
    if (!ok) {
      fail(status, ERR_INVALID);
      continue;
    }
    g.pos[k] = p;
    g.w[k] = w;
    g.recs[k] = recs;
    g.ent[k] = (uint64_t)a + 32 + 4 * (uint64_t)rec[k];
  }
}

struct GrowIn {
  const uint32_t* words;
  __device__ uint64_t operator()(int64_t k) const { return words[k]; }
};

// Blocks copied into the arena in list order, zero words added, header size
// and offset entry updated; the arena's use grows by the listed sizes.
// Nothing is written when a record failed its check or the arena is full.
__global__ __launch_bounds__(BLOCK) void k_grow_move(uint8_t* msgs, int64_t cap, const int64_t* msg_off, int64_t nseg,
                                                     const uint32_t* words, GrowScratch g, int64_t* arena_used,
                                                     uint32_t* status) {
  if (status_of(status) & ANY_ERR) return;
  const int64_t n = g.meta[0], used = g.meta[1], a0 = msg_off[nseg];
  const uint64_t total = g.scan[n];
  if (a0 + used + 8 * (int64_t)total > cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fail(status, ERR_CAPACITY);
    return;
  }
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (int64_t)gridDim.x * BLOCK;
  if (tid == 0) *arena_used = used + 8 * (int64_t)total;
  for (int64_t k = tid; k < n; k += stride) {
    const uint64_t at = (uint64_t)(a0 + used) + 8 * g.scan[k], w = g.w[k], nw = words[k];
    const uint64_t* src = reinterpret_cast<const uint64_t*>(msgs + g.pos[k]);
    uint64_t* dst = reinterpret_cast<uint64_t*>(msgs + at);
    for (uint64_t i = 0; i < w; ++i) dst[i] = i == 1 ? (src[1] & 0xFFFFFFFFull) | (nw << 32) : src[i];
    for (uint64_t i = w; i < nw; ++i) dst[i] = 0;
    *reinterpret_cast<uint32_t*>(msgs + g.ent[k]) = (uint32_t)((at - g.recs[k]) / 8);
  }
}

struct CmpScratch {
  uint64_t* mrec;  // [nseg+1] records of message s (0 when its header is bad)
  uint64_t* rpre;  // [nseg+1]
  uint64_t* wscan; // [rec_cap+1] words of the records before r
  uint64_t* msz;   // [nseg+1] output message sizes
  int64_t* meta;   // [0] records of all messages
};

__global__ __launch_bounds__(BLOCK) void k_cmp_setup(const uint8_t* msgs, int64_t cap, const int64_t* msg_off,
                                                     int64_t nseg, CmpScratch c, ClearFirst cf, uint32_t* status) {
  do_clear_first(cf);
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t s = tid; s < nseg; s += stride) {
    const int64_t a = msg_off[s], b = msg_off[s + 1];
    uint32_t nn = 0;
    uint64_t rw = 0;
    const bool ok = a >= 0 && b >= a && b <= cap && !(a & 7) && tam1_header(msgs + a, b - a, &nn, &rw);
    if (!ok) fail(status, ERR_INVALID);
    c.mrec[s] = ok ? nn : 0;
  }
}

// Record r of all messages: its block located through its offset (anywhere
// in the buffer) and checked; value = its words.
struct CRecIn {
  const uint8_t* msgs;
  int64_t cap;
  const int64_t* msg_off;
  const uint64_t* rpre;
  const uint64_t* mrec;
  int64_t nseg;
  uint32_t* status;
  int64_t lo = 0, hi = 0;
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(rpre, 0, nseg, (uint64_t)first);
    hi = wave_last_le<uint64_t>(rpre, lo, nseg, (uint64_t)last);
  }
  // All rounds in stages: message, its descriptors, the offset, the header
  // word (read from the buffer's start when out of range).
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    int64_t s[R];
    uint64_t i[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t it = wbase + r * WAVE + l, rc = it < n ? it : n - 1;
      s[r] = last_le<uint64_t>(rpre, lo, hi + 1, (uint64_t)rc);
      i[r] = (uint64_t)rc;
    }
    uint64_t a[R], nn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      a[r] = (uint64_t)msg_off[s[r]];
      nn[r] = mrec[s[r]];
      i[r] -= rpre[s[r]];
    }
    __builtin_amdgcn_sched_barrier(0);
    uint64_t p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = a[r] + 32 + 8 * ((nn[r] + 1) / 2) + 8 * (uint64_t)ld32(msgs + a[r] + 32 + 4 * i[r]);
    __builtin_amdgcn_sched_barrier(0);
    uint64_t w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] = ld64(msgs + (p[r] + 16 <= (uint64_t)cap ? p[r] : 0) + 8) >> 32;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool live = wbase + r * WAVE + l < n;
      const bool ok = p[r] + 16 <= (uint64_t)cap && w[r] >= 2 && p[r] + 8 * w[r] <= (uint64_t)cap;
      bad = bad || (live && !ok);
      v[r] = live && ok ? w[r] : 0;
    }
    if (bad) fail(status, ERR_INVALID);
  }
};

__global__ __launch_bounds__(BLOCK) void k_cmp_sizes(int64_t nseg, CmpScratch c, uint32_t* status) {
  if (status_of(status) & ANY_ERR) return;
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * BLOCK) {
    const uint64_t nn = c.mrec[s];
    c.msz[s] = 32 + 8 * ((nn + 1) / 2) + 8 * (c.wscan[c.rpre[s + 1]] - c.wscan[c.rpre[s]]);
  }
}

// Message headers and the zero pad of an odd offset table (one thread per
// message).
__global__ __launch_bounds__(BLOCK) void k_cmp_heads(int64_t nseg, CmpScratch c, uint8_t* out, const int64_t* out_off,
                                                     uint32_t* status) {
  if (status_of(status) & ANY_ERR) return;
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * BLOCK) {
    const uint64_t nn = c.mrec[s];
    uint8_t* m = out + out_off[s];
    uint64_t* h = reinterpret_cast<uint64_t*>(m);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);  // version 1, flags 0
    h[1] = nn;
    h[2] = c.wscan[c.rpre[s + 1]] - c.wscan[c.rpre[s]];
    h[3] = 0;
    if (nn & 1) *reinterpret_cast<uint32_t*>(m + 32 + 4 * nn) = 0;
  }
}

// Records: a wave takes 64 consecutive records (their messages found once
// per wave), writes their offset entries, tabulates source and destination
// words in LDS and copies the words lane-parallel (consecutive lanes,
// consecutive words; CW_U words per lane in flight).
constexpr int CW_U = 4;
struct CopyTab {
  uint64_t q[WAVE + 1];
  uint64_t src[WAVE];
  uint64_t dst[WAVE];
};
__global__ __launch_bounds__(BLOCK) void k_cmp_write(const uint8_t* msgs, const int64_t* msg_off, int64_t nseg,
                                                     CmpScratch c, uint8_t* out, const int64_t* out_off,
                                                     uint32_t* status) {
  __shared__ CopyTab s_t[WAVES];
  if (status_of(status) & ANY_ERR) return;
  const int64_t Rt = c.meta[0];
  const int l = lane_id(), wv = wave_id();
  CopyTab& t = s_t[wv];
  const uint64_t* src64 = reinterpret_cast<const uint64_t*>(msgs);
  uint64_t* dst64 = reinterpret_cast<uint64_t*>(out);
  for (int64_t r0 = ((int64_t)blockIdx.x * WAVES + wv) * WAVE; r0 < Rt; r0 += (int64_t)gridDim.x * BLOCK) {
    const int64_t r = r0 + l, last = r0 + WAVE - 1 < Rt ? r0 + WAVE - 1 : Rt - 1;
    const int n = (int)(last - r0 + 1);
    const int64_t rc = r < Rt ? r : Rt - 1;
    const int64_t s = wave_seg(c.rpre, nseg, (uint64_t)rc, (uint64_t)r0, (uint64_t)last);
    const uint64_t a = (uint64_t)msg_off[s], nn = c.mrec[s], i = (uint64_t)rc - c.rpre[s];
    const uint64_t p = a + 32 + 8 * ((nn + 1) / 2) + 8 * (uint64_t)ld32(msgs + a + 32 + 4 * i);
    const uint64_t q = c.wscan[rc] - c.wscan[c.rpre[s]];  // the record's canonical offset
    const uint64_t o = (uint64_t)out_off[s];
    const uint64_t wr = c.wscan[rc] - c.wscan[r0];        // words before it in the wave
    if (r < Rt) {
      *reinterpret_cast<uint32_t*>(out + o + 32 + 4 * i) = (uint32_t)q;
      t.q[l] = wr;
      t.src[l] = p / 8;
      t.dst[l] = (o + 32 + 8 * ((nn + 1) / 2)) / 8 + q;
    }
    if (l == 0) t.q[n] = c.wscan[last + 1] - c.wscan[r0];
    wave_sync();
    const uint64_t tot = t.q[n];
    for (uint64_t q0 = l; q0 < tot; q0 += CW_U * WAVE) {
      uint64_t v[CW_U], d[CW_U];
#pragma unroll
      for (int j = 0; j < CW_U; ++j) {
        const uint64_t qq = q0 + (uint64_t)j * WAVE < tot ? q0 + (uint64_t)j * WAVE : tot - 1;
        int lo = 0, hi = n;  // the last record whose first word is <= qq
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (t.q[mid] <= qq) lo = mid;
          else hi = mid;
        }
        const uint64_t w = qq - t.q[lo];
        v[j] = src64[t.src[lo] + w];
        d[j] = t.dst[lo] + w;
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < CW_U; ++j)
        if (q0 + (uint64_t)j * WAVE < tot) dst64[d[j]] = v[j];
    }
    wave_sync();
  }
}

int64_t cmp_rec_bound(int64_t cap) { return cap / 16 + 1; }

GrowScratch carve_grow(Arena& ar, int64_t n) {
  GrowScratch g;
  g.pos = ar.take<uint64_t>(n + 1);
  g.w = ar.take<uint64_t>(n + 1);
  g.recs = ar.take<uint64_t>(n + 1);
  g.ent = ar.take<uint64_t>(n + 1);
  g.scan = ar.take<uint64_t>(n + 1);
  g.meta = ar.take<int64_t>(4);
  return g;
}

CmpScratch carve_cmp(Arena& ar, int64_t nseg, int64_t cap) {
  CmpScratch c;
  c.mrec = ar.take<uint64_t>(nseg + 1);
  c.rpre = ar.take<uint64_t>(nseg + 1);
  c.wscan = ar.take<uint64_t>(cmp_rec_bound(cap) + 1);
  c.msz = ar.take<uint64_t>(nseg + 1);
  c.meta = ar.take<int64_t>(4);
  return c;
}

}  // namespace

namespace ta {
size_t grow_scratch(int64_t n, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  carve_grow(ar, n);
  *tiles = ceil_div(n + 1, SCAN_TILE) + 1;
  return ar.used + 256;
}
size_t compact_scratch(int64_t nseg, int64_t cap, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  carve_cmp(ar, nseg, cap);
  *tiles = ceil_div(cmp_rec_bound(cap) + 1, SCAN_TILE) + 1;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_view_grow(ta_ctx* c, uint8_t* msgs, int64_t cap, const int64_t* msg_off, int64_t nseg,
                                  const int32_t* seg, const uint32_t* rec, const uint32_t* words, int64_t n,
                                  int64_t* arena_used, void* stream) {
  if (!c || cap < 0 || cap > GROW_CAP_MAX || (cap > 0 && !msgs) || !msg_off || nseg < 0 || n < 0 ||
      (n > 0 && (!seg || !rec || !words)) || !arena_used)
    return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  int64_t tiles;
  ta_status st = ensure_scratch(c, grow_scratch(n, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const GrowScratch g = carve_grow(ar, n);
  k_grow_check<<<grid_for(c, n, BLOCK), BLOCK, 0, s>>>(msgs, cap, msg_off, nseg, seg, rec, words, n, arena_used, g,
                                                       clear_first(c, ceil_div(n + 1, SCAN_TILE)), c->d_status);
  k_scan<GrowIn><<<grid_for(c, n + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(GrowIn{words}, g.meta, n, g.scan,
                                                                     lookback(c, 0));
  k_grow_move<<<grid_for(c, n, BLOCK), BLOCK, 0, s>>>(msgs, cap, msg_off, nseg, words, g, arena_used, c->d_status);
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_view_compact(ta_ctx* c, const uint8_t* msgs, int64_t cap, const int64_t* msg_off,
                                     int64_t nseg, uint8_t* out, int64_t out_cap, int64_t* out_off, void* stream) {
  if (!c || cap < 0 || (cap > 0 && !msgs) || !msg_off || nseg < 0 || out_cap < 0 || (out_cap > 0 && !out) ||
      !out_off)
    return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (nseg == 0) return zero_i64(out_off, 1, s);
  const int64_t rb = cmp_rec_bound(cap);
  int64_t tiles;
  ta_status st = ensure_scratch(c, compact_scratch(nseg, cap, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const CmpScratch m = carve_cmp(ar, nseg, cap);
  k_cmp_setup<<<grid_for(c, nseg, BLOCK), BLOCK, 0, s>>>(msgs, cap, msg_off, nseg, m,
                                                         clear_first(c, ceil_div(rb + 1, SCAN_TILE)), c->d_status);
  {
    ColScan cs{};
    cs.in[0] = m.mrec;
    cs.out[0] = m.rpre;
    cs.cap[0] = ~0ull;
    cs.meta_idx[0] = 0;
    cs.meta = m.meta;
    cs.status = c->d_status;
    cs.n = nseg;
    k_scan_cols<<<1, 1024, 0, s>>>(cs);
  }
  k_scan<CRecIn><<<grid_for(c, rb + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(
      CRecIn{msgs, cap, msg_off, m.rpre, m.mrec, nseg, c->d_status}, m.meta, rb, m.wscan, lookback(c, 0));
  k_cmp_sizes<<<grid_for(c, nseg, BLOCK), BLOCK, 0, s>>>(nseg, m, c->d_status);
  {
    ColScan cs{};
    cs.in[0] = m.msz;
    cs.out[0] = reinterpret_cast<uint64_t*>(out_off);
    cs.cap[0] = (uint64_t)out_cap;
    cs.meta_idx[0] = -1;
    cs.status = c->d_status;
    cs.n = nseg;
    k_scan_cols<<<1, 1024, 0, s>>>(cs);
  }
  k_cmp_heads<<<grid_for(c, nseg, BLOCK), BLOCK, 0, s>>>(nseg, m, out, out_off, c->d_status);
  k_cmp_write<<<grid_for(c, rb, BLOCK), BLOCK, 0, s>>>(msgs, msg_off, nseg, m, out, out_off, c->d_status);
  TA_LAUNCH_CHECK();
  return TA_OK;
}
