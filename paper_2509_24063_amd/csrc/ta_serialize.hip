// ta_serialize.hip -- TA IO serialization (Sec. 2.2.1, "Serialization").
//
// The paper copies every memory block of the agent tree in order into one
// buffer, replacing the vtable pointer by a class id and pointers by
// markers.  Here a record is the agent's uid, a header word (class,
// behaviour count, size), its fp64 fields, its int32 attributes and its
// behaviour blocks, in that order; an offset table at the start of each
// message replaces pointer fix-ups, so a GPU thread reaches record i in O(1).
//
// Kernels (all segments in one launch each):
//   k_ser_begin  checks the segment table, clears the look-back array
//   k_scan       exclusive scan of record sizes (words) over all records
//   k_ser_sizes  message sizes; k_scan_cols turns them into offsets
//   k_ser_heads  message headers
//   k_ser_pack   one thread per record: fields gathered from the store into
//                LDS (runs of records that fit together), offset-table
//                entry written; the records leave LDS in coalesced stores
#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

struct SerScratch {
  uint64_t* wpre;  // [idx_cap+1] exclusive prefix of record words
  uint64_t* size;  // [nseg] message sizes
  int64_t* meta;   // [0] records, [1] total words to pack (0 on error)
};

__global__ __launch_bounds__(BLOCK) void k_ser_begin(const int64_t* seg_off, int64_t nseg, int64_t idx_cap,
                                                     SerScratch sc, ClearFirst cf, uint32_t* status) {
  do_clear_first(cf);
  const bool bad_ends = seg_off[0] != 0 || seg_off[nseg] > idx_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (bad_ends) fail(status, ERR_INVALID);
    sc.meta[0] = bad_ends ? 0 : seg_off[nseg];
    sc.meta[1] = 0;
  }
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * BLOCK)
    if (seg_off[s + 1] < seg_off[s]) fail(status, ERR_INVALID);
}

// Words of each selected record: 2 + fields + attribute pairs + behaviour
// words, from the agent's class and behaviour range.  Loaded in stages (all
// indices, then all agents' class and behaviour offsets, then the class
// tables) for the scan's rounds together.
struct WordsIn {
  const int32_t* idx;
  const uint16_t* cls;
  const int64_t* beh_off;
  const uint16_t* nf;
  const uint16_t* ni;
  uint32_t ncls;
  int64_t n_agents;
  uint32_t* status;
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    int64_t a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      a[r] = idx[i < n ? i : n - 1];
    }
    __builtin_amdgcn_sched_barrier(0);
    uint32_t c[R];
    int64_t b0[R], b1[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ok[r] = a[r] >= 0 && a[r] < n_agents;
      c[r] = 0;
      b0[r] = b1[r] = 0;
      if (ok[r]) {
        c[r] = cls[a[r]];
        b0[r] = beh_off[a[r]];
        b1[r] = beh_off[a[r] + 1];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ok[r] = ok[r] && c[r] < ncls && b1[r] >= b0[r] && !((b1[r] - b0[r]) & 7) && !(b0[r] & 7);
      bad = bad || !ok[r];
      v[r] = ok[r] ? 2 + nf[c[r]] + (ni[c[r]] + 1) / 2 + (uint64_t)(b1[r] - b0[r]) / 8 : 2;
      if (wbase + r * WAVE + l >= n) v[r] = 0;
    }
    if (bad) fail(status, ERR_INVALID);
  }
};

// Message sizes (one thread per segment), scanned by k_scan_cols into the
// message offsets; then k_ser_heads writes the headers.
__device__ void ser_sizes(const int64_t* seg_off, int64_t nseg, SerScratch sc, uint32_t* status) {
  const bool bad = (status_of(status) & (1u << ERR_INVALID)) != 0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t n = bad ? 0 : (uint64_t)(seg_off[s + 1] - seg_off[s]);
    const uint64_t rw = bad ? 0 : sc.wpre[seg_off[s + 1]] - sc.wpre[seg_off[s]];
    sc.size[s] = tam1_size(n, rw);
  }
}

__global__ __launch_bounds__(BLOCK) void k_ser_sizes(const int64_t* seg_off, int64_t nseg, SerScratch sc,
                                                     uint32_t* status) {
  ser_sizes(seg_off, nseg, sc, status);
}

__device__ void ser_heads(const int64_t* seg_off, int64_t nseg, SerScratch sc, uint8_t* out, int64_t out_cap,
                          const int64_t* msg_off, uint32_t* status) {
  const bool bad = (status_of(status) & (1u << ERR_INVALID)) != 0;
  const uint64_t total = (uint64_t)msg_off[nseg];
  const bool fits = total <= (uint64_t)out_cap && !bad;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!bad && !fits) fail(status, ERR_CAPACITY);
    sc.meta[1] = fits ? (int64_t)sc.wpre[sc.meta[0]] : 0;
  }
  if (!fits) return;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nseg; s += (int64_t)gridDim.x * blockDim.x) {
    uint8_t* m = out + msg_off[s];
    const uint64_t n = (uint64_t)(seg_off[s + 1] - seg_off[s]);
    const uint64_t rw = sc.wpre[seg_off[s + 1]] - sc.wpre[seg_off[s]];
    uint64_t* h = reinterpret_cast<uint64_t*>(m);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);
    h[1] = n;
    h[2] = rw;
    h[3] = 0;
    if (n & 1) *reinterpret_cast<uint32_t*>(m + 32 + 4 * n) = 0;
  }
}

__global__ __launch_bounds__(BLOCK) void k_ser_heads(const int64_t* seg_off, int64_t nseg, SerScratch sc,
                                                     uint8_t* out, int64_t out_cap, const int64_t* msg_off,
                                                     uint32_t* status) {
  ser_heads(seg_off, nseg, sc, out, out_cap, msg_off, status);
}

// Few segments: message sizes, their offsets and the headers in one block.
__global__ __launch_bounds__(1024) void k_ser_layout1(const int64_t* seg_off, int64_t nseg, SerScratch sc,
                                                      uint8_t* out, int64_t out_cap, int64_t* msg_off, ColScan cs,
                                                      uint32_t* status) {
  __shared__ uint64_t s_w[16];
  ser_sizes(seg_off, nseg, sc, status);
  __syncthreads();
  scan_columns_small(cs, 1, s_w);
  ser_heads(seg_off, nseg, sc, out, out_cap, msg_off, status);
}

struct PackArgs {
  const uint64_t* uid;
  const uint16_t* cls;
  const uint16_t* nb;
  const double* f64;
  int64_t fstride;
  const int32_t* i32;
  int64_t istride;
  const int64_t* beh_off;
  const uint8_t* beh;
  const uint16_t* nf;
  const uint16_t* ni;
  const int32_t* idx;
  const int64_t* seg_off;
  int64_t nseg;
  const int64_t* msg_off;
  uint8_t* out;
  uint64_t* keys;  // nullable: uid and header word of every record (record order)
};

constexpr int PACK_CAP = 1024;  // record words one wave stages in LDS
constexpr int PACK_CHUNK = 8;   // payload words a lane gathers at a time

// One lane per record: it gathers the agent's fields and writes its offset
// table entry.  The wave's records are assembled in LDS in batches -- runs
// of consecutive records of one message that fit PACK_CAP words together --
// and each batch is written with coalesced stores; a single record larger
// than PACK_CAP words is written by its lane directly.
__global__ __launch_bounds__(BLOCK) void k_ser_pack(PackArgs a, SerScratch sc) {
  __shared__ uint64_t s_buf[WAVES][PACK_CAP];
  const int64_t R = sc.meta[0];
  if (sc.meta[1] == 0) return;  // nothing to write (error, capacity, or no words)
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  const uint64_t* seg_off = reinterpret_cast<const uint64_t*>(a.seg_off);
  const int l = lane_id(), wv = wave_id();
  uint64_t* buf = s_buf[wv];
  for (int64_t base = (int64_t)blockIdx.x * BLOCK + wv * WAVE; base < R; base += stride) {
    const int64_t r = base + l;
    const int64_t re = base + WAVE < R ? base + WAVE : R;
    const uint64_t last = (uint64_t)(re - 1);
    const int64_t s = wave_seg(seg_off, a.nseg, (uint64_t)(r < R ? r : R - 1), (uint64_t)base, last);
    uint64_t wr = 0, words = 0, uid = 0, nb = 0;
    uint64_t* rec = nullptr;  // the record's place in its message
    int32_t ag = 0;
    uint32_t c = 0, F = 0, I = 0, IW = 0;
    int64_t boff = 0;
    if (r < R) {
      // everything read per agent and per message, before the first store
      ag = a.idx[r];
      c = a.cls[ag];
      uid = a.uid[ag];
      nb = a.nb[ag];
      boff = a.beh_off[ag];
      const int64_t first = a.seg_off[s];
      const uint64_t n = (uint64_t)(a.seg_off[s + 1] - first);
      wr = sc.wpre[r];
      const uint64_t ws = sc.wpre[first];
      words = sc.wpre[r + 1] - wr;
      uint8_t* m = a.out + a.msg_off[s];
      F = a.nf[c];
      I = a.ni[c];
      IW = (I + 1) / 2;
      *reinterpret_cast<uint32_t*>(m + 32 + 4 * (r - first)) = (uint32_t)(wr - ws);
      rec = reinterpret_cast<uint64_t*>(m + 32 + 8 * ((n + 1) / 2) + 8 * (wr - ws));
      if (a.keys)
        *reinterpret_cast<ulonglong2*>(a.keys + 2 * r) = ulonglong2{uid, (uint64_t)c | (nb << 16) | (words << 32)};
    }
    // The record's words into dst: header, F fields, IW attribute pairs,
    // behaviour words.  The 64-bit words (fields and behaviour words) are
    // gathered PACK_CHUNK at a time, then the attribute pairs; every load of
    // a chunk is issued before its stores and takes its address by
    // selection, not behind a branch (an unused one reads the agent's uid).
    auto gather = [&](uint64_t* dst) {
      dst[0] = uid;
      dst[1] = (uint64_t)c | (nb << 16) | (words << 32);
      const uint64_t* bsrc = reinterpret_cast<const uint64_t*>(a.beh + boff);
      const uint64_t* dummy = a.uid + ag;
      const uint32_t Q = (uint32_t)(words - 2 - IW);  // fields + behaviour words
      for (uint32_t q0 = 0; q0 < Q; q0 += PACK_CHUNK) {
        uint64_t t[PACK_CHUNK];
#pragma unroll
        for (int j = 0; j < PACK_CHUNK; ++j) {
          const uint32_t q = q0 + j;
          const uint64_t* src = q < F ? reinterpret_cast<const uint64_t*>(a.f64 + (int64_t)q * a.fstride + ag)
                                      : (q < Q ? bsrc + (q - F) : dummy);
          t[j] = *src;
        }
#pragma unroll
        for (int j = 0; j < PACK_CHUNK; ++j) {
          const uint32_t q = q0 + j;
          if (q < Q) dst[q < F ? 2 + q : 2 + IW + q] = t[j];
        }
      }
      for (uint32_t j0 = 0; j0 < IW; j0 += PACK_CHUNK / 2) {
        uint32_t lo[PACK_CHUNK / 2], hi[PACK_CHUNK / 2];
#pragma unroll
        for (int j = 0; j < PACK_CHUNK / 2; ++j) {
          const uint32_t q = 2 * (j0 + j);
          const uint32_t* d32 = reinterpret_cast<const uint32_t*>(dummy);
          lo[j] = *(q < I ? reinterpret_cast<const uint32_t*>(a.i32 + (int64_t)q * a.istride + ag) : d32);
          hi[j] = *(q + 1 < I ? reinterpret_cast<const uint32_t*>(a.i32 + (int64_t)(q + 1) * a.istride + ag) : d32);
        }
#pragma unroll
        for (int j = 0; j < PACK_CHUNK / 2; ++j) {
          const uint32_t q = 2 * (j0 + j);
          if (j0 + j < IW) dst[2 + F + j0 + j] = (uint64_t)lo[j] | ((uint64_t)(q + 1 < I ? hi[j] : 0u) << 32);
        }
      }
    };
    // batches: from the first pending lane, the run of lanes in its message
    // whose records end within PACK_CAP words of its record's start (the
    // records of a message are consecutive in the words' order)
    uint64_t pending = __ballot(r < R);
    while (pending) {
      const int lead = __ffsll((unsigned long long)pending) - 1;
      const uint64_t bs = readlane64(wr, lead);
      const int64_t bseg = (int64_t)readlane64((uint64_t)s, lead);
      const bool mine = ((pending >> l) & 1) && s == bseg && wr + words - bs <= PACK_CAP;
      const uint64_t batch = __ballot(mine);
      if (!batch) {  // the lead record alone is larger than the LDS buffer
        if (l == lead) gather(rec);
        pending &= pending - 1;
        continue;
      }
      if (mine) gather(buf + (wr - bs));
      wave_sync();
      const int hi_lane = 63 - __clzll((long long)batch);
      const uint64_t be = readlane64(wr + words, hi_lane);
      uint64_t* out = reinterpret_cast<uint64_t*>(readlane64(reinterpret_cast<uint64_t>(rec), lead));
      for (uint64_t p = l; p < be - bs; p += WAVE) out[p] = buf[p];
      wave_sync();  // the buffer is refilled by the next batch
      pending &= ~batch;
    }
  }
}

SerScratch carve(Arena& ar, int64_t nseg, int64_t idx_cap) {
  SerScratch sc;
  sc.wpre = ar.take<uint64_t>(idx_cap + 1);
  sc.size = ar.take<uint64_t>(nseg + 1);
  sc.meta = ar.take<int64_t>(4);
  return sc;
}

}  // namespace

namespace ta {
size_t serialize_scratch(int64_t nseg, int64_t idx_cap, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  carve(ar, nseg, idx_cap);
  *tiles = ceil_div(idx_cap + 1, SCAN_TILE) + 1;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_serialize(ta_ctx* c, const ta_agents* ag, const int32_t* idx, const int64_t* seg_off,
                                  int64_t nseg, int64_t idx_cap, uint8_t* out, int64_t out_cap, int64_t* msg_off,
                                  uint64_t* keys_out, int64_t keys_cap, void* stream) {
  if (!c || !ag || nseg < 0 || !seg_off || !msg_off || idx_cap < 0 || (idx_cap > 0 && !idx) || out_cap < 0 ||
      (out_cap > 0 && !out) || ag->n < 0 || ag->f64_stride < ag->n || ag->i32_stride < ag->n ||
      (keys_out && (keys_cap < idx_cap || ((uintptr_t)keys_out & 15))))
    return TA_ERR_INVALID;
  if (nseg == 0) return zero_i64(msg_off, 1, (hipStream_t)stream);
  use_family(c, FAM_SERIALIZE);
  int64_t tiles;
  ta_status st = ensure_scratch(c, serialize_scratch(nseg, idx_cap, &tiles), tiles);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{c->scratch, c->scratch_cap, 0};
  SerScratch sc = carve(ar, nseg, idx_cap);
  const int gseg = grid_for(c, nseg, BLOCK);
  k_ser_begin<<<gseg, BLOCK, 0, s>>>(seg_off, nseg, idx_cap, sc, clear_first(c, ceil_div(idx_cap + 1, SCAN_TILE)),
                                  c->d_status);
  WordsIn win{idx, ag->cls, ag->beh_off, c->d_nf, c->d_ni, c->n_classes, ag->n, c->d_status};
  k_scan<WordsIn><<<grid_for(c, idx_cap + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(win, sc.meta, idx_cap, sc.wpre, lookback(c, 0));
  {
    ColScan cs{};
    cs.in[0] = sc.size;
    cs.out[0] = reinterpret_cast<uint64_t*>(msg_off);
    cs.cap[0] = ~0ull;  // the output capacity is checked with the headers
    cs.meta_idx[0] = -1;
    cs.status = c->d_status;
    cs.n = nseg;
    if (nseg <= FUSE_NSEG) {
      k_ser_layout1<<<1, 1024, 0, s>>>(seg_off, nseg, sc, out, out_cap, msg_off, cs, c->d_status);
    } else {
      k_ser_sizes<<<gseg, BLOCK, 0, s>>>(seg_off, nseg, sc, c->d_status);
      k_scan_cols<<<1, 1024, 0, s>>>(cs);
      k_ser_heads<<<gseg, BLOCK, 0, s>>>(seg_off, nseg, sc, out, out_cap, msg_off, c->d_status);
    }
  }
  {
    Timed tm(c, "serialize_pack", s);
    PackArgs pa{ag->uid, ag->cls, ag->nb, ag->f64, ag->f64_stride, ag->i32, ag->i32_stride, ag->beh_off,
                ag->beh, c->d_nf, c->d_ni, idx, seg_off, nseg, msg_off, out, keys_out};
    // words: at most idx_cap records of at most 2 + 64 + 32 + behaviour words; the
    // grid only needs to be large enough to fill the chip
    k_ser_pack<<<c->grid, BLOCK, 0, s>>>(pa, sc);
  }
  TA_LAUNCH_CHECK();
  return TA_OK;
}
