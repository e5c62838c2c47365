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
//   k_ser_msgoff one block: message sizes, their offsets, the headers
//   k_ser_pack   one thread per output word: each block stages the metadata
//                of the records its 1024 words touch in LDS and writes the
//                words with coalesced 8-byte stores; it also writes the
//                offset table entries of the records starting in its window
#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

constexpr int PACK_WPT = 4;
constexpr int PACK_BW = BLOCK * PACK_WPT;   // words per block window
constexpr int PACK_MAXREC = PACK_BW / 2 + 2;  // records are >= 2 words

struct SerScratch {
  uint64_t* wpre;  // [idx_cap+1] exclusive prefix of record words
  int64_t* meta;   // [0] records, [1] total words to pack (0 on error)
};

__global__ __launch_bounds__(BLOCK) void k_ser_begin(const int64_t* seg_off, int64_t nseg, int64_t idx_cap,
                                                     SerScratch sc, ClearFirst cf, uint32_t* status) {
  do_clear_first(cf);
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = seg_off[0] != 0 || seg_off[nseg] > idx_cap;
  __syncthreads();
  for (int64_t s = threadIdx.x; s < nseg; s += BLOCK)
    if (seg_off[s + 1] < seg_off[s]) s_bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_bad) fail(status, ERR_INVALID);
    sc.meta[0] = s_bad ? 0 : seg_off[nseg];
    sc.meta[1] = 0;
  }
}

struct WordsIn {
  const int32_t* idx;
  const uint16_t* cls;
  const int64_t* beh_off;
  const uint16_t* nf;
  const uint16_t* ni;
  uint32_t ncls;
  int64_t n_agents;
  uint32_t* status;
  __device__ uint64_t operator()(int64_t r) const {
    const int64_t a = idx[r];
    if (a < 0 || a >= n_agents) {
      fail(status, ERR_INVALID);
      return 2;
    }
    const uint32_t c = cls[a];
    const int64_t b0 = beh_off[a], b1 = beh_off[a + 1];
    if (c >= ncls || b1 < b0 || ((b1 - b0) & 7) || (b0 & 7)) {
      fail(status, ERR_INVALID);
      return 2;
    }
    return 2 + nf[c] + (ni[c] + 1) / 2 + (uint64_t)(b1 - b0) / 8;
  }
};

__global__ __launch_bounds__(1024) void k_ser_msgoff(const int64_t* seg_off, int64_t nseg, SerScratch sc,
                                                     uint8_t* out, int64_t out_cap, int64_t* msg_off,
                                                     uint32_t* status) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry;
  const bool bad = (status_of(status) & (1u << ERR_INVALID)) != 0;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < nseg; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    uint64_t size = 0;
    if (s < nseg) {
      const uint64_t n = bad ? 0 : (uint64_t)(seg_off[s + 1] - seg_off[s]);
      const uint64_t rw = bad ? 0 : sc.wpre[seg_off[s + 1]] - sc.wpre[seg_off[s]];
      size = tam1_size(n, rw);
    }
    const uint64_t incl = wave_incl_scan(size);
    if (lane_id() == 63) s_w[threadIdx.x / 64] = incl;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      pre += (i < (int)(threadIdx.x / 64)) ? s_w[i] : 0;
      tot += s_w[i];
    }
    if (s < nseg) msg_off[s] = (int64_t)(s_carry + pre + incl - size);
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  const uint64_t total = s_carry;
  const bool fits = total <= (uint64_t)out_cap && !bad;
  if (threadIdx.x == 0) {
    msg_off[nseg] = (int64_t)total;
    if (!bad && !fits) fail(status, ERR_CAPACITY);
    sc.meta[1] = fits ? (int64_t)sc.wpre[sc.meta[0]] : 0;
  }
  if (!fits) return;
  __syncthreads();
  for (int64_t s = threadIdx.x; s < nseg; s += 1024) {
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
};

__global__ __launch_bounds__(BLOCK) void k_ser_pack(PackArgs a, SerScratch sc) {
  __shared__ uint64_t s_start[PACK_MAXREC + 1];  // record start words (global word space)
  __shared__ int64_t s_obase[PACK_MAXREC];       // byte offset of record start in out
  __shared__ int32_t s_agent[PACK_MAXREC];
  __shared__ uint32_t s_meta[PACK_MAXREC];       // class | nf << 8 | ni << 16 (i32 words)
  __shared__ int64_t s_r0;
  __shared__ int32_t s_nrec;
  const int64_t R = sc.meta[0];
  const uint64_t Wt = (uint64_t)sc.meta[1];
  for (uint64_t q0 = (uint64_t)blockIdx.x * PACK_BW; q0 < Wt; q0 += (uint64_t)gridDim.x * PACK_BW) {
    const uint64_t qe = q0 + PACK_BW < Wt ? q0 + PACK_BW : Wt;
    if (threadIdx.x == 0) {
      const int64_t r0 = last_le<uint64_t>(sc.wpre, 0, R, q0);
      const int64_t r1 = last_le<uint64_t>(sc.wpre, 0, R, qe - 1);
      s_r0 = r0;
      s_nrec = (int32_t)(r1 - r0 + 1);
    }
    __syncthreads();
    const int64_t r0 = s_r0;
    const int nrec = s_nrec;
    for (int k = threadIdx.x; k < nrec; k += BLOCK) {
      const int64_t r = r0 + k;
      const int32_t ag = a.idx[r];
      const uint32_t c = a.cls[ag];
      const int64_t s = last_le<int64_t>(a.seg_off, 0, a.nseg, r);
      const int64_t first = a.seg_off[s];
      const uint64_t n = (uint64_t)(a.seg_off[s + 1] - first);
      const uint64_t wr = sc.wpre[r], ws = sc.wpre[first];
      s_start[k] = wr;
      s_agent[k] = ag;
      s_meta[k] = c | ((uint32_t)a.nf[c] << 8) | ((uint32_t)a.ni[c] << 16);
      const int64_t mbase = a.msg_off[s];
      s_obase[k] = mbase + 32 + 8 * (int64_t)((n + 1) / 2) + 8 * (int64_t)(wr - ws);
      if (wr >= q0) *reinterpret_cast<uint32_t*>(a.out + mbase + 32 + 4 * (r - first)) = (uint32_t)(wr - ws);
    }
    if (threadIdx.x == 0) s_start[nrec] = sc.wpre[r0 + nrec];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PACK_WPT; ++j) {
      const uint64_t q = q0 + (uint64_t)j * BLOCK + threadIdx.x;
      if (q >= qe) break;
      // record of word q: last staged start <= q
      int lo = 0, hi = nrec;
      while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (s_start[m] <= q) lo = m;
        else hi = m;
      }
      const uint64_t k = q - s_start[lo];
      const int32_t ag = s_agent[lo];
      const uint32_t meta = s_meta[lo];
      const uint32_t F = (meta >> 8) & 0xFF, I = meta >> 16, IW = (I + 1) / 2;
      uint64_t v;
      if (k == 0) {
        v = a.uid[ag];
      } else if (k == 1) {
        const uint64_t words = s_start[lo + 1] - s_start[lo];
        v = (uint64_t)(meta & 0xFF) | ((uint64_t)a.nb[ag] << 16) | (words << 32);
      } else if (k < 2 + F) {
        v = __double_as_longlong(a.f64[(int64_t)(k - 2) * a.fstride + ag]);
      } else if (k < 2 + F + IW) {
        const int64_t j2 = 2 * (int64_t)(k - 2 - F);
        const uint32_t lo32 = (uint32_t)a.i32[j2 * a.istride + ag];
        const uint32_t hi32 = (j2 + 1 < (int64_t)I) ? (uint32_t)a.i32[(j2 + 1) * a.istride + ag] : 0u;
        v = (uint64_t)lo32 | ((uint64_t)hi32 << 32);
      } else {
        v = *reinterpret_cast<const uint64_t*>(a.beh + a.beh_off[ag] + 8 * (int64_t)(k - 2 - F - IW));
      }
      *reinterpret_cast<uint64_t*>(a.out + s_obase[lo] + 8 * (int64_t)k) = v;
    }
    __syncthreads();
  }
}

SerScratch carve(Arena& ar, int64_t idx_cap) {
  SerScratch sc;
  sc.wpre = ar.take<uint64_t>(idx_cap + 1);
  sc.meta = ar.take<int64_t>(4);
  return sc;
}

}  // namespace

namespace ta {
size_t serialize_scratch(int64_t nseg, int64_t idx_cap, int64_t* tiles) {
  (void)nseg;
  Arena ar{nullptr, 0, 0};
  carve(ar, idx_cap);
  *tiles = ceil_div(idx_cap + 1, SCAN_TILE) + 1;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_serialize(ta_ctx* c, const ta_agents* ag, const int32_t* idx, const int64_t* seg_off,
                                  int64_t nseg, int64_t idx_cap, uint8_t* out, int64_t out_cap, int64_t* msg_off,
                                  void* stream) {
  if (!c || !ag || nseg < 0 || !seg_off || !msg_off || idx_cap < 0 || (idx_cap > 0 && !idx) || out_cap < 0 ||
      (out_cap > 0 && !out) || ag->n < 0 || ag->f64_stride < ag->n || ag->i32_stride < ag->n)
    return TA_ERR_INVALID;
  if (nseg == 0) return hipMemsetAsync(msg_off, 0, 8, (hipStream_t)stream) == hipSuccess ? TA_OK : TA_ERR_HIP;
  int64_t tiles;
  ta_status st = ensure_scratch(c, serialize_scratch(nseg, idx_cap, &tiles), tiles);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{c->scratch, c->scratch_cap, 0};
  SerScratch sc = carve(ar, idx_cap);
  k_ser_begin<<<1, BLOCK, 0, s>>>(seg_off, nseg, idx_cap, sc, clear_first(c), c->d_status);
  WordsIn win{idx, ag->cls, ag->beh_off, c->d_nf, c->d_ni, c->n_classes, ag->n, c->d_status};
  k_scan<WordsIn><<<grid_for(c, idx_cap + 1, SCAN_TILE), BLOCK, 0, s>>>(win, sc.meta, sc.wpre, lookback(c, 0));
  k_ser_msgoff<<<1, 1024, 0, s>>>(seg_off, nseg, sc, out, out_cap, msg_off, c->d_status);
  {
    Timed tm(c, "serialize_pack", s);
    PackArgs pa{ag->uid, ag->cls, ag->nb, ag->f64, ag->f64_stride, ag->i32, ag->i32_stride, ag->beh_off,
                ag->beh, c->d_nf, c->d_ni, idx, seg_off, nseg, msg_off, out};
    // words: at most idx_cap records of at most 2 + 64 + 32 + behaviour words; the
    // grid only needs to be large enough to fill the chip
    k_ser_pack<<<c->grid, BLOCK, 0, s>>>(pa, sc);
  }
  TA_LAUNCH_CHECK();
  return TA_OK;
}
