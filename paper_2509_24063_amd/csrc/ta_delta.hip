// ta_delta.hip -- delta encoding and decoding of TAM1 messages (Sec. 2.3).
//
// Sender and receiver keep the same reference R (the previous exchange's
// message of the pair).  The sender moves every agent found in both the
// current message C and R to its reference position, leaves an empty
// placeholder for vanished ones and appends new ones; it writes the
// difference against R for matched agents.  The receiver restores the message
// from R and drops the placeholders; the original order is not restored.
//
// Encoder kernels (all segments per launch):
//   k_enc_setup    one thread per segment: message headers, record counts,
//                  hash and join sizes; k_scan_cols turns them into prefixes
//   k_join_count   per tile of records: validate, gather uid and header,
//                  count items per hash bucket of the segment
//   k_scan         bucket counts -> bucket starts
//   k_join_scatter (uid, item) pairs into their buckets
//   k_join_bucket  one block per bucket: LDS hash table pairs current and
//                  reference items with equal uids (duplicates rejected); a
//                  bucket too large for LDS joins in a global table of its own
//   k_scan x2      packed (count << 34 | words) prefixes over R slots
//                  (matched) and C records (new)
//   k_enc_seg2/3   per segment layout, C' offsets and headers
//   k_enc_mdir     matched-record directory (C word, R word, residual start)
//                  and the segment and first record of every residual group
//   k_enc_groups   plain mode: per 64-word group, C' words, the residual
//                  C xor R (in registers), its block; a look-back over tiles
//                  of groups places the blocks
//                  learned mode: the same kernel also forms the residual
//                  against the predictions, keeps the smaller block of each
//                  group and flags the segment's choices; k_choose_mode
//                  picks each segment's mode, k_enc_fixup rewrites the rare
//                  tied groups of learned segments
//   k_enc_fixed    encoding offsets and headers; presence bitmaps, word
//                  bitmaps, block size tables; then the new records: their
//                  sizes, C' offsets and words, into the encoding and into C'
// Decoder: k_dec_setup (header checks), k_dec_rslots (reference slots,
// presence bits), scans of matched slots, new records and group blocks,
// k_dec_seg2 (checks against the header, C' headers), k_dec_mdir (then the
// new records into C'), then k_dec_unpack (group blocks -> residual -> C' =
// D xor X in one pass).
#include <initializer_list>

#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_predict.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int PK = 34;  // packed scan value: count << 34 | words
constexpr uint64_t WMASK = (1ull << PK) - 1;
constexpr int BLK_MAX = 544;          // 32 nibble bytes + 512 significant bytes

constexpr int FOLD_SLOTS = 16;

struct Entry {
  unsigned long long key;
  uint32_t ci, ri;
};

struct Seg {
  uint64_t cmsg, rmsg;        // byte offsets of the messages
  uint64_t cbody, rbody;      // byte offsets of their record areas
  uint64_t nc, nr, rwc, rwr;  // records and record words
  uint64_t hsize, hbase;      // hash slots (power of two) and first slot
  uint64_t fold;              // XOR of the reference uids
  uint64_t n_match, W, n_new, new_words;
  uint64_t mbase, dbase, nbase, npbase;  // global prefixes: matched, residual words, new, new words
  uint64_t G, PG;             // residual groups, presence words
  uint64_t fixed, fixed_excl; // fixed encoding bytes and their prefix
  uint64_t oref;              // offset of this segment's C' message
  uint64_t encm;              // offset of this segment's encoding (decoder: given)
  uint64_t mode;              // 0 plain, 1 learned
  uint64_t rfold;             // decoder: XOR of the reference uids it holds
  uint64_t var;               // decoder: group block bytes announced by the header
  uint64_t size_plain, size_learned;  // encoder, learned mode: block bytes both ways
  uint64_t jB, jT, jTC, jTJ;  // join: buckets, count tiles (C tiles first), items per tile
  uint64_t jebase;            // join: first count entry of the segment
  uint64_t cpw;               // word index of C' for residual position 0 (C' word of position d = cpw + d)
};

// Directory entry of a matched record (learned calls, or a history to
// write): where its reference record is, and its slot and segment.
struct alignas(16) MDir {
  uint64_t rword;   // R record word index in ref
  uint64_t gs;      // global reference slot | segment << 34
};
__device__ inline int64_t mdir_seg(const MDir& e) { return (int64_t)(e.gs >> 34); }
__device__ inline uint64_t mdir_slot(const MDir& e) { return e.gs & ((1ull << 34) - 1); }
// Decoder: what unpacking one residual group needs, written by the
// directory pass so that the unpack reads it with one 64-byte scalar load.
struct alignas(64) GDesc {
  uint64_t blk;    // byte offset of the group's block in the encodings
  uint64_t bm;     // word bitmap of the group's residual
  uint64_t out;    // word index in C' of the group's first residual word
  uint64_t g0w;    // the group's first residual position
  uint64_t rbw;    // word index of the segment's reference record area
  uint32_t k0;     // matched record holding the group's first word
  uint32_t size;   // block bytes (the size byte times 8, the mixed-mode flag taken off)
  uint32_t nlive;  // residual words of the group (1..64)
  uint32_t usep;   // 1: the residual is against the prediction
  uint32_t pad[2];
};
static_assert(sizeof(GDesc) == 64, "one scalar load per group");



// 64-bit bit mixer for hash buckets and table slots: D. Stafford's "Mix01"
// variant of the MurmurHash3 64-bit finalizer ("Better Bit Mixing -
// Improving on MurmurHash3's 64-bit Finalizer", 2011): xor-shift 31,
// multiply, xor-shift 27, multiply, xor-shift 33 with his published
// multipliers.
__device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 31;
  x *= 0x7fb5d329728ea185ull;
  x ^= x >> 27;
  x *= 0x81dadef4bc2dd44dull;
  x ^= x >> 33;
  return x;
}

// Binary search over a per-segment prefix array pre[0..nseg] (non-decreasing):
// the segment holding global item g.
__device__ inline int64_t seg_of(const uint64_t* pre, int64_t nseg, uint64_t g) {
  return last_le<uint64_t>(pre, 0, nseg, g);
}

// XOR-reduce v over the lanes of this wave that belong to the same segment and
// fold it into dst[segment] with one atomic per segment present in the wave.
// fold_base points at slot 0 of segment 0; the wave adds into one of
// FOLD_SLOTS slots chosen by its position so waves rarely share an address.
__device__ inline void seg_xor(uint64_t* fold_base, size_t stride_words, int64_t s, bool active, uint64_t v) {
  uint64_t pending = __ballot(active);
  const uint32_t slot = (blockIdx.x * WAVES + wave_id()) % FOLD_SLOTS;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int64_t s0 = __shfl(s, leader, WAVE);
    const bool mine = active && s == s0;
    const uint64_t part = wave_xor(mine ? v : 0);
    if (lane_id() == leader && part)
      atomicXor((unsigned long long*)(fold_base + stride_words * s0 + slot), (unsigned long long)part);
    pending &= ~__ballot(mine);
  }
}
__device__ inline uint64_t fold_of(const uint64_t* parts) {
  uint64_t f = 0;
  for (int i = 0; i < FOLD_SLOTS; ++i) f ^= parts[i];
  return f;
}

struct Common {
  int64_t nseg;
  Seg* seg;
  uint64_t* cpre;  // [nseg+1] record prefixes (C / encoding new records)
  uint64_t* rpre;  // [nseg+1] reference slot prefixes
  uint64_t* gpre;  // [nseg+1] residual group prefixes
  uint64_t* ppre;  // [nseg+1] presence word prefixes
  uint64_t* npre;  // [nseg+1] new record prefixes
  uint64_t* tpre;  // [nseg+1] join count tiles
  uint64_t* bpre;  // [nseg+1] join buckets
  uint64_t* hpre;  // [nseg+1] hash slot prefixes
  uint64_t* jepre; // [nseg+1] join count entry prefixes
  uint64_t* fxpre; // [nseg+1] fixed encoding byte prefixes
  uint64_t* opre;  // [nseg+1] C' message offsets
  uint64_t* cols;  // [COL_MAX][nseg+1] per segment values to scan
  uint64_t* fold;  // [nseg][FOLD_SLOTS] partial XORs of reference uids (spread to avoid atomic contention)
  int64_t* meta;   // [0] C records [1] R records [2] hash slots [3] groups [4] presence words [5] matched
                   // [6] new records [7] new words [8] unused [9] fixed bytes [10] join tiles
                   // [11] join count entries [12] join buckets [13] join bucket overflow
  uint32_t* status;
  uint32_t op;     // difference operator of the call: 0 XOR, 1 byte-wise subtraction mod 256
};

// The difference of Sec. 2.3, which the paper leaves open.  OP 0: XOR.
// OP 1: each byte subtracted on its own modulo 256, all eight at once: the
// top bit of every byte of c is set and cleared in x so no borrow leaves a
// byte, and the top bits are then corrected (c7 ^ x7 ^ borrow).  Its
// inverse adds the low seven bits of each byte (no carry can leave it) and
// corrects the top bits the same way.  Zero bytes are those of the XOR.
constexpr uint64_t BYTE_TOP = 0x8080808080808080ull;
template <int OP>
__device__ inline uint64_t diff_word(uint64_t c, uint64_t x) {
  if constexpr (OP == 0) return c ^ x;
  else return ((c | BYTE_TOP) - (x & ~BYTE_TOP)) ^ ((c ^ ~x) & BYTE_TOP);
}
template <int OP>
__device__ inline uint64_t undiff_word(uint64_t d, uint64_t x) {
  if constexpr (OP == 0) return d ^ x;
  else return ((d & ~BYTE_TOP) + (x & ~BYTE_TOP)) ^ ((d ^ x) & BYTE_TOP);
}

// Partitioned join: every segment's C and R uids are split into B hash
// buckets (mean <= JB_TARGET items), and one block joins each bucket in LDS.
constexpr int JT = 2048;          // minimum items per counting tile
constexpr int JT_MAX_TILES = 64;  // counting tiles per segment side at most
#ifndef TA_JB_TARGET
#define TA_JB_TARGET 1024
#endif
constexpr int JB_TARGET = TA_JB_TARGET;
constexpr int JC_U = 4;           // join count and bucket: items per thread and pass
constexpr int JS_U = 16;          // join scatter: items per thread and pass (a tile's items in few passes)
constexpr int RS_U = 4;           // record directories: reference slots per lane and pass
constexpr int RL_U = 6;           // decoder reference slots: slots per lane and pass
constexpr int JB_MAX = 8192;      // buckets per segment (LDS histogram)
// A bucket holds JB_TARGET / 2 .. JB_TARGET items on average; JCAP at 1.5x
// the target keeps the bucket block at 32 KB of LDS (five blocks per CU),
// larger buckets take the global-table path.
#ifndef TA_JCAP
#define TA_JCAP 1536
#endif
#ifndef TA_JTAB
#define TA_JTAB 2048
#endif
constexpr int JCAP = TA_JCAP;     // items of one bucket held in LDS
constexpr int JTAB = TA_JTAB;     // LDS hash slots (a power of two above JCAP)
static_assert(JTAB > JCAP && (JTAB & (JTAB - 1)) == 0, "the LDS table must never fill");
__device__ inline uint32_t join_bucket(uint64_t uid, uint64_t B) { return (uint32_t)(mix64(uid) & (B - 1)); }

// ---------------------------------------------------------------------------
// one block of 1024 threads: per segment values and their prefixes
struct BlockScan1024 {
  uint64_t* s_w;  // [16]
  __device__ uint64_t excl(uint64_t v, uint64_t* tot) {
    const uint64_t incl = wave_incl_scan(v);
    if (lane_id() == 63) s_w[threadIdx.x / 64] = incl;
    __syncthreads();
    uint64_t pre = 0, t = 0;
    for (int i = 0; i < 16; ++i) {
      pre += (i < (int)(threadIdx.x / 64)) ? s_w[i] : 0;
      t += s_w[i];
    }
    __syncthreads();
    *tot = t;
    return pre + incl - v;
  }
};

__device__ inline uint64_t pow2ceil(uint64_t x) {
  if (x <= 1) return x;
  return 1ull << (64 - __clzll((long long)(x - 1)));
}

__device__ inline uint64_t* col(const Common& cm, int c) { return cm.cols + (size_t)c * (cm.nseg + 1); }

// Column scan over per-segment values: column c of cm.cols into out[c].
inline ColScan col_scan(const Common& cm, std::initializer_list<uint64_t*> outs, std::initializer_list<int> meta_idx,
                        std::initializer_list<int64_t> caps) {
  ColScan a{};
  int c = 0;
  for (uint64_t* o : outs) {
    a.in[c] = cm.cols + (size_t)c * (cm.nseg + 1);
    a.out[c] = o;
    a.cap[c] = ~0ull;
    ++c;
  }
  c = 0;
  for (int m : meta_idx) a.meta_idx[c++] = (int8_t)m;
  c = 0;
  for (int64_t v : caps) a.cap[c++] = v < 0 ? ~0ull : (uint64_t)v;
  a.meta = cm.meta;
  a.status = cm.status;
  a.n = cm.nseg;
  return a;
}

// One thread per segment: message headers, record counts, hash and join
// sizes (scanned afterwards by k_scan_cols).
__device__ void enc_setup(Common cm, const uint8_t* cur, int64_t cur_len,
                          const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                          const int64_t* ref_off, ClearFirst cf) {
  do_clear_first(cf);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * blockDim.x) {
    uint64_t nc = 0, nr = 0, hs = 0, jt = 0, je = 0, jb = 0;
    Seg& g = cm.seg[s];
    const int64_t ca = cur_off[s], cb = cur_off[s + 1], ra = ref_off[s], rb = ref_off[s + 1];
    uint32_t n;
    uint64_t rw;
    bool ok = ca >= 0 && cb >= ca && cb <= cur_len && !(ca & 7) && ra >= 0 && rb >= ra && rb <= ref_len &&
              !(ra & 7);
    if (ok && tam1_header(cur + ca, cb - ca, &n, &rw)) {
      nc = n;
      g.rwc = rw;
    } else {
      ok = false;
    }
    if (ok && tam1_header(ref + ra, rb - ra, &n, &rw)) {
      nr = n;
      g.rwr = rw;
    } else {
      ok = false;
    }
    if (!ok) {
      fail(cm.status, ERR_INVALID);
      nc = nr = 0;
    }
    g.cmsg = ca;
    g.rmsg = ra;
    g.cbody = ca + 32 + 8 * ((nc + 1) / 2);
    g.rbody = ra + 32 + 8 * ((nr + 1) / 2);
    g.nc = nc;
    g.nr = nr;
    hs = pow2ceil(2 * nr);  // neighbour-count table (learned calls): at most nr cells
    g.hsize = hs;
    g.fold = 0;
    for (int k = 0; k < FOLD_SLOTS; ++k) cm.fold[s * FOLD_SLOTS + k] = 0;
    g.mode = 0;
    // join layout: B buckets, counting tiles of TJ items (C tiles, then R tiles)
    uint64_t B = pow2ceil((nc + nr + JB_TARGET - 1) / JB_TARGET);
    if (B < 1) B = 1;
    if (B > JB_MAX) B = JB_MAX;
    uint64_t TJ = (nc > nr ? nc : nr) / JT_MAX_TILES + 1;
    if (TJ < JT) TJ = JT;
    g.jB = B;
    g.jTJ = TJ;
    g.jTC = (nc + TJ - 1) / TJ;
    g.jT = g.jTC + (nr + TJ - 1) / TJ;
    jt = g.jT;
    je = g.jT * B;
    jb = B;
    col(cm, 0)[s] = nc;
    col(cm, 1)[s] = nr;
    col(cm, 2)[s] = hs;
    col(cm, 3)[s] = jt;
    col(cm, 4)[s] = je;
    col(cm, 5)[s] = jb;
  }
}

__global__ __launch_bounds__(BLOCK) void k_enc_setup(Common cm, const uint8_t* cur, int64_t cur_len,
                                                     const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                                                     const int64_t* ref_off, ClearFirst cf) {
  enc_setup(cm, cur, cur_len, cur_off, ref, ref_len, ref_off, cf);
}

// Global-table join: only used when a join bucket overflowed its LDS block.
struct JoinArgs {
  Common cm;
  const uint8_t* cur;
  const uint8_t* ref;
  uint64_t* juid;    // [C+R] uid of every item (items of a side without keys)
  uint64_t* jhdr;    // [C+R] header word of every item (the same)
  uint32_t* cwords;
  uint32_t* rwords;
  uint32_t* cnt;     // [count entries] items per (segment, bucket, tile)
  uint64_t* cnt_pre; // [count entries + 1]
  uint64_t* part;    // [2 (C+R)] bucketed items: uid, item
  int32_t* m;
  uint8_t* cflag;
  Entry* tab;        // open-addressing tables of buckets too large for LDS
  const uint64_t* ckeys;  // nullable: uid and header word of every current record (2 words each)
  const uint64_t* rkeys;  // nullable: the same for the reference
};

// A bucketed join item: uid and item index, moved as one 16-byte access
// (the pair array is 256-byte aligned).
struct alignas(16) Pair {
  uint64_t uid, item;
};

struct JTile {
  int64_t s;
  uint64_t lt, i0, i1;  // items [i0, i1) of one side of the segment
  bool isC;
};
// (t is the same in every lane: the tile's segment is kept in a scalar register)
__device__ inline JTile join_tile(const Seg* segs, const uint64_t* tpre, int64_t nseg, int64_t t) {
  JTile jt;
  jt.s = (int64_t)uniform32((uint32_t)last_le<uint64_t>(tpre, 0, nseg, (uint64_t)t));
  const Seg& g = segs[jt.s];
  jt.lt = (uint64_t)t - tpre[jt.s];
  jt.isC = jt.lt < g.jTC;
  const uint64_t k = jt.isC ? jt.lt : jt.lt - g.jTC;
  const uint64_t n = jt.isC ? g.nc : g.nr;
  jt.i0 = k * g.jTJ;
  jt.i1 = jt.i0 + g.jTJ < n ? jt.i0 + g.jTJ : n;
  return jt;
}

// J1: validate every record, gather uid and header, count items per bucket.
// (segs, tpre, cpre, rpre, jepre: read-only in the join kernels; as restrict
// parameters their uniform reads become scalar loads)
__global__ __launch_bounds__(BLOCK) void k_join_count(JoinArgs a, const Seg* __restrict__ segs,
                                                      const uint64_t* __restrict__ tpre,
                                                      const uint64_t* __restrict__ cpre,
                                                      const uint64_t* __restrict__ rpre,
                                                      const uint64_t* __restrict__ jepre) {
  __shared__ uint32_t s_hist[JB_MAX];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Tt = cm.meta[10];
  const uint64_t Ct = (uint64_t)cm.meta[0];
  for (int64_t t = blockIdx.x; t < Tt; t += gridDim.x) {
    const JTile jt = join_tile(segs, tpre, cm.nseg, t);
    const Seg& g = segs[jt.s];
    const uint64_t B = g.jB;
    for (uint64_t b = threadIdx.x; b < B; b += BLOCK) s_hist[b] = 0;
    __syncthreads();
    const uint8_t* msg = jt.isC ? a.cur + g.cmsg : a.ref + g.rmsg;
    const uint32_t n = (uint32_t)(jt.isC ? g.nc : g.nr);
    const uint64_t rw = jt.isC ? g.rwc : g.rwr;
    const uint64_t gbase = jt.isC ? cpre[jt.s] : Ct + rpre[jt.s];
    const uint64_t* keys = jt.isC ? a.ckeys : a.rkeys;
    const uint64_t kbase = jt.isC ? cpre[jt.s] : rpre[jt.s];
    uint64_t fold = 0;
    bool bad = false;
    // JC_U items per thread and pass: their records' loads are issued
    // together (indices past the tile read its first item, unused)
    for (uint64_t i0 = jt.i0; i0 < jt.i1; i0 += (uint64_t)BLOCK * JC_U) {
      Tam1Loc loc[JC_U];
      uint64_t uid[JC_U], hdr[JC_U];
      bool ok[JC_U];
#pragma unroll
      for (int u = 0; u < JC_U; ++u) {
        const uint64_t i = i0 + threadIdx.x + (uint64_t)u * BLOCK;
        loc[u] = tam1_locate(msg, n, rw, (uint32_t)(i < jt.i1 ? i : jt.i0));
      }
      if (keys) {  // (uniform) the record words from the compact key array
#pragma unroll
        for (int u = 0; u < JC_U; ++u) {
          const uint64_t i = i0 + threadIdx.x + (uint64_t)u * BLOCK;
          const ulonglong2 kv = *reinterpret_cast<const ulonglong2*>(keys + 2 * (kbase + (i < jt.i1 ? i : jt.i0)));
          uid[u] = kv.x;
          hdr[u] = kv.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < JC_U; ++u) tam1_words(msg, n, loc[u], &uid[u], &hdr[u]);
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the checks below every record load
#pragma unroll
      for (int u = 0; u < JC_U; ++u) ok[u] = tam1_valid(loc[u], hdr[u]) && uid[u] != 0;
#pragma unroll
      for (int u = 0; u < JC_U; ++u) {
        const uint64_t i = i0 + threadIdx.x + (uint64_t)u * BLOCK;
        if (i >= jt.i1) continue;
        if (!ok[u]) {
          bad = true;
          continue;
        }
        if (!keys) {  // (uniform) a side with keys is read from them by the later passes
          a.juid[gbase + i] = uid[u];
          a.jhdr[gbase + i] = hdr[u];
        }
        if (jt.isC) a.cwords[cpre[jt.s] + i] = (uint32_t)(hdr[u] >> 32);
        else a.rwords[rpre[jt.s] + i] = (uint32_t)(hdr[u] >> 32);
        atomicAdd(&s_hist[join_bucket(uid[u], B)], 1u);
        if (!jt.isC) fold ^= uid[u];
      }
    }
    if (bad) fail(cm.status, ERR_INVALID);
    if (!jt.isC) {
      fold = wave_xor(fold);
      if (lane_id() == 0 && fold)
        atomicXor((unsigned long long*)&cm.fold[jt.s * FOLD_SLOTS + (t * WAVES + wave_id()) % FOLD_SLOTS],
                  (unsigned long long)fold);
    }
    __syncthreads();
    uint32_t* dst = a.cnt + jepre[jt.s] + jt.lt;
    for (uint64_t b = threadIdx.x; b < B; b += BLOCK) dst[b * g.jT] = s_hist[b];
    __syncthreads();
  }
}

struct JCntIn {
  const uint32_t* a;
  __device__ uint64_t operator()(int64_t i) const { return a[i]; }
};

// J3: scatter (uid, item) pairs into their buckets.
__global__ __launch_bounds__(BLOCK) void k_join_scatter(JoinArgs a, const Seg* __restrict__ segs,
                                                        const uint64_t* __restrict__ tpre,
                                                        const uint64_t* __restrict__ cpre,
                                                        const uint64_t* __restrict__ rpre,
                                                        const uint64_t* __restrict__ jepre,
                                                        const uint64_t* __restrict__ cnt_pre) {
  __shared__ uint32_t s_off[JB_MAX];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Tt = cm.meta[10];
  const uint64_t Ct = (uint64_t)cm.meta[0];
  for (int64_t t = blockIdx.x; t < Tt; t += gridDim.x) {
    const JTile jt = join_tile(segs, tpre, cm.nseg, t);
    const Seg& g = segs[jt.s];
    const uint64_t B = g.jB;
    const uint64_t* src = cnt_pre + jepre[jt.s] + jt.lt;
    // bucket starts relative to the segment's first entry (fits 32 bits:
    // a segment holds < 2^28 + 2^28 items)
    const uint64_t seg0 = uniform64(cnt_pre[jepre[jt.s]]);
    for (uint64_t b = threadIdx.x; b < B; b += BLOCK) s_off[b] = (uint32_t)(src[b * g.jT] - seg0);
    __syncthreads();
    const uint64_t gbase = jt.isC ? cpre[jt.s] : Ct + rpre[jt.s];
    // the tile's uids: from its side's keys (every second word) or from the
    // count pass's copies
    const uint64_t* keys = jt.isC ? a.ckeys : a.rkeys;
    const uint64_t* usrc = keys ? keys + 2 * (jt.isC ? cpre[jt.s] : rpre[jt.s]) : a.juid + gbase;
    const uint64_t ust = keys ? 2 : 1;
    // JS_U items per thread and pass, their uids loaded together; each pair
    // goes out as one 16-byte store
    for (uint64_t i0 = jt.i0; i0 < jt.i1; i0 += (uint64_t)BLOCK * JS_U) {
      uint64_t uid[JS_U];
#pragma unroll
      for (int u = 0; u < JS_U; ++u) {
        const uint64_t i = i0 + threadIdx.x + (uint64_t)u * BLOCK;
        uid[u] = usrc[ust * (i < jt.i1 ? i : jt.i1 - 1)];
      }
#pragma unroll
      for (int u = 0; u < JS_U; ++u) {
        const uint64_t i = i0 + threadIdx.x + (uint64_t)u * BLOCK;
        if (i < jt.i1) {
          const uint32_t pos = atomicAdd(&s_off[join_bucket(uid[u], B)], 1u);
          *reinterpret_cast<Pair*>(a.part + 2 * (seg0 + pos)) = Pair{uid[u], gbase + i};
        }
      }
    }
    __syncthreads();
  }
}

// A bucket with more items than LDS holds, joined by its block alone in an
// open-addressing table of its own in global memory: slots [4 p0, 4 p0 + H)
// of the table array, H = pow2ceil(2 n) <= 4 n (so buckets never share
// slots).  Same results as the LDS join: a current and a reference item with
// equal uids are partners; a second item of one side is a duplicate.
__device__ void join_bucket_global(const JoinArgs& a, uint64_t p0, uint32_t n, uint64_t Ct, uint64_t cbase) {
  const Common& cm = a.cm;
  Entry* tab = a.tab + 4 * p0;
  uint32_t H = 1;
  while (H < 2 * n) H <<= 1;
  for (uint32_t h = threadIdx.x; h < H; h += BLOCK) {
    tab[h].key = 0;
    tab[h].ci = NONE;
    tab[h].ri = NONE;
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n; k += BLOCK) {
    const Pair pr = *reinterpret_cast<const Pair*>(a.part + 2 * (p0 + k));
    uint32_t h = (uint32_t)mix64(pr.uid) & (H - 1);
    for (uint32_t probe = 0; probe < H; ++probe) {
      const unsigned long long prev = atomicCAS(&tab[h].key, 0ull, (unsigned long long)pr.uid);
      if (prev == 0ull || prev == (unsigned long long)pr.uid) {
        uint32_t* ip = pr.item >= Ct ? &tab[h].ri : &tab[h].ci;
        if (atomicCAS(ip, NONE, (uint32_t)pr.item) != NONE) fail(cm.status, ERR_INVALID);  // duplicate uid
        break;
      }
      h = (h + 1) & (H - 1);
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n; k += BLOCK) {
    const Pair pr = *reinterpret_cast<const Pair*>(a.part + 2 * (p0 + k));
    uint32_t h = (uint32_t)mix64(pr.uid) & (H - 1);
    for (uint32_t probe = 0; probe < H && tab[h].key != pr.uid; ++probe) h = (h + 1) & (H - 1);
    const bool isR = pr.item >= Ct;
    const uint32_t partner = isR ? tab[h].ci : tab[h].ri;
    if (isR) a.m[pr.item - Ct] = partner != NONE ? (int32_t)(partner - cbase) : -1;
    else a.cflag[pr.item] = partner != NONE ? 1 : 0;
  }
  __syncthreads();
}

// J4: one block per bucket: an LDS hash table pairs current and reference
// items with equal uids; a second item of the same side, or a third item,
// is a duplicate.
__global__ __launch_bounds__(BLOCK) void k_join_bucket(JoinArgs a, const Seg* __restrict__ segs,
                                                       const uint64_t* __restrict__ bpre,
                                                       const uint64_t* __restrict__ cpre,
                                                       const uint64_t* __restrict__ jepre,
                                                       const uint64_t* __restrict__ cnt_pre) {
  __shared__ uint64_t s_uid[JCAP];
  __shared__ uint32_t s_id[JCAP];
  __shared__ uint32_t s_partner[JCAP];
  __shared__ uint32_t s_tab[JTAB];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Bt = cm.meta[12];
  const uint64_t Ct = (uint64_t)cm.meta[0];
  for (int64_t bk = blockIdx.x; bk < Bt; bk += gridDim.x) {
    const int64_t s = (int64_t)uniform32((uint32_t)last_le<uint64_t>(bpre, 0, cm.nseg, (uint64_t)bk));
    const Seg& g = segs[s];
    const uint64_t b = (uint64_t)bk - bpre[s];
    const uint64_t p0 = uniform64(cnt_pre[jepre[s] + b * g.jT]), p1 = uniform64(cnt_pre[jepre[s] + (b + 1) * g.jT]);
    const uint32_t n = (uint32_t)(p1 - p0);
    if (n > JCAP) {  // uniform: a bucket too large for LDS joins in global memory
      join_bucket_global(a, p0, n, Ct, cpre[s]);
      continue;
    }
    // JC_U pairs per thread at a time, loaded before any is stored to LDS
    for (uint32_t k0 = threadIdx.x; k0 < n; k0 += BLOCK * JC_U) {
      Pair pr[JC_U];
#pragma unroll
      for (int u = 0; u < JC_U; ++u) {
        const uint32_t k = k0 + u * BLOCK;
        pr[u] = *reinterpret_cast<const Pair*>(a.part + 2 * (p0 + (k < n ? k : n - 1)));
      }
#pragma unroll
      for (int u = 0; u < JC_U; ++u) {
        const uint32_t k = k0 + u * BLOCK;
        if (k < n) {
          s_uid[k] = pr[u].uid;
          s_id[k] = (uint32_t)pr[u].item;
          s_partner[k] = NONE;
        }
      }
    }
    for (uint32_t k = threadIdx.x; k < JTAB; k += BLOCK) s_tab[k] = 0;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < n; k += BLOCK) {
      const uint64_t uid = s_uid[k];
      uint32_t h = (uint32_t)(mix64(uid) >> 40) & (JTAB - 1);
      for (int probe = 0; probe < JTAB; ++probe) {
        const uint32_t old = atomicCAS(&s_tab[h], 0u, k + 1);
        if (old == 0) break;
        const uint32_t o = old - 1;
        if (s_uid[o] == uid) {
          if ((s_id[k] >= Ct) == (s_id[o] >= Ct) || atomicCAS(&s_partner[o], NONE, k) != NONE) {
            fail(cm.status, ERR_INVALID);  // duplicate uid
          } else {
            s_partner[k] = o;
          }
          break;
        }
        h = (h + 1) & (JTAB - 1);
      }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < n; k += BLOCK) {
      const uint32_t id = s_id[k], p = s_partner[k];
      const bool matched = p != NONE;  // same uid; the headers are compared by RMatchIn
      if (id >= Ct) {
        a.m[id - Ct] = matched ? (int32_t)(s_id[p] - cpre[s]) : -1;
      } else {
        a.cflag[id] = matched ? 1 : 0;
      }
    }
    __syncthreads();
  }
}

// count << 34 | words of matched reference slots.  A slot is matched when
// its uid was found in the current message and the two header words are
// equal; a uid match with another header is undone here (the slot becomes
// unmatched, the current record new).  Reference slots and their partners
// run in the same order, so both header reads are close to sequential.
// Loaded in stages for the scan's rounds together: partners and segments,
// then segment bounds, sizes and reference headers, then partner headers.
struct RMatchIn {
  static constexpr int ROUNDS = 16;  // a tile of 8192 slots: fewer tiles to look back over
  Common cm;
  int32_t* m;
  const uint32_t* rwords;
  const uint64_t* jhdr;  // [C+R] header words: current records, then reference slots
  uint8_t* cflag;
  const uint64_t* ckeys;  // nullable: the current records' header words are read from these
  const uint64_t* rkeys;  // nullable: the same for the reference slots
  int64_t lo = 0, hi = 0;  // segments of the wave's slots
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(cm.rpre, 0, cm.nseg, (uint64_t)first);
    hi = wave_last_le<uint64_t>(cm.rpre, lo, cm.nseg, (uint64_t)last);
  }
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    const uint64_t Ct = (uint64_t)cm.meta[0];
    const uint64_t* hdr_r = rkeys ? rkeys + 1 : jhdr + Ct;
    const uint64_t* hdr_c = ckeys ? ckeys + 1 : jhdr;
    const uint64_t rst = rkeys ? 2 : 1, cst = ckeys ? 2 : 1;
    int64_t g[R], s[R];
    int32_t mi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      g[r] = i < n ? i : n - 1;
      mi[r] = m[g[r]];
      s[r] = lo == hi ? lo : last_le<uint64_t>(cm.rpre, lo, hi + 1, (uint64_t)g[r]);
    }
    __builtin_amdgcn_sched_barrier(0);
    uint64_t nc[R], cp[R], hr[R];
    uint32_t rw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      nc[r] = cm.seg[s[r]].nc;
      cp[r] = cm.cpre[s[r]];
      rw[r] = rwords[g[r]];
      hr[r] = hdr_r[rst * (uint64_t)g[r]];
    }
    __builtin_amdgcn_sched_barrier(0);
    // (after an earlier error the join may not have run: stay inside the segment)
    bool ok[R];
    uint64_t hc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ok[r] = mi[r] >= 0 && (uint64_t)mi[r] < nc[r];
      hc[r] = ok[r] ? hdr_c[cst * (cp[r] + (uint64_t)mi[r])] : 0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ok[r] && hc[r] != hr[r]) {
        m[g[r]] = -1;
        cflag[cp[r] + (uint64_t)mi[r]] = 0;
        ok[r] = false;
      }
      v[r] = ok[r] && wbase + r * WAVE + l < n ? (1ull << PK) | rw[r] : 0;
    }
  }
};
struct CNewIn {  // count << 34 | words of new current records; nlist[rank] = index of each new record
  static constexpr int ROUNDS = 16;  // a tile of 8192 records
  const uint8_t* cflag;
  const uint32_t* cwords;
  uint32_t* nlist;
  __device__ uint64_t operator()(int64_t g) const {
    const uint64_t w = cwords[g];
    return cflag[g] ? 0 : ((1ull << PK) | w);
  }
  __device__ void emit(int64_t g, uint64_t excl, uint64_t v) const {
    if (v) nlist[excl >> PK] = (uint32_t)g;
  }
};

// Per segment layout after matching (one thread per segment); the sizes
// are scanned by k_scan_cols, then k_enc_seg3 places the C' messages.
__device__ void enc_seg2(Common cm, const uint64_t* rscan, const uint64_t* cscan,
                         uint64_t* mstart) {
  if (status_of(cm.status) & ANY_ERR) {
    // sizes of zero: the scans that follow stay within their arrays
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * blockDim.x)
      for (int c = 0; c < 4; ++c) col(cm, c)[s] = 0;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cm.meta[5] = (int64_t)(rscan[cm.meta[1]] >> PK);
    cm.meta[6] = (int64_t)(cscan[cm.meta[0]] >> PK);
    cm.npre[cm.nseg] = (uint64_t)cm.meta[6];
    cm.meta[7] = (int64_t)(cscan[cm.meta[0]] & WMASK);
    mstart[cm.meta[5]] = rscan[cm.meta[1]] & WMASK;  // end of the last matched record
  }
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * blockDim.x) {
    Seg& g = cm.seg[s];
    g.fold = fold_of(cm.fold + s * FOLD_SLOTS);
    const uint64_t rs = rscan[cm.rpre[s]], re = rscan[cm.rpre[s + 1]];
    const uint64_t cs = cscan[cm.cpre[s]], ce = cscan[cm.cpre[s + 1]];
    g.mbase = rs >> PK;
    g.n_match = (re >> PK) - g.mbase;
    g.dbase = rs & WMASK;
    g.W = (re & WMASK) - g.dbase;
    g.nbase = cs >> PK;
    g.n_new = (ce >> PK) - g.nbase;
    cm.npre[s] = g.nbase;
    g.npbase = cs & WMASK;
    g.new_words = (ce & WMASK) - g.npbase;
    const uint64_t G = (g.W + 63) / 64, PG = (g.nr + 63) / 64;
    g.G = G;
    g.PG = PG;
    const uint64_t fixed = 64 + 8 * PG + 8 * G + round8(G) + round8(4 * g.n_new) + 8 * g.new_words;
    g.fixed = fixed;
    col(cm, 0)[s] = G;
    col(cm, 1)[s] = fixed;
    col(cm, 2)[s] = tam1_size(g.n_match + g.n_new, g.W + g.new_words);
    col(cm, 3)[s] = PG;
  }
}

__global__ __launch_bounds__(BLOCK) void k_enc_seg2(Common cm, const uint64_t* rscan, const uint64_t* cscan,
                                                    uint64_t* mstart) {
  enc_seg2(cm, rscan, cscan, mstart);
}

// C' offsets and headers (the prefixes of k_enc_seg2's sizes are in).
__device__ void enc_seg3(Common cm, uint8_t* newref, int64_t newref_cap,
                         int64_t* newref_off, uint64_t* gex) {
  if (status_of(cm.status) & ANY_ERR) return;
  const bool fits = cm.opre[cm.nseg] <= (uint64_t)newref_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    newref_off[cm.nseg] = (int64_t)cm.opre[cm.nseg];
    gex[cm.meta[3]] = 0;
    if (!fits) fail(cm.status, ERR_CAPACITY);
  }
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * blockDim.x) {
    Seg& g = cm.seg[s];
    const uint64_t oref = cm.opre[s];
    g.fixed_excl = cm.fxpre[s];
    g.oref = oref;
    const uint64_t n = g.n_match + g.n_new;
    g.cpw = (oref + 32 + 8 * ((n + 1) / 2)) / 8 - g.dbase;
    newref_off[s] = (int64_t)oref;
    if (!fits) continue;
    uint8_t* o = newref + oref;
    uint64_t* h = reinterpret_cast<uint64_t*>(o);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);
    h[1] = n;
    h[2] = g.W + g.new_words;
    h[3] = 0;
    if (n & 1) *reinterpret_cast<uint32_t*>(o + 32 + 4 * n) = 0;
  }
}

__global__ __launch_bounds__(BLOCK) void k_enc_seg3(Common cm, uint8_t* newref, int64_t newref_cap,
                                                    int64_t* newref_off, uint64_t* gex) {
  enc_seg3(cm, newref, newref_cap, newref_off, gex);
}

// Directory of matched records; C' offsets of matched records.
// Groups whose first residual word lies in a matched record (local words
// [q0, q0+w)) of segment s: remember the segment, so a group's wave finds it
// without searching.
__device__ inline void map_groups(const Common& cm, int64_t s, uint64_t q0, uint64_t w, uint32_t* gseg,
                                  uint32_t* gfirst = nullptr, uint64_t k = 0) {
  for (uint64_t lg = (q0 + 63) / 64; 64 * lg < q0 + w; ++lg) {
    gseg[cm.gpre[s] + lg] = (uint32_t)s;
    if (gfirst) gfirst[cm.gpre[s] + lg] = (uint32_t)k;  // the matched record holding the group's first word
  }
}

// Decoder: descriptors of the groups whose first residual word lies in
// matched record k (local residual words [q0, q0 + w) of segment s).  The
// group's bitmap and size byte are read from the encoding's tables (inside
// it: the header checks passed); its block offset is the segment's block
// area plus the prefix of the group sizes within the segment.
__device__ inline void map_groups_dec(const Common& cm, const Seg& sg, int64_t s, uint64_t q0, uint64_t w,
                                      uint64_t k, const uint8_t* enc, const uint64_t* gex, GDesc* gd) {
  for (uint64_t lg = (q0 + 63) / 64; 64 * lg < q0 + w; ++lg) {
    const uint64_t gg = cm.gpre[s] + lg;
    const uint8_t* e = enc + sg.encm;
    const uint32_t byte = e[64 + 8 * sg.PG + 8 * sg.G + lg];
    const uint32_t md = (uint32_t)sg.mode;
    GDesc d;
    d.blk = sg.encm + sg.fixed + (gex[gg] - gex[cm.gpre[s]]);
    d.bm = ld64(e + 64 + 8 * sg.PG + 8 * lg);
    d.out = sg.cpw + sg.dbase + 64 * lg;
    d.g0w = sg.dbase + 64 * lg;
    d.rbw = sg.rbody / 8;
    d.k0 = (uint32_t)k;
    d.size = 8u * (md == 2 ? byte & 0x7Fu : byte);
    d.nlive = (uint32_t)(sg.W - 64 * lg < 64 ? sg.W - 64 * lg : 64);
    d.usep = md == 1 || (md == 2 && (byte >> 7)) ? 1u : 0u;
    d.pad[0] = d.pad[1] = 0;
    ulonglong2* dst = reinterpret_cast<ulonglong2*>(gd + gg);
    const ulonglong2* src = reinterpret_cast<const ulonglong2*>(&d);
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = src[i];
  }
}

// Learned calls: the neighbour table's entries cleared whole, as 16-byte
// stores (the table is 256-byte aligned), by the grid of the pass that runs
// before the table is built; hist_cap must cover every reference slot.
__device__ inline void nbr_clear(const Common& cm, Entry* tab, int64_t hist_cap) {
  if (hist_cap < cm.meta[1]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fail(cm.status, ERR_INVALID);
    return;
  }
  static_assert(sizeof(Entry) == 16, "one 16-byte store per entry");
  const int64_t H = cm.meta[2];
  ulonglong2* t = reinterpret_cast<ulonglong2*>(tab);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < H; i += (int64_t)gridDim.x * blockDim.x)
    t[i] = ulonglong2{0, 0};
}

// Directory of the matched records, in C' order: C and R word, residual
// start, slot (learned mode), or the C and R word offsets in the segment's
// record areas (plain mode); C' offsets; groups' segment and first record.
// A wave takes RS_U * 64 consecutive reference slots per pass and issues
// their loads in two stages before it stores anything.  Learned calls (ntab
// set) then clear the neighbour table.  Six waves per SIMD: the pass is
// bound by its loads in flight, and at 81 registers it ran at five (23 ->
// 29 us on 1.5e6 slots).
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void k_enc_mdir(Common cm, const uint8_t* cur, const uint8_t* ref,
                                                    const int32_t* m, const uint64_t* rscan, const uint32_t* rwords,
                                                    MDir* mdir, uint64_t* crw, uint64_t* mstart, uint8_t* newref,
                                                    uint32_t* gseg, uint32_t* gfirst, const uint64_t* juid,
                                                    const uint64_t* jhdr, const uint64_t* rkeys, uint64_t* okeys,
                                                    uint64_t okeys_cap, Entry* ntab, int64_t hist_cap) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  const int l = lane_id();
  constexpr int64_t SPAN = (int64_t)WAVE * RS_U;
  const int64_t nwv = (int64_t)gridDim.x * WAVES;
  for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave_id()) * SPAN; base < Rt; base += nwv * SPAN) {
    const int64_t last = base + SPAN - 1 < Rt ? base + SPAN - 1 : Rt - 1;
    const int64_t lo = wave_last_le<uint64_t>(cm.rpre, 0, cm.nseg, (uint64_t)base);
    const int64_t hi = wave_last_le<uint64_t>(cm.rpre, lo, cm.nseg, (uint64_t)last);
    // slot values, the R offset and the C offset (of the message header for
    // an unmatched slot: always there); slots past the end read the last one
    int64_t sv[RS_U];
    int32_t iv[RS_U];
    uint64_t rsv[RS_U];
    uint32_t rwv[RS_U], roff[RS_U], coff[RS_U];
#pragma unroll
    for (int u = 0; u < RS_U; ++u) {
      const int64_t g = base + (int64_t)u * WAVE + l;
      const int64_t gc = g <= last ? g : last;
      const int64_t sx = lo == hi ? lo : last_le<uint64_t>(cm.rpre, lo, hi + 1, (uint64_t)gc);
      sv[u] = sx;
      iv[u] = m[gc];
      rsv[u] = rscan[gc];
      rwv[u] = rwords[gc];
      roff[u] = ld32(ref + cm.seg[sx].rmsg + 32 + 4 * ((uint64_t)gc - cm.rpre[sx]));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < RS_U; ++u) {
      const Seg& sg = cm.seg[sv[u]];
      coff[u] = ld32(cur + sg.cmsg + (iv[u] >= 0 ? 32 + 4 * (uint64_t)iv[u] : 0));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < RS_U; ++u) {
      const int64_t g = base + (int64_t)u * WAVE + l;
      if (g > last || iv[u] < 0) continue;
      const int64_t sx = sv[u];
      const Seg& sg = cm.seg[sx];
      const uint64_t k = rsv[u] >> PK;
      const uint64_t d = rsv[u] & WMASK;
      if (mdir) {  // learned mode or a history to write: the full entry
        mdir[k] = MDir{sg.rbody / 8 + roff[u], (uint64_t)g | ((uint64_t)sx << 34)};
      }
      if (crw) crw[k] = (uint64_t)coff[u] | ((uint64_t)roff[u] << 32);
      if (okeys) {  // C' record k + (new records of earlier segments): the slot's uid and header
        const uint64_t Ct = (uint64_t)cm.meta[0], o = k + cm.npre[sx];
        if (o < okeys_cap)
          *reinterpret_cast<ulonglong2*>(okeys + 2 * o) =
              rkeys ? *reinterpret_cast<const ulonglong2*>(rkeys + 2 * (uint64_t)g)
                    : ulonglong2{juid[Ct + (uint64_t)g], jhdr[Ct + (uint64_t)g]};
        else
          fail(cm.status, ERR_CAPACITY);
      }
      mstart[k] = d;
      *reinterpret_cast<uint32_t*>(newref + sg.oref + 32 + 4 * (k - sg.mbase)) = (uint32_t)(d - sg.dbase);
      map_groups(cm, sx, d - sg.dbase, rwv[u], gseg, gfirst, k);
    }
  }
  if (ntab) nbr_clear(cm, ntab, hist_cap);
}

// Assemble the block of one group in LDS (b64: BLK_MAX/8 + 1 words).
// Every lane ORs its nibble and its significant bytes into the 64-bit words
// they fall in (one or two words: no byte stores).  Returns the block size in
// bytes.
// The same block from values the caller already has: the word's length in
// bytes, the inclusive scan of the lengths over the wave, the group's bitmap
// and block size.
__device__ inline void build_block_from(uint64_t D, uint32_t len, uint32_t sig_incl, uint64_t bm, uint32_t size,
                                        uint64_t* b64) {
  const int l = lane_id();
  const uint32_t nib = ((uint32_t)__popcll(bm) + 1) / 2;
  for (uint32_t k = l; k < size / 8; k += WAVE) b64[k] = 0;
  wave_sync();
  if (D) {
    const uint32_t t = __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
    atomicOr((unsigned long long*)&b64[t / 16], (unsigned long long)len << (4 * (t % 16)));
    const uint32_t so = nib + sig_incl - len;
    const uint32_t sh = 8 * (so % 8);
    atomicOr((unsigned long long*)&b64[so / 8], (unsigned long long)(D << sh));
    if (sh && sh + 8 * len > 64) atomicOr((unsigned long long*)&b64[so / 8 + 1], (unsigned long long)(D >> (64 - sh)));
  }
  wave_sync();
}

__device__ inline uint32_t build_block(uint64_t D, uint64_t* b64, uint64_t* bitmap_out) {
  const int l = lane_id();
  const uint64_t bm = __ballot(D != 0);
  const uint32_t len = D ? (uint32_t)(8 - (__clzll((long long)D) >> 3)) : 0u;
  const uint32_t popc = (uint32_t)__popcll(bm);
  const uint32_t nib = (popc + 1) / 2;
  const uint32_t sig_incl = wave_incl_scan32(len);
  const uint32_t sig_tot = (uint32_t)__builtin_amdgcn_readlane((int)sig_incl, 63);
  const uint32_t size = (nib + sig_tot + 7) & ~7u;
  for (uint32_t k = l; k < size / 8; k += WAVE) b64[k] = 0;
  wave_sync();
  if (D) {
    // nibble t (t-th non-zero word): byte t/2, low nibble first = bits 4t of the block
    const uint32_t t = (uint32_t)__popcll(bm & lanemask_lt(l));
    atomicOr((unsigned long long*)&b64[t / 16], (unsigned long long)len << (4 * (t % 16)));
    const uint32_t so = nib + sig_incl - len;
    const uint32_t sh = 8 * (so % 8);
    atomicOr((unsigned long long*)&b64[so / 8], (unsigned long long)(D << sh));
    if (sh && sh + 8 * len > 64) atomicOr((unsigned long long*)&b64[so / 8 + 1], (unsigned long long)(D >> (64 - sh)));
  }
  wave_sync();
  *bitmap_out = bm;
  return size;
}

// Largest i < n with a[i] <= x (a non-decreasing, a[0] <= x): a search in LDS.
__device__ inline int lds_last_le(const uint64_t* a, int n, uint64_t x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (a[m] <= x) lo = m;
    else hi = m;
  }
  return lo;
}

// New records a wave copies (up to 64): word prefix within the wave (q[n]
// = total), first source word, first destination words (uint64 indices).
struct NewTab {
  uint64_t q[WAVE + 1];
  uint64_t src[WAVE];
  uint64_t dst1[WAVE];
  uint64_t dst2[WAVE];
  uint64_t kidx[WAVE];  // decoder: the record's index among all C' records (for its key)
};

#ifndef TA_UNPACK_PG
#define TA_UNPACK_PG 1
#endif
constexpr int UNPACK_PG = TA_UNPACK_PG;  // the decoder's groups per wave at a time

// Residual and packing in one pass.  A wave takes EG_R consecutive 64-word
// groups; for each, the matched records overlapping it (at most 33, one per
// lane, lane 0 holding the one with the group's first word) give every
// word's C and R words: C goes to C', D = C xor R stays in registers with
// its block size.  Learned calls also form D2 = C xor X (X: the prediction
// for predicted words, else R) and keep the smaller block.  Tiles of EG_TILE groups (one block) are
// handed out in order and join a decoupled look-back over their block
// bytes, which gives every group's block offset; then each group's block is
// built in LDS and written in place.  The dense residual never goes to
// memory.
#ifndef TA_EG_R
#define TA_EG_R 4
#endif
#ifndef TA_EG_BLOCK
#define TA_EG_BLOCK 512
#endif
constexpr int EG_R = TA_EG_R;                 // groups per wave and tile
constexpr int EG_BLOCK = TA_EG_BLOCK;         // threads per block
constexpr int EG_WAVES = EG_BLOCK / WAVE;
constexpr int EG_TILE = EG_WAVES * EG_R;      // groups per tile

struct GroupArgs {
  Common cm;
  const uint64_t* cur;     // (words)
  const uint64_t* ref;     // (words)
  const uint64_t* crw;     // [matched] C and R word offsets of every matched record (in the record areas)
  const uint64_t* mstart;  // [matched+1] residual start of every matched record
  uint64_t* newref;        // C' (words)
  uint8_t* enc;
  int64_t enc_cap;
  uint64_t* bm;   // [groups] word bitmaps (learned: of the variant written)
  uint8_t* gsz;   // [groups] block sizes / 8 (learned: the smaller variant's)
  uint64_t* gex;  // [groups+1] exclusive prefix of block bytes (gex[groups] = total)
  // learned calls only
  const uint64_t* pred_x;  // [matched][4] predicted words 2..5
  const uint8_t* pred_on;  // [matched] the record's words 2..5 are predicted
  uint8_t* gch;            // [groups] bits 0-1: 0 plain block written, 1 learned block (strictly
                           // smaller), 2 plain block written for a tie whose learned block differs;
                           // bit 2: the learned block is smaller, bit 3: the plain block is smaller
};

// Learned calls: the group's variant.  The block of a group is the smaller
// one (learned on a strict win); a tie keeps the plain bytes unless its
// segment turns out to be learned (mode 1), which k_enc_fixup handles.  The
// size and so every block offset is min(plain, learned) whatever the
// segment's mode.  The group's choice byte also says which block was
// smaller; k_choose_mode reduces those bits per segment (no atomics on the
// segments' words while the groups are formed).
constexpr uint8_t GCH_VARIANT = 3, GCH_LEARNED_SMALLER = 4, GCH_PLAIN_SMALLER = 8;

// (segs, gpre, gseg, gfirst: read-only here; as restrict parameters their
// uniform reads become scalar loads.  The learned kernel is held to six
// waves per SIMD, as the plain one has by itself: 75 registers, no spill.)
template <int OP, bool LRN>
__global__ __launch_bounds__(EG_BLOCK) __attribute__((amdgpu_waves_per_eu(LRN ? 6 : 1))) void k_enc_groups(GroupArgs a, const Seg* __restrict__ segs,
                                                         const uint64_t* __restrict__ gpre,
                                                         const uint32_t* __restrict__ gseg,
                                                         const uint32_t* __restrict__ gfirst, LookBack lb) {
  constexpr int BW = BLK_MAX / 8 + 1;
  __shared__ uint64_t s_blk[EG_WAVES][BW];
  __shared__ uint32_t s_mark[EG_WAVES][EG_R][WAVE];  // record-start marks: group index + 1
  __shared__ uint64_t s_wave[EG_WAVES];
  __shared__ uint32_t s_ticket;
  __shared__ uint64_t s_prefix;
  lb_clear_next(lb);
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Gt = cm.meta[3], M = cm.meta[5];
  if (Gt <= 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.gex[0] = 0;
    return;
  }
  const int64_t ntiles = (Gt + EG_TILE - 1) / EG_TILE;
  // blocks beyond the tile count leave before taking a ticket
  if ((int64_t)blockIdx.x >= ntiles) return;
  const int l = lane_id(), wv = wave_id();
  const uint64_t le_mask = lanemask_le(l);
#pragma unroll
  for (int x = 0; x < EG_R; ++x) s_mark[wv][x][l] = 0;  // no group's tag
  wave_sync();
  // Tiles are pipelined: a block computes a new tile and publishes its
  // aggregate before it finishes the previous one (look-back, then blocks),
  // so the wait for predecessors overlaps the next tile's loads.
  bool have = false;  // a computed tile waiting for its prefix
  uint32_t tp = 0;
  uint64_t Dp[EG_R], woffp = 0, totp = 0;
  uint32_t szp[EG_R], incp[EG_R];
#pragma unroll
  for (int x = 0; x < EG_R; ++x) {
    Dp[x] = 0;
    szp[x] = incp[x] = 0;
  }
  for (;;) {
    const uint32_t t = lb_take_ticket(lb, &s_ticket);
    const bool got = (int64_t)t < ntiles;  // the same in the whole block
    uint64_t D[EG_R];
    uint32_t size[EG_R], inclv[EG_R];
    uint64_t woff = 0, tot = 0;
    if (got) {
      const int64_t g0 = (int64_t)t * EG_TILE + (int64_t)wv * EG_R;
      // The wave's groups in steps, each issuing its loads for every group
      // before any is used: record tables, then C and R words.  Groups past the
      // end work on the last group (clamped: no branch around loads) and store
      // nothing.
      int64_t gc[EG_R];
      bool gv[EG_R], has[EG_R];
      uint64_t mst[EG_R], cwd[EG_R], rwd[EG_R], k0v[EG_R];
      uint32_t pon[EG_R];
#pragma unroll
      for (int x = 0; x < EG_R; ++x) {
        gv[x] = g0 + x < Gt;
        gc[x] = gv[x] ? g0 + x : Gt - 1;
        // lane i <= 32: start, C word and R word of record k0 + i (a group
        // implies a matched record, so M >= 1 and the clamped index is valid)
        const uint64_t k0 = uniform32(gfirst[gc[x]]);
        k0v[x] = k0;
        has[x] = l <= 32 && k0 + l < (uint64_t)M;
        const uint64_t kk = has[x] ? k0 + l : (uint64_t)M - 1;
        mst[x] = a.mstart[kk];
        const uint64_t crw = a.crw[kk];
        cwd[x] = (uint32_t)crw;
        rwd[x] = crw >> 32;
        pon[x] = LRN ? (uint32_t)a.pred_on[kk] : 0u;
      }
      __builtin_amdgcn_sched_barrier(0);
      // start relative to the group (clamped to [-2^30, 64]), words relative to
      // the segment's record areas; lanes 1..32 mark the starts inside the group
      int relv[EG_R];
      uint32_t cwv[EG_R], rwv[EG_R];
#pragma unroll
      for (int x = 0; x < EG_R; ++x) {
        const int64_t sx = (int64_t)uniform32(gseg[gc[x]]);
        const Seg& sg = segs[sx];
        const uint64_t g0w = uniform64(sg.dbase + 64 * ((uint64_t)gc[x] - gpre[sx]));  // first residual position
        const int64_t r = (int64_t)mst[x] - (int64_t)g0w;
        relv[x] = !has[x] ? 64 : (r > 64 ? 64 : (r < -(1 << 30) ? -(1 << 30) : (int)r));
        cwv[x] = (uint32_t)cwd[x];
        rwv[x] = (uint32_t)rwd[x];
        if (l >= 1 && relv[x] >= 1 && relv[x] < WAVE) s_mark[wv][x][relv[x]] = (uint32_t)gc[x] + 1;
      }
      wave_sync();
      uint64_t cv[EG_R], xv[EG_R], pv[EG_R];
      bool live[EG_R], prd[EG_R];
#pragma unroll
      for (int x = 0; x < EG_R; ++x) {
        const int64_t sx = (int64_t)uniform32(gseg[gc[x]]);
        const Seg& sg = segs[sx];
        const uint64_t lg = uniform64((uint64_t)gc[x] - gpre[sx]);
        const int rel = relv[x];
        const uint32_t cw = cwv[x], rw = rwv[x];
        const uint64_t starts = __ballot(s_mark[wv][x][l] == (uint32_t)gc[x] + 1);
        const int idx = __popcll(starts & le_mask);  // <= 32
        const uint32_t off = (uint32_t)(l - __shfl(rel, idx, WAVE));
        const uint32_t cwi = (uint32_t)__shfl((int)cw, idx, WAVE), rwi = (uint32_t)__shfl((int)rw, idx, WAVE);
        live[x] = gv[x] && 64 * lg + (uint64_t)l < sg.W;
        // (a word that is not live reads word 0 of lane 0's record, the one
        // holding the group's first word: in the segment, always valid)
        const uint32_t cw0 = (uint32_t)__builtin_amdgcn_readlane((int)cw, 0);
        const uint32_t rw0 = (uint32_t)__builtin_amdgcn_readlane((int)rw, 0);
        cv[x] = a.cur[uniform64(sg.cbody / 8) + (live[x] ? cwi + off : cw0)];
        xv[x] = a.ref[uniform64(sg.rbody / 8) + (live[x] ? rwi + off : rw0)];
        if constexpr (LRN) {
          // a predicted word (2..5 of a predicted record) is taken against the
          // prediction; others read prediction 0 (valid: M >= 1), unused
          prd[x] = live[x] && __shfl((int)pon[x], idx, WAVE) != 0 && off >= 2 && off < 6;
          pv[x] = a.pred_x[prd[x] ? 4 * (k0v[x] + (uint64_t)idx) + (off - 2) : 0];
        } else {
          prd[x] = false;
          pv[x] = 0;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // C' words, residual words and block sizes
      uint64_t wsum = 0;
#pragma unroll
      for (int x = 0; x < EG_R; ++x) {
        D[x] = live[x] ? diff_word<OP>(cv[x], xv[x]) : 0;
        const int64_t sx = (int64_t)uniform32(gseg[gc[x]]);
        const Seg& sg = segs[sx];
        if (live[x]) a.newref[sg.cpw + sg.dbase + 64 * ((uint64_t)gc[x] - gpre[sx]) + (uint64_t)l] = cv[x];
        uint64_t bmw = __ballot(D[x] != 0);
        const uint32_t len = D[x] ? (uint32_t)(8 - (__clzll((long long)D[x]) >> 3)) : 0u;
        inclv[x] = wave_incl_scan32(len);
        const uint32_t sig = (uint32_t)__builtin_amdgcn_readlane((int)inclv[x], 63);
        size[x] = gv[x] ? ((((uint32_t)__popcll(bmw) + 1) / 2 + sig + 7) & ~7u) : 0u;
        uint8_t choice = 0;
        if constexpr (LRN) {
          const uint64_t D2 = live[x] ? diff_word<OP>(cv[x], prd[x] ? pv[x] : xv[x]) : 0;
          const uint64_t bm2 = __ballot(D2 != 0);
          const uint32_t len2 = D2 ? (uint32_t)(8 - (__clzll((long long)D2) >> 3)) : 0u;
          const uint32_t incl2 = wave_incl_scan32(len2);
          const uint32_t sig2 = (uint32_t)__builtin_amdgcn_readlane((int)incl2, 63);
          const uint32_t size2 = gv[x] ? ((((uint32_t)__popcll(bm2) + 1) / 2 + sig2 + 7) & ~7u) : 0u;
          const uint8_t smaller = (size2 < size[x] ? GCH_LEARNED_SMALLER : 0) | (size[x] < size2 ? GCH_PLAIN_SMALLER : 0);
          if (size2 < size[x]) {  // uniform
            D[x] = D2;
            bmw = bm2;
            inclv[x] = incl2;
            size[x] = size2;
            choice = 1;
          } else if (size2 == size[x] && __ballot(D2 != D[x])) {
            choice = 2;
          }
          choice |= smaller;
        }
        if (gv[x] && l == 0) {
          a.bm[gc[x]] = bmw;
          a.gsz[gc[x]] = (uint8_t)(size[x] / 8);
          if constexpr (LRN) a.gch[gc[x]] = choice;
        }
        wsum += size[x];
      }
      // the tile's block bytes: waves, then its aggregate for the look-back
      if (l == 0) s_wave[wv] = wsum;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EG_WAVES; ++i) {
        woff += (i < wv) ? s_wave[i] : 0;
        tot += s_wave[i];
      }
      if (threadIdx.x == 0) lb_publish(lb, t, tot);
    }
    if (have) {  // the previous tile: its prefix, then its blocks
      if (threadIdx.x < WAVE) {
        const uint64_t e = lb_lookback(lb, tp, totp);
        if (threadIdx.x == 0) s_prefix = e;
      }
      __syncthreads();
      const int64_t g0p = (int64_t)tp * EG_TILE + (int64_t)wv * EG_R;
      // blocks: built in the wave's LDS buffer one at a time, written in place
      uint64_t pos = s_prefix + woffp;  // block bytes before this wave's first group
#pragma unroll
      for (int x = 0; x < EG_R; ++x) {
        const int64_t gg = g0p + x;
        if (gg >= Gt) break;
        if (l == 0) a.gex[gg] = pos;
        if (szp[x]) {
          const Seg& sg = segs[(int64_t)uniform32(gseg[gg])];
          const uint64_t at = uniform64(sg.fixed_excl + sg.fixed + pos);
          const uint32_t len = Dp[x] ? (uint32_t)(8 - (__clzll((long long)Dp[x]) >> 3)) : 0u;
          build_block_from(Dp[x], len, incp[x], __ballot(Dp[x] != 0), szp[x], s_blk[wv]);
          if (at + szp[x] > (uint64_t)a.enc_cap) {
            if (l == 0) fail(cm.status, ERR_CAPACITY);
          } else {
            uint64_t* dst = reinterpret_cast<uint64_t*>(a.enc + at);
            for (uint32_t w = l; w < szp[x] / 8; w += WAVE) dst[w] = s_blk[wv][w];
          }
          wave_sync();  // the buffer is rebuilt for the next group
        }
        pos += szp[x];
      }
      if ((int64_t)tp == ntiles - 1 && threadIdx.x == 0) a.gex[Gt] = s_prefix + totp;
    }
    __syncthreads();  // s_wave, s_prefix and the LDS buffers are reused
    if (!got) break;
    have = true;
    tp = t;
    woffp = woff;
    totp = tot;
    for (int x = 0; x < EG_R; ++x) {
      Dp[x] = D[x];
      szp[x] = size[x];
      incp[x] = inclv[x];
    }
  }
}

// Learned calls: each segment's mode from its groups' choice bytes -- plain
// (0) when no group's learned block is smaller, learned (1) when no group's
// plain block is smaller, else mixed (2) (a mixed encoding is never larger
// than either).  One block per segment ORs the bits of its groups, 16 bytes
// per thread and load where they are aligned.
__global__ __launch_bounds__(BLOCK) void k_choose_mode(Common cm, const uint8_t* gch) {
  __shared__ uint32_t s_or[WAVES];
  if (status_of(cm.status) & ANY_ERR) return;
  const int l = lane_id(), wv = wave_id();
  for (int64_t s = blockIdx.x; s < cm.nseg; s += gridDim.x) {
    const uint64_t g0 = cm.gpre[s], g1 = cm.gpre[s + 1];
    uint32_t f = 0;
    // the unaligned head and tail byte by byte, the aligned middle by 16 bytes
    const uint64_t a0 = (g0 + 15) & ~15ull, a1 = g1 & ~15ull;
    if (a0 >= a1) {
      for (uint64_t g = g0 + threadIdx.x; g < g1; g += BLOCK) f |= gch[g];
    } else {
      for (uint64_t g = g0 + threadIdx.x; g < a0; g += BLOCK) f |= gch[g];
      for (uint64_t g = a1 + threadIdx.x; g < g1; g += BLOCK) f |= gch[g];
      const uint4* v = reinterpret_cast<const uint4*>(gch + a0);
      for (uint64_t q = threadIdx.x; q < (a1 - a0) / 16; q += BLOCK) {
        const uint4 w = v[q];
        f |= w.x | w.y | w.z | w.w;
      }
    }
    f = (f | (f >> 8) | (f >> 16) | (f >> 24)) & (GCH_LEARNED_SMALLER | GCH_PLAIN_SMALLER);
    f = wave_or(f);
    if (l == 0) s_or[wv] = f;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int i = 0; i < WAVES; ++i) t |= s_or[i];
      cm.seg[s].mode = !(t & GCH_LEARNED_SMALLER) ? 0 : (!(t & GCH_PLAIN_SMALLER) ? 1 : 2);
    }
    __syncthreads();
  }
}

// Learned calls, after k_choose_mode: in a learned (mode 1) segment a group
// whose two blocks tie in size but differ was written with the plain bytes;
// its learned block replaces them (same size and offset) with its bitmap.
// One wave per such group; every other group is only looked at.
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_enc_fixup(GroupArgs a, const Seg* __restrict__ segs,
                                                     const uint64_t* __restrict__ gpre,
                                                     const uint32_t* __restrict__ gseg,
                                                     const uint32_t* __restrict__ gfirst) {
  __shared__ uint64_t s_blk[WAVES][BLK_MAX / 8 + 1];
  __shared__ uint32_t s_mark[WAVES][WAVE];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Gt = cm.meta[3], M = cm.meta[5];
  const int l = lane_id(), wv = wave_id();
  for (int64_t b0 = ((int64_t)blockIdx.x * WAVES + wv) * WAVE; b0 < Gt; b0 += (int64_t)gridDim.x * WAVES * WAVE) {
    const int64_t mine = b0 + l;
    bool todo = false;
    if (mine < Gt && (a.gch[mine] & GCH_VARIANT) == 2) todo = segs[gseg[mine]].mode == 1;
    uint64_t pending = __ballot(todo);
    while (pending) {
      const int lead = __ffsll((unsigned long long)pending) - 1;
      pending &= pending - 1;
      const int64_t gg = b0 + lead;
      const int64_t sx = (int64_t)uniform32(gseg[gg]);
      const Seg& sg = segs[sx];
      const uint64_t lg = (uint64_t)gg - gpre[sx];
      const uint64_t k0 = uniform32(gfirst[gg]);
      const bool has = l <= 32 && k0 + l < (uint64_t)M;
      const uint64_t kk = has ? k0 + l : (uint64_t)M - 1;
      const int64_t r = (int64_t)a.mstart[kk] - (int64_t)(sg.dbase + 64 * lg);
      const int rel = !has ? 64 : (r > 64 ? 64 : (r < -(1 << 30) ? -(1 << 30) : (int)r));
      const uint64_t crw = a.crw[kk];
      const uint32_t cw = (uint32_t)crw, rw = (uint32_t)(crw >> 32);
      const uint32_t pon = a.pred_on[kk];
      s_mark[wv][l] = 0;
      wave_sync();
      if (l >= 1 && rel >= 1 && rel < WAVE) s_mark[wv][rel] = 1;
      wave_sync();
      const uint64_t starts = __ballot(s_mark[wv][l] != 0);
      const int idx = __popcll(starts & lanemask_le(l));
      const uint32_t off = (uint32_t)(l - __shfl(rel, idx, WAVE));
      const bool live = 64 * lg + (uint64_t)l < sg.W;
      const uint32_t cwi = (uint32_t)__shfl((int)cw, idx, WAVE), rwi = (uint32_t)__shfl((int)rw, idx, WAVE);
      const uint32_t cw0 = (uint32_t)__builtin_amdgcn_readlane((int)cw, 0);
      const uint32_t rw0 = (uint32_t)__builtin_amdgcn_readlane((int)rw, 0);
      const uint64_t c = a.cur[sg.cbody / 8 + (live ? cwi + off : cw0)];
      const uint64_t x = a.ref[sg.rbody / 8 + (live ? rwi + off : rw0)];
      const bool prd = live && __shfl((int)pon, idx, WAVE) != 0 && off >= 2 && off < 6;
      const uint64_t pv = a.pred_x[prd ? 4 * (k0 + (uint64_t)idx) + (off - 2) : 0];
      const uint64_t D2 = live ? diff_word<OP>(c, prd ? pv : x) : 0;
      uint64_t bm2;
      const uint32_t size = build_block(D2, s_blk[wv], &bm2);
      if (l == 0) a.bm[gg] = bm2;
      const uint64_t at = sg.fixed_excl + sg.fixed + a.gex[gg];
      if (size && at + size <= (uint64_t)a.enc_cap) {
        uint64_t* dst = reinterpret_cast<uint64_t*>(a.enc + at);
        for (uint32_t w = l; w < size / 8; w += WAVE) dst[w] = s_blk[wv][w];
      }
      wave_sync();
    }
  }
}


// Copies of the words a wave tabulated in t (t.q[n] words in all), NC_U per
// lane in flight: all searches and loads first, then the stores.  dst2 may
// be null.
constexpr int NC_U = 4;
__device__ inline void copy_tab(const NewTab& t, int n, const uint64_t* src, uint64_t* dst1, uint64_t* dst2) {
  const uint64_t tot = t.q[n];
  for (uint64_t q0 = lane_id(); q0 < tot; q0 += NC_U * WAVE) {
    uint64_t v[NC_U], d1[NC_U], d2[NC_U];
#pragma unroll
    for (int j = 0; j < NC_U; ++j) {
      const uint64_t q = q0 + (uint64_t)j * WAVE < tot ? q0 + (uint64_t)j * WAVE : tot - 1;
      const int i = lds_last_le(t.q, n, q);
      const uint64_t w = q - t.q[i];
      v[j] = src[t.src[i] + w];
      d1[j] = t.dst1[i] + w;
      d2[j] = t.dst2[i] + w;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NC_U; ++j)
      if (q0 + (uint64_t)j * WAVE < tot) {
        dst1[d1[j]] = v[j];
        if (dst2) dst2[d2[j]] = v[j];
      }
  }
}

// New C records, 64 consecutive ones of the list the scan of new records
// wrote (so that runs of new records spread over many waves), from the
// wave's first rb: their sizes into the encoding's table, their C' offsets,
// and their words into the encoding and into C', copied lane-parallel
// (consecutive lanes, consecutive words) from a table in LDS.  The
// segment's encoding offset is taken from the group block prefix (encm).
__device__ inline void enc_new_wave(const Common& cm, int64_t rb, int64_t Nn, const uint64_t* cscan,
                                    const uint32_t* nlist, const uint32_t* cwords, const uint8_t* cur,
                                    uint8_t* enc, uint8_t* newref, const uint64_t* gex, const uint64_t* juid,
                                    const uint64_t* jhdr, const uint64_t* ckeys, uint64_t* okeys,
                                    uint64_t okeys_cap, NewTab& t) {
  const int l = lane_id();
  const int64_t k = rb + l;
  const int n = (int)(Nn - rb < WAVE ? Nn - rb : WAVE);
  const int64_t gc = nlist[k < Nn ? k : Nn - 1];
  const int64_t sg = wave_seg(cm.cpre, cm.nseg, (uint64_t)gc, readlane64((uint64_t)gc, 0),
                              readlane64((uint64_t)gc, n - 1));
  const Seg& g = cm.seg[sg];
  const uint64_t cs = cscan[gc];
  const uint64_t words = k < Nn ? cwords[gc] : 0;
  const uint32_t o = ld32(cur + g.cmsg + 32 + 4 * (uint64_t)(gc - (int64_t)cm.cpre[sg]));
  if (k < Nn) {
    const uint64_t encm = g.fixed_excl + gex[cm.gpre[sg]];
    const uint64_t r = (cs >> PK) - g.nbase;      // index among the segment's new records
    const uint64_t qs = (cs & WMASK) - g.npbase;  // word within the segment's new records
    const uint64_t nn = g.n_match + g.n_new;
    uint8_t* ns = enc + encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G);
    *reinterpret_cast<uint32_t*>(ns + 4 * r) = (uint32_t)words;
    if (r == g.n_new - 1 && (g.n_new & 1)) *reinterpret_cast<uint32_t*>(ns + 4 * (r + 1)) = 0;
    *reinterpret_cast<uint32_t*>(newref + g.oref + 32 + 4 * (g.n_match + r)) = (uint32_t)(g.W + qs);
    if (okeys) {  // C' record: after the segment's matched ones
      const uint64_t ko = g.mbase + g.nbase + g.n_match + r;
      if (ko < okeys_cap)
        *reinterpret_cast<ulonglong2*>(okeys + 2 * ko) =
            ckeys ? *reinterpret_cast<const ulonglong2*>(ckeys + 2 * (uint64_t)gc) : ulonglong2{juid[gc], jhdr[gc]};
      else fail(cm.status, ERR_CAPACITY);
    }
    t.src[l] = (g.cbody + 8 * (uint64_t)o) / 8;
    t.dst1[l] = (encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + round8(4 * g.n_new)) / 8 + qs;
    t.dst2[l] = (g.oref + 32 + 8 * ((nn + 1) / 2)) / 8 + g.W + qs;
  }
  const uint64_t winc = wave_incl_scan(words);
  if (k < Nn) t.q[l] = winc - words;
  if (l == WAVE - 1) t.q[n] = winc;
  wave_sync();
  copy_tab(t, n, reinterpret_cast<const uint64_t*>(cur), reinterpret_cast<uint64_t*>(enc),
           reinterpret_cast<uint64_t*>(newref));
  wave_sync();
}

constexpr int FX_PW = 8;  // presence words per wave in k_enc_fixed

// The encodings' offsets and headers (per segment), then their fixed
// sections: presence bitmaps (one wave per 64 reference slots), word bitmaps
// and block size tables (per group), then the new records (enc_new_wave, 64
// to a wave).  A segment's encoding starts at its fixed bytes' prefix plus
// the block bytes before its first group.  The offsets are written even
// when the encodings do not fit (they give the size needed); nothing else is
// written then.
struct NewArgs {
  const uint64_t* cscan;
  const uint32_t* nlist;
  const uint32_t* cwords;
  const uint8_t* cur;
  uint8_t* newref;
  const uint64_t* juid;
  const uint64_t* jhdr;
  const uint64_t* ckeys;
  uint64_t* okeys;
  uint64_t okeys_cap;
};
// (five waves per SIMD: 96 registers, no spill)
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_enc_fixed(Common cm, const int32_t* m, const uint64_t* bm,
                                                     const uint8_t* gsz, const uint8_t* gch, const uint64_t* gex,
                                                     uint8_t* enc, int64_t enc_cap, int64_t* enc_off,
                                                     uint8_t* modes, NewArgs na) {
  __shared__ NewTab s_t[WAVES];
  if (status_of(cm.status) & ANY_ERR) return;
  const uint64_t total_bytes = (uint64_t)cm.meta[9] + gex[cm.meta[3]];
  const bool fits = total_bytes <= (uint64_t)enc_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    enc_off[cm.nseg] = (int64_t)total_bytes;
    if (!fits) fail(cm.status, ERR_CAPACITY);
  }
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * BLOCK) {
    Seg& g = cm.seg[s];
    const uint64_t off = g.fixed_excl + gex[cm.gpre[s]];
    g.encm = off;
    enc_off[s] = (int64_t)off;
    if (modes) modes[s] = (uint8_t)g.mode;
    if (!fits) continue;
    uint64_t* h = reinterpret_cast<uint64_t*>(enc + off);
    h[0] = (uint64_t)TAD1_MAGIC | (1ull << 32) | ((uint64_t)g.mode << 48) | (1ull << 56);
    h[1] = g.nr | (g.n_match << 32);
    h[2] = g.n_new | ((uint64_t)cm.op << 32);
    h[3] = g.rwr;
    h[4] = g.fold;
    h[5] = g.W;
    h[6] = g.new_words;
    h[7] = gex[cm.gpre[s + 1]] - gex[cm.gpre[s]];
  }
  if (!fits) return;
  auto encm = [&](int64_t s) { return cm.seg[s].fixed_excl + gex[cm.gpre[s]]; };
  // wave tasks: presence words first, FX_PW to a wave (the slot loads of all
  // FX_PW words in flight at once), then groups, 64 to a wave, then new
  // records, 64 to a wave
  const int64_t P = cm.meta[4], B = cm.meta[3];
  const int64_t Nn = (int64_t)(na.cscan[cm.meta[0]] >> PK);
  const int64_t TP = (P + FX_PW - 1) / FX_PW, TG = (B + 63) / 64, TN = (Nn + WAVE - 1) / WAVE;
  const int l = lane_id();
  for (int64_t task = (int64_t)blockIdx.x * WAVES + wave_id(); task < TP + TG + TN;
       task += (int64_t)gridDim.x * WAVES) {
    const int64_t wbase = 64 * (task - TP);  // groups: the wave's first group
    const int64_t it = wbase + l;
    if (task >= TP + TG) {
      enc_new_wave(cm, WAVE * (task - TP - TG), Nn, na.cscan, na.nlist, na.cwords, na.cur, enc, na.newref, gex,
                   na.juid, na.jhdr, na.ckeys, na.okeys, na.okeys_cap, s_t[wave_id()]);
    } else if (task < TP) {
      const int64_t pw0 = task * FX_PW, pl = pw0 + FX_PW - 1 < P ? pw0 + FX_PW - 1 : P - 1;
      const int64_t lo = seg_of(cm.ppre, cm.nseg, (uint64_t)pw0);
      const int64_t hi = last_le<uint64_t>(cm.ppre, lo, cm.nseg, (uint64_t)pl);
      int64_t sj[FX_PW];
      uint64_t idx[FX_PW], dst[FX_PW];
      bool ok[FX_PW];
#pragma unroll
      for (int j = 0; j < FX_PW; ++j) {
        const int64_t pw = pw0 + j < pl ? pw0 + j : pl;
        sj[j] = last_le<uint64_t>(cm.ppre, lo, hi + 1, (uint64_t)pw);
        const uint64_t jj = 64 * (pw - cm.ppre[sj[j]]) + (uint64_t)l;
        ok[j] = pw0 + j <= pl && jj < cm.seg[sj[j]].nr;
        idx[j] = ok[j] ? cm.rpre[sj[j]] + jj : 0;
        dst[j] = encm(sj[j]) + 64 + 8 * (pw - cm.ppre[sj[j]]);
      }
      int32_t mv[FX_PW];
#pragma unroll
      for (int j = 0; j < FX_PW; ++j) mv[j] = m[idx[j]];
      __builtin_amdgcn_sched_barrier(0);
      uint64_t word = 0, at = 0;
#pragma unroll
      for (int j = 0; j < FX_PW; ++j) {
        const uint64_t w = __ballot(ok[j] && mv[j] >= 0);
        if (l == j) {
          word = w;
          at = dst[j];
        }
      }
      if (l < FX_PW && pw0 + l <= pl) *reinterpret_cast<uint64_t*>(enc + at) = word;
    } else {  // groups
      const int64_t g0 = wbase;
      const int64_t gl = g0 + 63 < B ? g0 + 63 : B - 1;
      const int64_t gg = it;
      const int64_t s = wave_seg(cm.gpre, cm.nseg, (uint64_t)(gg < B ? gg : B - 1), (uint64_t)g0, (uint64_t)gl);
      if (gg >= B) continue;
      const Seg& g = cm.seg[s];
      const uint64_t lg = gg - cm.gpre[s];
      uint8_t* sec = enc + encm(s) + 64 + 8 * g.PG;
      *reinterpret_cast<uint64_t*>(sec + 8 * lg) = bm[gg];
      sec += 8 * g.G;
      // mixed segments: bit 7 marks a group whose block is the learned one
      sec[lg] = (uint8_t)(gsz[gg] | (gch && g.mode == 2 && (gch[gg] & GCH_VARIANT) == 1 ? 0x80u : 0u));
      if (lg == g.G - 1)
        for (uint64_t b = g.G; b < round8(g.G); ++b) sec[b] = 0;
    }
  }
}

// =============================================================================
// Decoder
// =============================================================================
// One thread per segment: header checks and section sizes (scanned
// afterwards by k_scan_cols).
__device__ void dec_setup(Common cm, const uint8_t* enc, int64_t enc_len,
                          const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                          const int64_t* ref_off, bool have_pred, ClearFirst cf) {
  do_clear_first(cf);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * blockDim.x) {
    uint64_t nr = 0, G = 0, nn = 0, osz = 0, PG = 0, hs = 0;
    for (int k = 0; k < FOLD_SLOTS; ++k) cm.fold[s * FOLD_SLOTS + k] = 0;
    {
      Seg& g = cm.seg[s];
      const int64_t ea = enc_off[s], eb = enc_off[s + 1], ra = ref_off[s], rb = ref_off[s + 1];
      uint32_t code = 0;
      uint32_t n;
      uint64_t rw;
      if (!(ea >= 0 && eb >= ea && eb <= enc_len && !(ea & 7) && ra >= 0 && rb >= ra && rb <= ref_len && !(ra & 7)))
        code = ERR_INVALID;
      else if (eb - ea < 64)
        code = ERR_CORRUPT;
      const uint8_t* e = enc + ea;
      uint64_t h[8] = {0};
      if (!code) {
        for (int k = 0; k < 8; ++k) h[k] = ld64(e + 8 * k);
        const uint32_t magic = (uint32_t)h[0], ver = (uint32_t)(h[0] >> 32) & 0xFFFF;
        const uint32_t mode = (uint32_t)(h[0] >> 48) & 0xFF, packer = (uint32_t)(h[0] >> 56);
        if (magic != TAD1_MAGIC || ver != 1 || packer != 1 || mode > 2 || (h[2] >> 32) > 1) code = ERR_CORRUPT;
        // both ends of a pair agree on the predictor and on the operator
        else if ((mode >= 1 && !have_pred) || (h[2] >> 32) != cm.op) code = ERR_INVALID;
        g.mode = mode;
      }
      if (!code && !tam1_header(ref + ra, rb - ra, &n, &rw)) code = ERR_INVALID;
      if (!code) {
        g.rmsg = ra;
        g.nr = n;
        g.rwr = rw;
        g.rbody = ra + 32 + 8 * ((n + 1) / 2);
        const uint64_t n_ref = h[1] & 0xFFFFFFFFu, n_match = h[1] >> 32, n_new = h[2] & 0xFFFFFFFFu;
        const uint64_t ref_words = h[3], W = h[5], new_words = h[6], var = h[7];
        const uint64_t len = (uint64_t)(eb - ea);
        g.fold = h[4];
        g.rfold = 0;
        g.var = var;
        if (n_ref != n || ref_words != rw) {
          code = ERR_REF;
        } else if (n_match > n_ref || W > ref_words || n_new > len / 4 || new_words > len / 8 || var > len ||
                   new_words < 2 * n_new) {
          code = ERR_CORRUPT;
        } else {
          const uint64_t Gs = (W + 63) / 64, PGs = (n_ref + 63) / 64;
          const uint64_t fixed = 64 + 8 * PGs + 8 * Gs + round8(Gs) + round8(4 * n_new) + 8 * new_words;
          if (fixed + var != len) {
            code = ERR_CORRUPT;
          } else {
            // zero tails: presence bits past n_ref, bitmap bits past W, table pads
            const uint8_t* pres = e + 64;
            const uint8_t* bits = pres + 8 * PGs;
            const uint8_t* gs = bits + 8 * Gs;
            const uint8_t* ns = gs + round8(Gs);
            if ((n_ref & 63) && (ld64(pres + 8 * (PGs - 1)) >> (n_ref & 63))) code = ERR_CORRUPT;
            if ((W & 63) && (ld64(bits + 8 * (Gs - 1)) >> (W & 63))) code = ERR_CORRUPT;
            for (uint64_t b = Gs; b < round8(Gs); ++b)
              if (gs[b]) code = ERR_CORRUPT;
            if ((n_new & 1) && ld32(ns + 4 * n_new)) code = ERR_CORRUPT;
            g.encm = ea;
            g.n_match = n_match;
            g.W = W;
            g.n_new = n_new;
            g.new_words = new_words;
            g.G = Gs;
            g.PG = PGs;
            g.fixed = fixed;
            nr = n;
            G = Gs;
            nn = n_new;
            PG = PGs;
            osz = tam1_size(n_match + n_new, W + new_words);
            hs = pow2ceil(2 * nr);
            g.hsize = hs;
          }
        }
      }
      if (code) {
        fail(cm.status, code);
        nr = G = nn = osz = PG = hs = 0;
      }
    }
    col(cm, 0)[s] = nr;
    col(cm, 1)[s] = G;
    col(cm, 2)[s] = nn;
    col(cm, 3)[s] = osz;
    col(cm, 4)[s] = PG;
    col(cm, 5)[s] = hs;
  }
}

__global__ __launch_bounds__(BLOCK) void k_dec_setup(Common cm, const uint8_t* enc, int64_t enc_len,
                                                     const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                                                     const int64_t* ref_off, bool have_pred, ClearFirst cf) {
  dec_setup(cm, enc, enc_len, enc_off, ref, ref_len, ref_off, have_pred, cf);
}

// Few segments: a call's per-segment passes and their column scans in one
// block of 1024 threads (one launch instead of two or three).
__global__ __launch_bounds__(1024) void k_enc_setup1(Common cm, const uint8_t* cur, int64_t cur_len,
                                                     const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                                                     const int64_t* ref_off, ClearFirst cf, ColScan cs, int ncols) {
  __shared__ uint64_t s_w[16];
  enc_setup(cm, cur, cur_len, cur_off, ref, ref_len, ref_off, cf);
  __syncthreads();
  scan_columns_small(cs, ncols, s_w);
}
__global__ __launch_bounds__(1024) void k_enc_layout1(Common cm, const uint64_t* rscan, const uint64_t* cscan,
                                                      uint64_t* mstart, ColScan cs, int ncols, uint8_t* newref,
                                                      int64_t newref_cap, int64_t* newref_off, uint64_t* gex) {
  __shared__ uint64_t s_w[16];
  enc_seg2(cm, rscan, cscan, mstart);
  __syncthreads();
  scan_columns_small(cs, ncols, s_w);
  enc_seg3(cm, newref, newref_cap, newref_off, gex);
}
__global__ __launch_bounds__(1024) void k_dec_setup1(Common cm, const uint8_t* enc, int64_t enc_len,
                                                     const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                                                     const int64_t* ref_off, bool have_pred, ClearFirst cf,
                                                     ColScan cs, int ncols) {
  __shared__ uint64_t s_w[16];
  dec_setup(cm, enc, enc_len, enc_off, ref, ref_len, ref_off, have_pred, cf);
  __syncthreads();
  scan_columns_small(cs, ncols, s_w);
}

// Every reference slot: its size in words, whether the encoding keeps it
// (presence bit), and the XOR of the reference uids (compared with the
// encoding's later).  A wave takes RL_U * 64 consecutive slots per pass, RL_U
// per lane, and issues all their loads before it stores anything.
// (segs, rpre: read-only here; as restrict parameters, reads with a
// wave-uniform segment become scalar loads)
__global__ __launch_bounds__(BLOCK) void k_dec_rslots(Common cm, const uint8_t* enc, const uint8_t* ref,
                                                      uint32_t* rwords, uint8_t* rmatch,
                                                      const Seg* __restrict__ segs,
                                                      const uint64_t* __restrict__ rpre, const uint64_t* rkeys) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  const int l = lane_id();
  constexpr int64_t SPAN = (int64_t)WAVE * RL_U;
  const int64_t nwv = (int64_t)gridDim.x * WAVES;
  bool bad = false;
  for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave_id()) * SPAN; base < Rt; base += nwv * SPAN) {
    const int64_t last = base + SPAN - 1 < Rt ? base + SPAN - 1 : Rt - 1;
    const int64_t lo = wave_last_le<uint64_t>(rpre, 0, cm.nseg, (uint64_t)base);
    const int64_t hi = wave_last_le<uint64_t>(rpre, lo, cm.nseg, (uint64_t)last);
    uint64_t uid[RL_U], hdr[RL_U], pw[RL_U], jv[RL_U];
    int64_t sv[RL_U];
    bool ok[RL_U];
    Tam1Loc loc[RL_U];
    // slots past the end read the last one (unused); all offsets and
    // presence words are loaded before any record word
    const bool one = lo == hi;  // uniform: the whole pass in one segment
    if (one) {
      const int64_t su = (int64_t)uniform32((uint32_t)lo);
      const Seg& sg = segs[su];
      const uint64_t r0 = rpre[su];
      const uint8_t* m = ref + sg.rmsg;
#pragma unroll
      for (int u = 0; u < RL_U; ++u) {
        const int64_t g = base + (int64_t)u * WAVE + l;
        const uint64_t j = (uint64_t)(g <= last ? g : last) - r0;
        loc[u] = tam1_locate(m, (uint32_t)sg.nr, sg.rwr, (uint32_t)j);
        pw[u] = ld64(enc + sg.encm + 64 + 8 * (j / 64));
        jv[u] = j;
        sv[u] = su;
      }
      if (rkeys) {
#pragma unroll
        for (int u = 0; u < RL_U; ++u) {
          const ulonglong2 kv = *reinterpret_cast<const ulonglong2*>(rkeys + 2 * (r0 + jv[u]));
          uid[u] = kv.x;
          hdr[u] = kv.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < RL_U; ++u) tam1_words(m, (uint32_t)sg.nr, loc[u], &uid[u], &hdr[u]);
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the checks below every record load
#pragma unroll
      for (int u = 0; u < RL_U; ++u) ok[u] = tam1_valid(loc[u], hdr[u]) && uid[u] != 0;
    } else {
#pragma unroll
      for (int u = 0; u < RL_U; ++u) {
        const int64_t g = base + (int64_t)u * WAVE + l;
        const int64_t s = last_le<uint64_t>(rpre, lo, hi + 1, (uint64_t)(g <= last ? g : last));
        const Seg& sg = segs[s];
        const uint64_t j = (uint64_t)(g <= last ? g : last) - rpre[s];
        loc[u] = tam1_locate(ref + sg.rmsg, (uint32_t)sg.nr, sg.rwr, (uint32_t)j);
        pw[u] = ld64(enc + sg.encm + 64 + 8 * (j / 64));
        jv[u] = j;
        sv[u] = s;
      }
#pragma unroll
      for (int u = 0; u < RL_U; ++u) {
        const Seg& sg = segs[sv[u]];
        if (rkeys) {
          const ulonglong2 kv = *reinterpret_cast<const ulonglong2*>(rkeys + 2 * (rpre[sv[u]] + jv[u]));
          uid[u] = kv.x;
          hdr[u] = kv.y;
        } else {
          tam1_words(ref + sg.rmsg, (uint32_t)sg.nr, loc[u], &uid[u], &hdr[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < RL_U; ++u) ok[u] = tam1_valid(loc[u], hdr[u]) && uid[u] != 0;
    }
    uint64_t f = 0;
#pragma unroll
    for (int u = 0; u < RL_U; ++u) {
      const int64_t g = base + (int64_t)u * WAVE + l;
      const bool active = g <= last;
      if (active) {
        if (!ok[u]) bad = true;
        rmatch[g] = (uint8_t)((pw[u] >> (jv[u] & 63)) & 1);
        rwords[g] = (uint32_t)(hdr[u] >> 32);
      }
      if (one) {
        if (active && ok[u]) f ^= uid[u];
      } else {
        seg_xor(cm.fold, FOLD_SLOTS, sv[u], active && ok[u], uid[u]);
      }
    }
    if (one) seg_xor(cm.fold, FOLD_SLOTS, lo, true, f);
  }
  if (bad) fail(cm.status, ERR_INVALID);
}

struct DMatchIn {
  static constexpr int ROUNDS = 16;  // a tile of 8192 slots
  const uint8_t* rmatch;
  const uint32_t* rwords;
  __device__ uint64_t operator()(int64_t g) const {
    const uint64_t w = rwords[g];
    return rmatch[g] ? ((1ull << PK) | w) : 0;
  }
};
// Words of new records, from the encodings' size tables, and group block
// bytes, from their group size tables: segment and its table's offset for
// the scan's rounds, then the table entries.
struct DNewIn {
  static constexpr int ROUNDS = 4;  // short scans: more tiles in flight
  Common cm;
  const uint8_t* enc;
  int64_t lo = 0, hi = 0;  // segments of the wave's items
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(cm.npre, 0, cm.nseg, (uint64_t)first);
    hi = wave_last_le<uint64_t>(cm.npre, lo, cm.nseg, (uint64_t)last);
  }
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    uint64_t at[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      const uint64_t x = (uint64_t)(i < n ? i : n - 1);
      const int64_t s = lo == hi ? lo : last_le<uint64_t>(cm.npre, lo, hi + 1, x);
      const Seg& g = cm.seg[s];
      at[r] = g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + 4 * (x - cm.npre[s]);
    }
    __builtin_amdgcn_sched_barrier(0);
    uint32_t sz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sz[r] = ld32(enc + at[r]);
    __builtin_amdgcn_sched_barrier(0);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bad = bad || sz[r] < 2;
      v[r] = wbase + r * WAVE + l >= n ? 0 : (sz[r] < 2 ? 2 : sz[r]);
    }
    if (bad) fail(cm.status, ERR_CORRUPT);
  }
};
struct DGroupIn {
  static constexpr int ROUNDS = 4;  // short scans: more tiles in flight
  Common cm;
  const uint8_t* enc;
  int64_t lo = 0, hi = 0;  // segments of the wave's items
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(cm.gpre, 0, cm.nseg, (uint64_t)first);
    hi = wave_last_le<uint64_t>(cm.gpre, lo, cm.nseg, (uint64_t)last);
  }
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    uint64_t at[R];
    uint8_t mk[R];  // mixed segments: bit 7 of a size byte is the group's flag
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      const uint64_t x = (uint64_t)(i < n ? i : n - 1);
      const int64_t s = lo == hi ? lo : last_le<uint64_t>(cm.gpre, lo, hi + 1, x);
      const Seg& g = cm.seg[s];
      at[r] = g.encm + 64 + 8 * g.PG + 8 * g.G + (x - cm.gpre[s]);
      mk[r] = g.mode == 2 ? 0x7F : 0xFF;
    }
    __builtin_amdgcn_sched_barrier(0);
    uint8_t b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = enc[at[r]];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = wbase + r * WAVE + l >= n ? 0 : 8 * (uint64_t)(b[r] & mk[r]);
  }
};

// Per segment: matched and new record bases, checks against the header,
// C' offsets and headers (one thread per segment).
__global__ __launch_bounds__(BLOCK) void k_dec_seg2(Common cm, const uint64_t* rscan, const uint64_t* nscan,
                                                    const uint64_t* gex, uint8_t* out, int64_t out_cap,
                                                    int64_t* out_off, uint64_t* mstart) {
  if (status_of(cm.status) & ANY_ERR) return;
  const bool fits = cm.opre[cm.nseg] <= (uint64_t)out_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cm.meta[5] = (int64_t)(rscan[cm.meta[1]] >> PK);
    mstart[cm.meta[5]] = rscan[cm.meta[1]] & WMASK;  // end of the last matched record
    cm.meta[7] = (int64_t)nscan[cm.meta[6]];
    out_off[cm.nseg] = (int64_t)cm.opre[cm.nseg];
    if (!fits) fail(cm.status, ERR_CAPACITY);
  }
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < cm.nseg; s += (int64_t)gridDim.x * BLOCK) {
    Seg& g = cm.seg[s];
    const uint64_t rs = rscan[cm.rpre[s]], re = rscan[cm.rpre[s + 1]];
    const uint64_t oref = cm.opre[s];
    g.oref = oref;
    out_off[s] = (int64_t)oref;
    g.mbase = rs >> PK;
    g.dbase = rs & WMASK;
    g.cpw = (oref + 32 + 8 * ((g.n_match + g.n_new + 1) / 2)) / 8 - g.dbase;
    const uint64_t nm = (re >> PK) - g.mbase, W = (re & WMASK) - g.dbase;
    g.npbase = nscan[cm.npre[s]];
    const uint64_t nw = nscan[cm.npre[s + 1]] - g.npbase;
    const uint64_t var = gex[cm.gpre[s + 1]] - gex[cm.gpre[s]];
    g.rfold = fold_of(cm.fold + s * FOLD_SLOTS);
    if (g.rfold != g.fold) fail(cm.status, ERR_REF);
    if (nm != g.n_match || W != g.W || nw != g.new_words || var != g.var) fail(cm.status, ERR_CORRUPT);
    // the header of this segment's C' (inside the output: oref + its size <= total <= out_cap)
    if (!fits) continue;
    uint8_t* o = out + oref;
    const uint64_t n = g.n_match + g.n_new;
    uint64_t* h = reinterpret_cast<uint64_t*>(o);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);
    h[1] = n;
    h[2] = g.W + g.new_words;
    h[3] = 0;
    if (n & 1) *reinterpret_cast<uint32_t*>(o + 32 + 4 * n) = 0;
  }
}

// New records from the encoding into C', and their offsets, for the 64 new
// records from the wave's first rb: tabulated in LDS, their words copied
// lane-parallel.  A new record's uid must be non-zero and its header must
// give the size the table announced.
__device__ inline void dec_new_wave(const Common& cm, int64_t rb, int64_t Nn, const uint64_t* nscan,
                                    const uint8_t* enc, uint8_t* out, uint64_t* okeys, uint64_t okeys_cap,
                                    NewTab& t) {
  const int l = lane_id();
  const uint64_t* e64 = reinterpret_cast<const uint64_t*>(enc);
  uint64_t* o64 = reinterpret_cast<uint64_t*>(out);
  const int64_t r = rb + l;
  const int64_t re = rb + WAVE - 1 < Nn ? rb + WAVE - 1 : Nn - 1;
  const int n = (int)(re - rb + 1);
  const int64_t s = wave_seg(cm.npre, cm.nseg, (uint64_t)(r < Nn ? r : Nn - 1), (uint64_t)rb, (uint64_t)re);
  if (r < Nn) {
    const Seg& g = cm.seg[s];
    const uint64_t qs = nscan[r] - g.npbase;
    const uint64_t nn = g.n_match + g.n_new;
    t.q[l] = nscan[r] - nscan[rb];
    t.src[l] = (g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + round8(4 * g.n_new)) / 8 + qs;
    t.dst1[l] = (g.oref + 32 + 8 * ((nn + 1) / 2)) / 8 + g.W + qs;
    t.dst2[l] = nscan[r + 1] - nscan[r];  // size
    t.kidx[l] = g.mbase + g.n_match + (uint64_t)r;  // the record's index among all C' records
    *reinterpret_cast<uint32_t*>(out + g.oref + 32 + 4 * (g.n_match + (uint64_t)r - cm.npre[s])) =
        (uint32_t)(g.W + qs);
  }
  if (l == 0) t.q[n] = nscan[rb + n] - nscan[rb];
  wave_sync();
  const uint64_t tot = t.q[n];
  bool bad = false, cap = false;
  for (uint64_t q0 = l; q0 < tot; q0 += NC_U * WAVE) {  // NC_U words per lane in flight
    uint64_t v[NC_U], d[NC_U], w[NC_U], sz[NC_U], ki[NC_U];
#pragma unroll
    for (int j = 0; j < NC_U; ++j) {
      const uint64_t q = q0 + (uint64_t)j * WAVE < tot ? q0 + (uint64_t)j * WAVE : tot - 1;
      const int i = lds_last_le(t.q, n, q);
      w[j] = q - t.q[i];
      v[j] = e64[t.src[i] + w[j]];
      d[j] = t.dst1[i] + w[j];
      sz[j] = t.dst2[i];
      ki[j] = t.kidx[i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NC_U; ++j)
      if (q0 + (uint64_t)j * WAVE < tot) {
        if ((w[j] == 0 && v[j] == 0) || (w[j] == 1 && (v[j] >> 32) != sz[j])) bad = true;
        o64[d[j]] = v[j];
        if (okeys && w[j] < 2) {  // the record's uid and header word
          if (ki[j] < okeys_cap) okeys[2 * ki[j] + w[j]] = v[j];
          else cap = true;
        }
      }
  }
  if (__ballot(bad) && l == 0) fail(cm.status, ERR_CORRUPT);
  if (__ballot(cap) && l == 0) fail(cm.status, ERR_CAPACITY);
  wave_sync();
}

// Directory of the matched records (decoder): R word, residual start,
// slot; word offsets of the records in the reference's record area; C'
// offsets; the descriptors of the residual groups.  Staged like the
// encoder's.  Then the new records into C' (dec_new_wave): only the
// unpacking follows, and it writes other words of C'.  hist_cap >= 0
// (learned calls): the history's capacity, checked here, before any new
// record is copied, as the neighbour table's pass checks it.
__global__ __launch_bounds__(BLOCK) void k_dec_mdir(Common cm, const uint8_t* ref, const uint8_t* rmatch,
                                                    const uint64_t* rscan, const uint32_t* rwords, MDir* mdir,
                                                    uint64_t* mstart, uint8_t* out, const uint8_t* enc,
                                                    const uint64_t* gex, GDesc* gdesc, uint32_t* mrw,
                                                    const uint64_t* rkeys, uint64_t* okeys, uint64_t okeys_cap,
                                                    const uint64_t* nscan, int64_t hist_cap, Entry* ntab) {
  __shared__ NewTab s_t[WAVES];
  if (status_of(cm.status) & ANY_ERR) return;
  if (hist_cap >= 0 && hist_cap < cm.meta[1]) {  // the prediction's history must cover every reference slot
    if (blockIdx.x == 0 && threadIdx.x == 0) fail(cm.status, ERR_INVALID);
    return;
  }
  const int64_t Rt = cm.meta[1];
  const int l = lane_id();
  constexpr int64_t SPAN = (int64_t)WAVE * RS_U;
  const int64_t nwv = (int64_t)gridDim.x * WAVES;
  for (int64_t base = ((int64_t)blockIdx.x * WAVES + wave_id()) * SPAN; base < Rt; base += nwv * SPAN) {
    const int64_t last = base + SPAN - 1 < Rt ? base + SPAN - 1 : Rt - 1;
    const int64_t lo = wave_last_le<uint64_t>(cm.rpre, 0, cm.nseg, (uint64_t)base);
    const int64_t hi = wave_last_le<uint64_t>(cm.rpre, lo, cm.nseg, (uint64_t)last);
    int64_t sv[RS_U];
    uint8_t mv[RS_U];
    uint64_t rsv[RS_U];
    uint32_t rwv[RS_U], roff[RS_U];
#pragma unroll
    for (int u = 0; u < RS_U; ++u) {
      const int64_t g = base + (int64_t)u * WAVE + l;
      const int64_t gc = g <= last ? g : last;
      const int64_t sx = lo == hi ? lo : last_le<uint64_t>(cm.rpre, lo, hi + 1, (uint64_t)gc);
      sv[u] = sx;
      mv[u] = rmatch[gc];
      rsv[u] = rscan[gc];
      rwv[u] = rwords[gc];
      roff[u] = ld32(ref + cm.seg[sx].rmsg + 32 + 4 * ((uint64_t)gc - cm.rpre[sx]));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < RS_U; ++u) {
      const int64_t g = base + (int64_t)u * WAVE + l;
      if (g > last || !mv[u]) continue;
      const int64_t sx = sv[u];
      const Seg& sg = cm.seg[sx];
      const uint64_t k = rsv[u] >> PK;
      const uint64_t d = rsv[u] & WMASK;
      if (mdir) {  // learned mode or a history to write: the full entry
        mdir[k] = MDir{sg.rbody / 8 + roff[u], (uint64_t)g | ((uint64_t)sx << 34)};
      }
      mstart[k] = d;
      mrw[k] = roff[u];  // word offset in the reference's record area
      if (okeys) {  // C' record k + (new records of earlier segments): the slot's uid and header
        const uint64_t* src = rkeys ? rkeys + 2 * g
                                    : reinterpret_cast<const uint64_t*>(ref + sg.rbody + 8 * (uint64_t)roff[u]);
        const uint64_t o = k + cm.npre[sx];
        if (o < okeys_cap) *reinterpret_cast<ulonglong2*>(okeys + 2 * o) = ulonglong2{src[0], src[1]};
        else fail(cm.status, ERR_CAPACITY);
      }
      *reinterpret_cast<uint32_t*>(out + sg.oref + 32 + 4 * (k - sg.mbase)) = (uint32_t)(d - sg.dbase);
      map_groups_dec(cm, sg, sx, d - sg.dbase, rwv[u], k, enc, gex, gdesc);
    }
  }
  // then the new records, 64 to a wave
  const int64_t Nn = cm.meta[6];
  for (int64_t rb = ((int64_t)blockIdx.x * WAVES + wave_id()) * WAVE; rb < Nn; rb += nwv * WAVE)
    dec_new_wave(cm, rb, Nn, nscan, enc, out, okeys, okeys_cap, s_t[wave_id()]);
  if (ntab) nbr_clear(cm, ntab, hist_cap);
}

struct UnpackArgs {
  Common cm;
  const uint8_t* enc;
  const uint64_t* ref;     // (words)
  const uint32_t* mrw;     // [matched] word offset of every matched record in its reference's record area
  const uint64_t* mstart;  // [matched+1]
  const uint64_t* pred_x;
  const uint8_t* pred_on;
  uint64_t* out;           // C' (words)
};

// Byte-granular funnel: the 32 bits of hi:lo starting at bit s (s < 32).
__device__ inline uint32_t funnel32(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

// One wave per 64-word group: read the block, rebuild the residual words D
// and write C' = D xor X, X the reference record (or its prediction on words
// 2..5).  A wave takes UNPACK_PG consecutive groups at a time and issues all
// their loads (descriptors, record tables, block words, reference words)
// before it consumes any.
//
// Each word's record: the records overlapping a group (at most 33, since
// records have at least two words) are held one per lane, lane 0 holding
// the one with the group's first word.  Lanes 1..32 mark their record's
// start word in LDS with a tag unique to the group, one ballot turns the
// marks into a start mask, and a word's record index is the number of
// starts at or below it.
//
// Every length, size, padding byte and unused nibble is checked, and the
// uid and header words of a matched record must have a zero residual.
// (gdesc: read-only here; as a restrict parameter its uniform reads become
// scalar loads)
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_dec_unpack(UnpackArgs a, const GDesc* __restrict__ gdesc,
                                                      const uint8_t* __restrict__ enc) {
  constexpr int BW = BLK_MAX / 8 + 1;  // block words, one spare for the two-word read
  __shared__ uint64_t s_blk[WAVES][UNPACK_PG][BW];
  __shared__ uint32_t s_mark[WAVES][UNPACK_PG][WAVE];  // record-start marks: group index + 1
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Gt = cm.meta[3], M = cm.meta[5];
  const int l = lane_id(), wv = wave_id();
#pragma unroll
  for (int x = 0; x < UNPACK_PG; ++x) s_mark[wv][x][l] = 0;  // no group's tag
  wave_sync();
  const uint64_t le_mask = lanemask_le(l);
  bool anybad = false;
  const int64_t nw = (int64_t)gridDim.x * WAVES;
  for (int64_t g0 = ((int64_t)blockIdx.x * WAVES + wv) * UNPACK_PG; g0 < Gt; g0 += nw * UNPACK_PG) {
    // the groups' descriptors (scalar registers) ...
    GDesc dv[UNPACK_PG];
    // ... and per lane: record start (relative to the group's first word)
    // and reference word offset of record k0 + lane, block words lane and 64 + lane
    int relv[UNPACK_PG];
    uint32_t rwv[UNPACK_PG];
    uint64_t b0v[UNPACK_PG], b1v[UNPACK_PG];
#pragma unroll
    for (int x = 0; x < UNPACK_PG; ++x) {
      const int64_t gg = g0 + x < Gt ? g0 + x : Gt - 1;
      dv[x] = gdesc[gg];
      const GDesc& d = dv[x];
      // (loads from clamped indices, not behind divergent branches: a group
      // implies a matched record, so M >= 1)
      const uint64_t k0 = d.k0;
      const bool has = l <= 32 && k0 + l < (uint64_t)M;
      const uint64_t kk = has ? k0 + l : (uint64_t)M - 1;
      const int64_t r = (int64_t)a.mstart[kk] - (int64_t)d.g0w;
      const uint32_t rwk = a.mrw[kk];
      // clamped to [-2^30, 64]: lane 0's record may start long before the group
      relv[x] = !has ? 64 : (r > 64 ? 64 : (r < -(1 << 30) ? -(1 << 30) : (int)r));
      rwv[x] = has ? rwk : 0u;
      b0v[x] = b1v[x] = 0;
      const uint32_t size = d.size;
      if (size > 0 && size <= BLK_MAX) {  // uniform; lanes past the block read its last word
        const uint64_t* src = reinterpret_cast<const uint64_t*>(enc + d.blk);
        const uint32_t nwd = size / 8;
        b0v[x] = src[(uint32_t)l < nwd ? (uint32_t)l : nwd - 1];
        if (size > 8 * WAVE) b1v[x] = src[(uint32_t)(WAVE + l) < nwd ? (uint32_t)(WAVE + l) : nwd - 1];
      }
    }
    // record starts inside each group
#pragma unroll
    for (int x = 0; x < UNPACK_PG; ++x)
      if (g0 + x < Gt && l >= 1 && l <= 32 && relv[x] >= 1 && relv[x] < WAVE)
        s_mark[wv][x][relv[x]] = (uint32_t)(g0 + x) + 1;
    wave_sync();
    // each word's record, and its reference word (loads issued for all groups)
    uint64_t xwv[UNPACK_PG];
    uint32_t offv[UNPACK_PG];
#pragma unroll
    for (int x = 0; x < UNPACK_PG; ++x) {
      const int64_t gg = g0 + x;
      xwv[x] = 0;
      offv[x] = 0;
      if (gg >= Gt) break;
      const GDesc& d = dv[x];
      const uint64_t starts = __ballot(s_mark[wv][x][l] == (uint32_t)gg + 1);
      const int idx = __popcll(starts & le_mask);  // <= 32
      const uint32_t off = (uint32_t)(l - __shfl(relv[x], idx, WAVE));
      const uint32_t rw = (uint32_t)__shfl((int)rwv[x], idx, WAVE);
      offv[x] = off;
      const bool live = (uint32_t)l < d.nlive;
      const uint64_t* rbody = a.ref + d.rbw;  // the segment's reference records
      // (a word that is not live reads word 0 of lane 0's record, the one
      // holding the group's first word: in the segment, always valid)
      const uint32_t ri = live ? rw + off : (uint32_t)__builtin_amdgcn_readlane((int)rwv[x], 0);
      if (d.usep) {  // uniform
        const uint64_t k = (uint64_t)d.k0 + (live ? (uint64_t)idx : 0);
        const bool pred = live && off >= 2 && off < 6 && a.pred_on[k];
        const uint64_t px = a.pred_x[4 * k + (pred ? off - 2 : 0)];
        const uint64_t rx = rbody[ri];
        xwv[x] = pred ? px : rx;
      } else {
        xwv[x] = rbody[ri];
      }
    }
    // blocks into LDS, residual words, output
#pragma unroll
    for (int x = 0; x < UNPACK_PG; ++x) {
      const int64_t gg = g0 + x;
      if (gg >= Gt) break;
      const GDesc& d = dv[x];
      uint64_t* blk = s_blk[wv][x];
      blk[l] = b0v[x];
      if (l < BW - WAVE) blk[WAVE + l] = b1v[x];
      wave_sync();
      const uint64_t bitmap = d.bm;
      const uint32_t size = d.size;
      const uint32_t popc = (uint32_t)__popcll(bitmap);
      const uint32_t nib = (popc + 1) / 2;
      const bool bit = (bitmap >> l) & 1;
      const uint32_t t = __builtin_amdgcn_mbcnt_hi((uint32_t)(bitmap >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bitmap, 0u));
      const uint8_t* b8 = reinterpret_cast<const uint8_t*>(blk);
      const uint32_t len = bit ? (uint32_t)(b8[t >> 1] >> (4 * (t & 1))) & 15u : 0u;
      bool bad = bit && (len - 1u > 7u);  // a length outside 1..8
      const uint32_t incl = wave_incl_scan32(len);
      const uint32_t end = nib + (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      const bool gbad = size > BLK_MAX || end > size || ((end + 7) & ~7u) != size;
      // the len bytes at so: two aligned words, funnel-shifted by bytes.  In
      // a good group every set word has so + len <= end <= size <= BLK_MAX;
      // anything else (a bad group, a zero length) reads word 0 instead and
      // is reported, so both reads stay inside the buffer.
      const uint32_t so0 = nib + incl - len;
      const uint32_t so = (gbad || so0 >= (uint32_t)BLK_MAX) ? 0u : so0;
      const uint32_t wi = so >> 3, sh = 8 * (so & 3);
      const uint64_t w0 = blk[wi], w1 = blk[wi + 1];
      const bool hi4 = (so & 4) != 0;
      const uint32_t c0 = hi4 ? (uint32_t)(w0 >> 32) : (uint32_t)w0;
      const uint32_t c1 = hi4 ? (uint32_t)w1 : (uint32_t)(w0 >> 32);
      const uint32_t c2 = hi4 ? (uint32_t)(w1 >> 32) : (uint32_t)w1;
      uint32_t dlo = funnel32(c1, c0, sh), dhi = funnel32(c2, c1, sh);
      if (len < 4) dlo &= (1u << (8 * len)) - 1u;
      dhi = len <= 4 ? 0u : (len < 8 ? dhi & ((1u << (8 * (len - 4))) - 1u) : dhi);
      const uint64_t D = bit ? ((uint64_t)dhi << 32) | dlo : 0;
      if (bit && !bad && (D >> (8 * (len - 1))) == 0) bad = true;  // a leading zero byte
      bool gchk = gbad;
      if (!gbad) {
        // padding after `end` (inside the last block word) and an unused high nibble
        if ((end & 7) && (blk[size / 8 - 1] >> (8 * (end & 7))) != 0) gchk = true;
        if ((popc & 1) && (b8[popc >> 1] >> 4) != 0) gchk = true;
      }
      if ((uint32_t)l < d.nlive) {
        if (offv[x] < 2 && D != 0) bad = true;
        a.out[d.out + (uint64_t)l] = undiff_word<OP>(D, xwv[x]);
      }
      anybad = anybad || bad || gchk;
    }
    wave_sync();
  }
  if (__ballot(anybad) && l == 0) fail(cm.status, ERR_CORRUPT);
}



// ---------------------------------------------------------------------------
// Learned predictor inside the exchange (both sides evaluate it identically
// from the reference and the per-slot history).

// Cell of a reference record from its words 2..4 (x, y, z at x[0..2]):
// floor(v / cell) per axis, packed in 21 bits each; false when not finite or
// out of range.
__device__ inline bool cell_key_of(const uint64_t* x, double cell, uint64_t* key) {
  uint64_t k = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = floor(__longlong_as_double((long long)x[a]) / cell);
    if (!(f > -1048576.0 && f < 1048576.0)) return false;
    k = (k << 21) | (uint64_t)((int64_t)f + 1048576);
  }
  *key = k;
  return true;
}

// Neighbour counts: per segment, an open-addressing table of the cells of
// its reference records (key, count), cleared by the directory pass before.
__device__ inline uint64_t ref_record_word(const Common& cm, const uint8_t* ref, int64_t s, uint64_t j) {
  const Seg& g = cm.seg[s];
  return g.rbody / 8 + ld32(ref + g.rmsg + 32 + 4 * j);
}

__global__ __launch_bounds__(BLOCK) void k_nbr_build(Common cm, const uint8_t* ref, const PredW* pw, Entry* tab) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  const double cell = pw->cell;
  const uint64_t* ref64 = reinterpret_cast<const uint64_t*>(ref);
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK + wave_id() * WAVE; base < Rt; base += stride) {
    const int64_t g = base + lane_id();
    const uint64_t last = (uint64_t)(base + WAVE - 1 < Rt ? base + WAVE - 1 : Rt - 1);
    const int64_t s = wave_seg(cm.rpre, cm.nseg, (uint64_t)(g < Rt ? g : Rt - 1), (uint64_t)base, last);
    uint64_t key = 0;
    bool v = false;
    if (g < Rt) {
      const uint64_t* rec = ref64 + ref_record_word(cm, ref, s, g - cm.rpre[s]);
      v = (rec[1] >> 32) >= 5 && cell_key_of(rec + 2, cell, &key);
    }
    // Lanes with the same segment and cell add their count with one atomic:
    // neighbouring records mostly share a cell, so a wave has few distinct
    // ones.  Each round of the loop only finds the lanes of the first pending
    // lane's (segment, cell); then every such first lane inserts its cell and
    // adds its count, all at once.
    uint64_t pending = __ballot(v);
    uint32_t count = 0;
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint64_t lk = readlane64(key, leader);
      const int64_t ls = (int64_t)readlane64((uint64_t)s, leader);
      const uint64_t same = __ballot(v && key == lk && s == ls);
      if (lane_id() == leader) count = (uint32_t)__popcll(same);
      pending &= ~same;
    }
    if (count) {
      const Seg& sg = cm.seg[s];
      const uint64_t H = sg.hsize;
      Entry* t = tab + cm.hpre[s];
      uint64_t h = mix64(key) & (H - 1);
      for (uint64_t probe = 0; probe < H; ++probe) {
        const unsigned long long prev = atomicCAS(&t[h].key, 0ull, (unsigned long long)key);
        if (prev == 0ull || prev == (unsigned long long)key) {
          atomicAdd(&t[h].ci, count);
          break;
        }
        h = (h + 1) & (H - 1);
      }
    }
  }
}

struct PredictArgs {
  Common cm;
  const uint64_t* ref;
  uint64_t ref_words;  // words of the reference buffer
  const MDir* mdir;
  const PredW* pw;
  const Entry* tab;
  const uint64_t* h1;  // history of reference slots
  const uint64_t* h2;
  const uint8_t* hlen;
  uint64_t* pred_x;    // [matched][4] predicted words 2..5
  uint8_t* pred_on;    // [matched]
  // history of C' for the matched records (o1 null: none asked for)
  uint64_t* o1;
  uint64_t* o2;
  uint8_t* olen;
  int64_t ocap;
  // training-window tap (encoder only; tcount null: off)
  const uint64_t* cur;
  const uint64_t* crw; // [matched] C (low) and R word offsets in the segments' record areas
  int32_t* tin;        // [tcap][12]
  float* ttgt;         // [tcap][4]
  int64_t tcap;
  unsigned long long* tcount;
};

// Prediction of the matched records, 64 per wave at a time (one per lane).
// A lane's loads go out together: its directory entry, then its record's
// header and words 2..5, its slot's history and its segment's table place;
// its inputs go to LDS as int8 planes; the MLP runs on four groups of 16
// rows; the lane writes its record's predicted words and, with a history
// to write, the record's C' history (h2 <- h1, h1 <- the reference words).
template <bool HIST>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_predict(PredictArgs a) {
  __shared__ PredW s_w;
  __shared__ MlpIn s_in[WAVES];
  __shared__ int32_t s_q[WAVES][WAVE][4];
  __shared__ uint8_t s_h[WAVES][16][64];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  load_weights(&s_w, a.pw);
  const MlpOps ops = mlp_ops(s_w);
  const double cell = s_w.cell;
  const int64_t M = cm.meta[5];
  // (over capacity k_hist_out reports the error; nothing is written here)
  const bool hist = HIST && M + cm.meta[6] <= a.ocap;
  const int l = lane_id(), wv = wave_id();
  const int64_t chunks = (M + WAVE - 1) / WAVE;
  for (int64_t ch = (int64_t)blockIdx.x * WAVES + wv; ch < chunks; ch += (int64_t)gridDim.x * WAVES) {
    const int64_t k = ch * WAVE + l;
    const bool live = k < M;
    const MDir e = a.mdir[live ? k : M - 1];
    const uint64_t g = mdir_slot(e);
    const int64_t s = mdir_seg(e);
    // words 2..5 are read before the record's size is known, from an address
    // kept inside the buffer (a matched record's message has a 32-byte
    // header, so the buffer holds at least 4 words); they are used only when
    // the record has them
    const uint64_t w0 = e.rword + 6 <= a.ref_words ? e.rword + 2 : a.ref_words - 4;
    const uint64_t hdr = a.ref[e.rword + 1];
    const int hl = a.hlen[g];
    uint64_t x[4], v1[4], v2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[c] = a.ref[w0 + c];
      v1[c] = a.h1[4 * g + c];
      v2[c] = a.h2[4 * g + c];
    }
    const uint64_t H = cm.seg[s].hsize, hp = cm.hpre[s];
    const uint64_t np = HIST ? cm.npre[s] : 0;
    __builtin_amdgcn_sched_barrier(0);  // every load above is in flight before any use
    const bool words6 = (hdr >> 32) >= 6;
    const bool on = live && hl >= 1 && words6;
    int32_t in[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) in[c] = 0;
    uint64_t key = 0;
    bool look = false;
    if (on) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double r = __longlong_as_double((long long)x[c]);
        const double d1 = __longlong_as_double((long long)v1[c]);
        const double d2 = __longlong_as_double((long long)v2[c]);
        in[c] = quantise(r - d1);
        in[4 + c] = hl >= 2 ? quantise(d1 - d2) : 0;
      }
      in[9] = (int32_t)((hdr >> 16) & 0xFFFF);
      in[10] = (int32_t)(hdr & 0xFFFF);
      in[11] = hl;
      look = cell_key_of(x, cell, &key);
    }
    if (look) {  // neighbour count of the record's cell, clamped to 127
      uint64_t h = mix64(key) & (H - 1);
      for (uint64_t probe = 0; probe < H; ++probe) {
        const Entry t = a.tab[hp + h];
        if (t.key == key) {
          in[8] = (int32_t)(t.ci > 127 ? 127 : t.ci);
          break;
        }
        if (t.key == 0) break;
        h = (h + 1) & (H - 1);
      }
    }
    if (a.tcount) {
      // a window: the inputs and the true move (C - R) in quanta of 2^-12
      float tg[4] = {0.f, 0.f, 0.f, 0.f};
      bool w = on;
      if (w) {
        const uint64_t* crec = a.cur + cm.seg[s].cbody / 8 + (uint32_t)a.crw[k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double d = (__longlong_as_double((long long)crec[2 + c]) -
                            __longlong_as_double((long long)x[c])) * 4096.0;
          tg[c] = (float)d;
          w = w && isfinite(tg[c]);
        }
      }
      const uint64_t mask = __ballot(w);
      if (mask) {
        const int lead = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (l == lead) base = atomicAdd(a.tcount, (unsigned long long)__popcll(mask));
        base = __shfl(base, lead, WAVE);
        const int64_t at = (int64_t)base + __popcll(mask & lanemask_lt(l));
        if (w && at < a.tcap) {
#pragma unroll
          for (int c = 0; c < 12; ++c) a.tin[12 * at + c] = in[c];
#pragma unroll
          for (int c = 0; c < 4; ++c) a.ttgt[4 * at + c] = tg[c];
        }
      }
    }
    mlp_in_store(s_in[wv], l, in);
    wave_sync();
    // rows of records that need no prediction are skipped 16 at a time
    const uint64_t need = __ballot(on);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if ((need >> (16 * r)) & 0xFFFFull) mlp16(s_w, ops, s_in[wv], 16 * r, s_h[wv], s_q[wv] + 16 * r);
    wave_sync();
    if (live) {
      a.pred_on[k] = on ? 1 : 0;
      if (on) {
        const int4 q4 = *reinterpret_cast<const int4*>(s_q[wv][l]);
        const int32_t q[4] = {q4.x, q4.y, q4.z, q4.w};
        uint64_t p[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double r = __longlong_as_double((long long)x[c]);
          p[c] = (q[c] != 0 && isfinite(r)) ? (uint64_t)__double_as_longlong(r + (double)q[c] * 0x1p-12) : x[c];
        }
        // (the arena array is 256-byte aligned: 32 bytes per record)
        *reinterpret_cast<ulonglong2*>(a.pred_x + 4 * k) = ulonglong2{p[0], p[1]};
        *reinterpret_cast<ulonglong2*>(a.pred_x + 4 * k + 2) = ulonglong2{p[2], p[3]};
      }
      if (hist) {
        const int64_t o = k + (int64_t)np;  // C' index of matched record k
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          a.o2[4 * o + c] = v1[c];
          a.o1[4 * o + c] = words6 ? x[c] : 0;
        }
        a.olen[o] = (uint8_t)(hl + 1 > 2 ? 2 : hl + 1);
      }
    }
    wave_sync();
  }
}

// History of C' (both sides): a matched record's slot history shifts by one
// exchange (h2 <- h1, h1 <- the reference's words 2..5); new records start
// empty.  C' record index: matched k -> k + new prefix of its segment;
// new r -> matched prefix + n_match of its segment + r.
struct HistArgs {
  Common cm;
  const uint64_t* ref;
  const MDir* mdir;
  const uint64_t* h1;  // nullable: no history yet
  const uint8_t* hlen;
  uint64_t* o1;
  uint64_t* o2;
  uint8_t* olen;
  int64_t ocap;
  bool new_only;       // the matched records' history was written by k_predict
};

// Four lanes per C' record (one per history word), 16 records per wave at a
// time: every load and store instruction of a wave covers 16 consecutive
// records' words.
__global__ __launch_bounds__(BLOCK) void k_hist_out(HistArgs a) {
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t M = cm.meta[5], Nn = cm.meta[6];
  if (M + Nn > a.ocap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fail(cm.status, ERR_CAPACITY);
    return;
  }
  const int l = lane_id(), c = l & 3;
  const int64_t first = a.new_only ? M : 0, total = M + Nn;
  const int64_t stride = (int64_t)gridDim.x * WAVES * 16;
  for (int64_t base = first + ((int64_t)blockIdx.x * WAVES + wave_id()) * 16; base < total; base += stride) {
    const int64_t it = base + (l >> 2);
    if (it >= total) continue;
    if (it < M) {
      const MDir e = a.mdir[it];
      const int64_t s = mdir_seg(e);
      const uint64_t g = mdir_slot(e);
      const uint64_t* rec = a.ref + e.rword;
      const bool has = (rec[1] >> 32) >= 6;
      const int64_t o = it + (int64_t)cm.npre[s];
      a.o2[4 * o + c] = a.h1 ? a.h1[4 * g + c] : 0;
      a.o1[4 * o + c] = has ? rec[2 + c] : 0;
      if (c == 0) {
        const int hl = a.hlen ? a.hlen[g] : 0;
        a.olen[o] = (uint8_t)(hl + 1 > 2 ? 2 : hl + 1);
      }
    } else {
      const int64_t r = it - M;
      const int64_t s = last_le<uint64_t>(cm.npre, 0, cm.nseg, (uint64_t)r);
      const Seg& g = cm.seg[s];
      const int64_t o = (int64_t)(g.mbase + g.n_match) + r;
      a.o1[4 * o + c] = a.o2[4 * o + c] = 0;
      if (c == 0) a.olen[o] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
struct Mem {
  Common cm;
  Entry* tab;
  uint32_t* cwords;
  uint32_t* rwords;
  int32_t* m;
  uint8_t* cflag;   // encoder: matched C records; decoder: matched R slots
  uint64_t* rscan;
  uint64_t* cscan;  // encoder: new C records; decoder: new record words
  uint32_t* nlist;  // encoder: indices of the new C records, in order
  MDir* mdir;
  uint64_t* crw;
  uint64_t* bm;
  uint8_t* gsz;
  uint64_t* gex;
  uint64_t* pred_x;
  uint8_t* pred_on;
  uint32_t* gseg;
  uint32_t* gfirst;
  GDesc* gdesc;     // decoder
  uint32_t* mrw;
  uint64_t* mstart;
  uint8_t* gch;
  uint64_t* juid;
  uint64_t* jhdr;
  uint32_t* jcnt;
  uint64_t* jcnt_pre;
  uint64_t* part;
};

struct Bounds {
  int64_t C, R, H, G, E, T, B, W;
};

Mem carve(Arena& ar, int64_t nseg, const Bounds& b, bool learned) {
  Mem m;
  m.cm.nseg = nseg;
  m.cm.seg = ar.take<Seg>(nseg + 1);
  m.cm.cpre = ar.take<uint64_t>(nseg + 1);
  m.cm.rpre = ar.take<uint64_t>(nseg + 1);
  m.cm.gpre = ar.take<uint64_t>(nseg + 1);
  m.cm.ppre = ar.take<uint64_t>(nseg + 1);
  m.cm.npre = ar.take<uint64_t>(nseg + 1);
  m.cm.tpre = ar.take<uint64_t>(nseg + 1);
  m.cm.bpre = ar.take<uint64_t>(nseg + 1);
  m.cm.hpre = ar.take<uint64_t>(nseg + 1);
  m.cm.jepre = ar.take<uint64_t>(nseg + 1);
  m.cm.fxpre = ar.take<uint64_t>(nseg + 1);
  m.cm.opre = ar.take<uint64_t>(nseg + 1);
  m.cm.cols = ar.take<uint64_t>(COL_MAX * (nseg + 1));
  m.cm.fold = ar.take<uint64_t>(FOLD_SLOTS * (nseg + 1));
  m.cm.meta = ar.take<int64_t>(16);
  m.cm.status = nullptr;
  m.cm.op = 0;
  m.tab = ar.take<Entry>(b.H);
  m.cwords = ar.take<uint32_t>(b.C);
  m.nlist = ar.take<uint32_t>(b.C);
  m.rwords = ar.take<uint32_t>(b.R);
  m.m = ar.take<int32_t>(b.R);
  m.cflag = ar.take<uint8_t>(std::max(b.C, b.R));
  m.rscan = ar.take<uint64_t>(b.R + 1);
  m.cscan = ar.take<uint64_t>(std::max(b.C, b.R) + 1);
  m.mdir = ar.take<MDir>(b.R);
  m.crw = ar.take<uint64_t>(b.R);
  m.bm = ar.take<uint64_t>(b.G);
  m.gsz = ar.take<uint8_t>(b.G);
  m.gex = ar.take<uint64_t>(b.G + 1);
  m.pred_x = learned ? ar.take<uint64_t>(4 * b.R) : nullptr;
  m.pred_on = learned ? ar.take<uint8_t>(b.R) : nullptr;
  m.gseg = ar.take<uint32_t>(b.G);
  m.gfirst = ar.take<uint32_t>(b.G);
  m.gdesc = ar.take<GDesc>(b.G);
  m.mrw = ar.take<uint32_t>(b.R);
  m.mstart = ar.take<uint64_t>(b.R + 1);
  m.gch = learned ? ar.take<uint8_t>(b.G) : nullptr;
  m.juid = ar.take<uint64_t>(b.C + b.R);
  m.jhdr = ar.take<uint64_t>(b.C + b.R);
  m.jcnt = ar.take<uint32_t>(b.E);
  m.jcnt_pre = ar.take<uint64_t>(b.E + 1);
  m.part = ar.take<uint64_t>(2 * (b.C + b.R));
  return m;
}

// True when an array of the history to write overlaps one of the history
// read: the prediction kernel reads the one while it writes the other.
inline bool hist_overlap(const ta_history* in, const ta_history* out) {
  if (!in || !out) return false;
  auto lo = [](const void* p) { return (uintptr_t)p; };
  auto hi = [](const void* p, int64_t n) { return (uintptr_t)p + (uintptr_t)(n > 0 ? n : 0); };
  const uintptr_t ia[3] = {lo(in->h1), lo(in->h2), lo(in->hlen)};
  const uintptr_t ib[3] = {hi(in->h1, 32 * in->cap), hi(in->h2, 32 * in->cap), hi(in->hlen, in->cap)};
  const uintptr_t oa[3] = {lo(out->h1), lo(out->h2), lo(out->hlen)};
  const uintptr_t ob[3] = {hi(out->h1, 32 * out->cap), hi(out->h2, 32 * out->cap), hi(out->hlen, out->cap)};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (ia[i] < ob[j] && oa[j] < ib[i]) return true;
  return false;
}

// Key arrays are 16-byte aligned (one uid and header word pair per record).
inline bool keys_ok(const ta_keys* k) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return al(k->cur) && al(k->ref) && al(k->out) && k->out_cap >= 0 && (k->out || k->out_cap == 0);
}

// Records are >= 20 bytes (two words and an offset), so the byte sizes
// bound the record counts; a record capacity (rec_cap > 0) tightens them and
// the column scans flag larger inputs as capacity errors.
inline int64_t rec_bound(int64_t len, int64_t rec_cap) {
  const int64_t b = len / 20 + 1;
  return rec_cap > 0 && rec_cap + 1 < b ? rec_cap + 1 : b;
}
Bounds enc_bounds(int64_t nseg, int64_t cur_len, int64_t ref_len, int64_t rec_cap) {
  Bounds b;
  b.C = rec_bound(cur_len, rec_cap);
  b.R = rec_bound(ref_len, rec_cap);
  b.H = 4 * (b.C + b.R) + 2 * nseg + 1;
  b.G = ref_len / 512 + nseg + 1;
  // join: per segment at most 130 counting tiles and 2 n/JB_TARGET + 1 buckets
  b.E = 260 * (b.C + b.R) / JB_TARGET + 130 * nseg + 1;
  b.T = (b.C + b.R) / JT + 2 * nseg + 1;
  b.B = 2 * (b.C + b.R) / JB_TARGET + nseg + 1;
  b.W = ref_len / 8 + 1;
  return b;
}
Bounds dec_bounds(int64_t nseg, int64_t enc_len, int64_t ref_len, int64_t rec_cap) {
  Bounds b;
  b.C = rec_bound(enc_len, rec_cap);  // new records
  b.R = rec_bound(ref_len, rec_cap);
  b.H = 4 * b.R + 2 * nseg + 1;  // neighbour-count tables (learned mode)
  b.G = ref_len / 512 + nseg + 1;
  b.E = 1;
  b.T = 1;
  b.B = 1;
  b.W = ref_len / 8 + 1;
  return b;
}

}  // namespace

namespace ta {
size_t encode_scratch(int64_t nseg, int64_t cur_len, int64_t ref_len, int64_t rec_cap, bool learned,
                      int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  const Bounds b = enc_bounds(nseg, cur_len, ref_len, rec_cap);
  carve(ar, nseg, b, learned);
  *tiles = std::max(ceil_div(std::max(std::max(std::max(b.C, b.R), b.E), b.G) + 1, SCAN_TILE_MIN),
                    ceil_div(b.G, EG_TILE)) + 2;
  return ar.used + 256;
}
size_t decode_scratch(int64_t nseg, int64_t enc_len, int64_t ref_len, int64_t out_cap, int64_t rec_cap,
                      bool learned, int64_t* tiles) {
  (void)out_cap;
  Arena ar{nullptr, 0, 0};
  const Bounds b = dec_bounds(nseg, enc_len, ref_len, rec_cap);
  carve(ar, nseg, b, learned);
  *tiles = ceil_div(std::max(std::max(b.C, b.R), b.G) + 1, SCAN_TILE_MIN) + 2;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_delta_encode(ta_ctx* c, int64_t nseg, const uint8_t* cur, int64_t cur_len,
                                     const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                                     const int64_t* ref_off, const ta_predictor* pred, const ta_history* hist_in,
                                     ta_history* hist_out, uint8_t* enc, int64_t enc_cap, int64_t* enc_off,
                                     uint8_t* newref, int64_t newref_cap, int64_t* newref_off, uint8_t* modes,
                                     const ta_keys* keys, void* stream) {
  if (!c || nseg < 0 || !cur_off || !ref_off || !enc_off || !newref_off || cur_len < 0 || ref_len < 0 ||
      enc_cap < 0 || newref_cap < 0 || (cur_len && !cur) || (ref_len && !ref) || (enc_cap && !enc) ||
      (newref_cap && !newref) || (pred && !hist_in) || (keys && !keys_ok(keys)) ||
      hist_overlap(hist_in, hist_out))
    return TA_ERR_INVALID;
  const uint64_t* ckeys = keys ? keys->cur : nullptr;
  const uint64_t* rkeys = keys ? keys->ref : nullptr;
  uint64_t* okeys = keys ? keys->out : nullptr;
  const uint64_t okeys_cap = keys && keys->out ? (uint64_t)keys->out_cap : 0;
  hipStream_t s = (hipStream_t)stream;
  if (nseg == 0) {
    ta_status z = zero_i64(enc_off, 1, s);
    return z ? z : zero_i64(newref_off, 1, s);
  }
  use_family(c, FAM_ENCODE);
  // packed scan fields: < 2^28 records (the record bound the scratch is
  // sized for, checked on the device), < 2^34 words
  if (rec_bound(cur_len, c->rec_cap) >= (1ll << 28) || cur_len / 8 >= (1ll << 34) ||
      rec_bound(ref_len, c->rec_cap) >= (1ll << 28) || ref_len / 8 >= (1ll << 34))
    return TA_ERR_INVALID;
  int64_t tiles;
  ta_status st = ensure_scratch(c, encode_scratch(nseg, cur_len, ref_len, c->rec_cap, pred != nullptr, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const Bounds b = enc_bounds(nseg, cur_len, ref_len, c->rec_cap);
  Mem m = carve(ar, nseg, b, pred != nullptr);
  m.cm.status = c->d_status;
  m.cm.op = c->diff_op;
  const int g = c->grid;
  const int gseg = grid_for(c, nseg, BLOCK);
  const bool few = nseg <= FUSE_NSEG;
  {
    Timed t_match(c, "encode_match", s);  // headers, UID join, layout and directory
    {
      const ClearFirst cf = clear_first(c, ceil_div(b.E + 1, SCAN_TILE));
      const ColScan cs = col_scan(m.cm, {m.cm.cpre, m.cm.rpre, m.cm.hpre, m.cm.tpre, m.cm.jepre, m.cm.bpre},
                                  {0, 1, 2, 10, 11, 12}, {b.C, b.R, b.H, b.T, b.E, b.B});
      if (few) {
        k_enc_setup1<<<1, 1024, 0, s>>>(m.cm, cur, cur_len, cur_off, ref, ref_len, ref_off, cf, cs, 6);
      } else {
        k_enc_setup<<<gseg, BLOCK, 0, s>>>(m.cm, cur, cur_len, cur_off, ref, ref_len, ref_off, cf);
        k_scan_cols<<<6, 1024, 0, s>>>(cs);
      }
    }
    {
      Timed tm(c, "encode_join", s);
      JoinArgs ja{m.cm, cur, ref, m.juid, m.jhdr, m.cwords, m.rwords, m.jcnt, m.jcnt_pre, m.part, m.m, m.cflag, m.tab,
                ckeys, rkeys};
      k_join_count<<<grid_for(c, b.T, 1), BLOCK, 0, s>>>(ja, m.cm.seg, m.cm.tpre, m.cm.cpre, m.cm.rpre, m.cm.jepre);
      k_scan<JCntIn><<<grid_for(c, b.E + 1, scan_tile<JCntIn>()), SCAN_BLOCK, 0, s>>>(JCntIn{m.jcnt}, m.cm.meta + 11, b.E, m.jcnt_pre,
                                                                       lookback(c, 0));
      k_join_scatter<<<grid_for(c, b.T, 1), BLOCK, 0, s>>>(ja, m.cm.seg, m.cm.tpre, m.cm.cpre, m.cm.rpre, m.cm.jepre,
                                                           m.jcnt_pre);
      k_join_bucket<<<grid_for(c, b.B, 1), BLOCK, 0, s>>>(ja, m.cm.seg, m.cm.bpre, m.cm.cpre, m.cm.jepre, m.jcnt_pre);
    }
    k_scan<RMatchIn><<<grid_for(c, b.R + 1, scan_tile<RMatchIn>()), SCAN_BLOCK, 0, s>>>(RMatchIn{m.cm, m.m, m.rwords, m.jhdr, m.cflag, ckeys, rkeys}, m.cm.meta + 1, b.R, m.rscan,
                                                                       lookback(c, 1));
    k_scan<CNewIn><<<grid_for(c, b.C + 1, scan_tile<CNewIn>()), SCAN_BLOCK, 0, s>>>(CNewIn{m.cflag, m.cwords, m.nlist}, m.cm.meta + 0, b.C, m.cscan,
                                                                     lookback(c, 2));
    {
      const ColScan cs = col_scan(m.cm, {m.cm.gpre, m.cm.fxpre, m.cm.opre, m.cm.ppre}, {3, 9, -1, 4}, {b.G, -1, -1, -1});
      if (few) {
        k_enc_layout1<<<1, 1024, 0, s>>>(m.cm, m.rscan, m.cscan, m.mstart, cs, 4, newref, newref_cap, newref_off, m.gex);
      } else {
        k_enc_seg2<<<gseg, BLOCK, 0, s>>>(m.cm, m.rscan, m.cscan, m.mstart);
        k_scan_cols<<<4, 1024, 0, s>>>(cs);
        k_enc_seg3<<<gseg, BLOCK, 0, s>>>(m.cm, newref, newref_cap, newref_off, m.gex);
      }
    }
    k_enc_mdir<<<grid_for(c, b.R, BLOCK * RS_U), BLOCK, 0, s>>>(m.cm, cur, ref, m.m, m.rscan, m.rwords,
                                                                pred || hist_out ? m.mdir : nullptr, m.crw,
                                                                m.mstart, newref, m.gseg, m.gfirst, m.juid, m.jhdr,
                                                                rkeys, okeys, okeys_cap, pred ? m.tab : nullptr,
                                                                pred && hist_in ? hist_in->cap : 0);
  }
  const PredW* pw = pred ? static_cast<const PredW*>(pred->dev) : nullptr;
  if (pw) {
    Timed tm(c, "predict", s);
    k_nbr_build<<<g, BLOCK, 0, s>>>(m.cm, ref, pw, m.tab);
    PredictArgs pa{m.cm,
                   reinterpret_cast<const uint64_t*>(ref),
                   (uint64_t)ref_len / 8,
                   m.mdir,
                   pw,
                   m.tab,
                   hist_in->h1,
                   hist_in->h2,
                   hist_in->hlen,
                   m.pred_x,
                   m.pred_on,
                   hist_out ? hist_out->h1 : nullptr,
                   hist_out ? hist_out->h2 : nullptr,
                   hist_out ? hist_out->hlen : nullptr,
                   hist_out ? hist_out->cap : 0,
                   reinterpret_cast<const uint64_t*>(cur),
                   m.crw,
                   c->tap_in,
                   c->tap_tgt,
                   c->tap_cap,
                   c->tap_count};
    if (hist_out)
      k_predict<true><<<grid_for(c, b.R, WAVE * WAVES), BLOCK, 0, s>>>(pa);
    else
      k_predict<false><<<grid_for(c, b.R, WAVE * WAVES), BLOCK, 0, s>>>(pa);
  }
  {
    Timed tm(c, "encode_groups", s);
    GroupArgs ga{m.cm, reinterpret_cast<const uint64_t*>(cur), reinterpret_cast<const uint64_t*>(ref), m.crw,
                 m.mstart, reinterpret_cast<uint64_t*>(newref), enc, enc_cap, m.bm, m.gsz, m.gex,
                 m.pred_x, m.pred_on, m.gch};
    const int gg = grid_for(c, b.G, EG_TILE);
    const LookBack lb = lookback(c, 3);
    if (pw) {
      if (c->diff_op)
        k_enc_groups<1, true><<<gg, EG_BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst, lb);
      else
        k_enc_groups<0, true><<<gg, EG_BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst, lb);
      k_choose_mode<<<grid_for(c, nseg, 1), BLOCK, 0, s>>>(m.cm, m.gch);
      const int gf = grid_for(c, b.G, WAVES * WAVE);
      if (c->diff_op)
        k_enc_fixup<1><<<gf, BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst);
      else
        k_enc_fixup<0><<<gf, BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst);
    } else {
      if (c->diff_op)
        k_enc_groups<1, false><<<gg, EG_BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst, lb);
      else
        k_enc_groups<0, false><<<gg, EG_BLOCK, 0, s>>>(ga, m.cm.seg, m.cm.gpre, m.gseg, m.gfirst, lb);
    }
  }
  k_enc_fixed<<<g, BLOCK, 0, s>>>(m.cm, m.m, m.bm, m.gsz, m.gch, m.gex, enc, enc_cap, enc_off, modes,
                                  NewArgs{m.cscan, m.nlist, m.cwords, cur, newref, m.juid, m.jhdr, ckeys, okeys,
                                          (uint64_t)okeys_cap});
  if (hist_out) {
    HistArgs ha{m.cm, reinterpret_cast<const uint64_t*>(ref), m.mdir, hist_in ? hist_in->h1 : nullptr,
                hist_in ? hist_in->hlen : nullptr, hist_out->h1, hist_out->h2, hist_out->hlen, hist_out->cap,
                pw != nullptr};
    k_hist_out<<<g, BLOCK, 0, s>>>(ha);
  }
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_delta_decode(ta_ctx* c, int64_t nseg, const uint8_t* enc, int64_t enc_len,
                                     const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                                     const int64_t* ref_off, const ta_predictor* pred, const ta_history* hist_in,
                                     ta_history* hist_out, uint8_t* out, int64_t out_cap, int64_t* out_off,
                                     const ta_keys* keys, void* stream) {
  if (!c || nseg < 0 || !enc_off || !ref_off || !out_off || enc_len < 0 || ref_len < 0 || out_cap < 0 ||
      (enc_len && !enc) || (ref_len && !ref) || (out_cap && !out) || (pred && !hist_in) || (keys && !keys_ok(keys)) ||
      hist_overlap(hist_in, hist_out))
    return TA_ERR_INVALID;
  const uint64_t* rkeys = keys ? keys->ref : nullptr;
  uint64_t* okeys = keys ? keys->out : nullptr;
  const uint64_t okeys_cap = keys && keys->out ? (uint64_t)keys->out_cap : 0;
  hipStream_t s = (hipStream_t)stream;
  if (nseg == 0) return zero_i64(out_off, 1, s);
  use_family(c, FAM_DECODE);
  if (enc_len / 8 >= (1ll << 34) || rec_bound(ref_len, c->rec_cap) >= (1ll << 28) || ref_len / 8 >= (1ll << 34))
    return TA_ERR_INVALID;
  int64_t tiles;
  ta_status st = ensure_scratch(c, decode_scratch(nseg, enc_len, ref_len, out_cap, c->rec_cap, pred != nullptr, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const Bounds b = dec_bounds(nseg, enc_len, ref_len, c->rec_cap);
  Mem m = carve(ar, nseg, b, pred != nullptr);
  m.cm.status = c->d_status;
  m.cm.op = c->diff_op;
  const int g = c->grid;
  const int gseg = grid_for(c, nseg, BLOCK);
  {
    const ClearFirst cf = clear_first(c, ceil_div(b.R + 1, SCAN_TILE));
    const ColScan cs = col_scan(m.cm, {m.cm.rpre, m.cm.gpre, m.cm.npre, m.cm.opre, m.cm.ppre, m.cm.hpre},
                                {1, 3, 6, -1, 4, 2}, {b.R, b.G, b.C, -1, -1, b.H});
    if (nseg <= FUSE_NSEG) {
      k_dec_setup1<<<1, 1024, 0, s>>>(m.cm, enc, enc_len, enc_off, ref, ref_len, ref_off, pred != nullptr, cf, cs, 6);
    } else {
      k_dec_setup<<<gseg, BLOCK, 0, s>>>(m.cm, enc, enc_len, enc_off, ref, ref_len, ref_off, pred != nullptr, cf);
      k_scan_cols<<<6, 1024, 0, s>>>(cs);
    }
  }
  k_dec_rslots<<<grid_for(c, b.R, BLOCK * RL_U), BLOCK, 0, s>>>(m.cm, enc, ref, m.rwords, m.cflag, m.cm.seg, m.cm.rpre,
                                                                rkeys);
  k_scan<DMatchIn><<<grid_for(c, b.R + 1, scan_tile<DMatchIn>()), SCAN_BLOCK, 0, s>>>(DMatchIn{m.cflag, m.rwords}, m.cm.meta + 1, b.R,
                                                                     m.rscan, lookback(c, 0));
  k_scan<DNewIn><<<grid_for(c, b.C + 1, scan_tile<DNewIn>()), SCAN_BLOCK, 0, s>>>(DNewIn{m.cm, enc}, m.cm.meta + 6, b.C, m.cscan,
                                                                   lookback(c, 1));
  k_scan<DGroupIn><<<grid_for(c, b.G + 1, scan_tile<DGroupIn>()), SCAN_BLOCK, 0, s>>>(DGroupIn{m.cm, enc}, m.cm.meta + 3, b.G, m.gex,
                                                                     lookback(c, 2));
  k_dec_seg2<<<gseg, BLOCK, 0, s>>>(m.cm, m.rscan, m.cscan, m.gex, out, out_cap, out_off, m.mstart);
  k_dec_mdir<<<grid_for(c, b.R, BLOCK * RS_U), BLOCK, 0, s>>>(m.cm, ref, m.cflag, m.rscan, m.rwords,
                                                              pred || hist_out ? m.mdir : nullptr, m.mstart, out, enc,
                                                              m.gex, m.gdesc, m.mrw, rkeys, okeys, okeys_cap, m.cscan,
                                                              pred && hist_in ? hist_in->cap : -1,
                                                              pred ? m.tab : nullptr);
  const PredW* pw = pred ? static_cast<const PredW*>(pred->dev) : nullptr;
  if (pw) {
    Timed tm(c, "predict", s);
    k_nbr_build<<<g, BLOCK, 0, s>>>(m.cm, ref, pw, m.tab);
    PredictArgs pa{m.cm,
                   reinterpret_cast<const uint64_t*>(ref),
                   (uint64_t)ref_len / 8,
                   m.mdir,
                   pw,
                   m.tab,
                   hist_in->h1,
                   hist_in->h2,
                   hist_in->hlen,
                   m.pred_x,
                   m.pred_on,
                   hist_out ? hist_out->h1 : nullptr,
                   hist_out ? hist_out->h2 : nullptr,
                   hist_out ? hist_out->hlen : nullptr,
                   hist_out ? hist_out->cap : 0,
                   nullptr,
                   nullptr,
                   nullptr,
                   nullptr,
                   0,
                   nullptr};
    if (hist_out)
      k_predict<true><<<grid_for(c, b.R, WAVE * WAVES), BLOCK, 0, s>>>(pa);
    else
      k_predict<false><<<grid_for(c, b.R, WAVE * WAVES), BLOCK, 0, s>>>(pa);
  }
  {
    Timed tm(c, "decode_unpack", s);
    UnpackArgs ua{m.cm,     enc,       reinterpret_cast<const uint64_t*>(ref), m.mrw, m.mstart,
                  m.pred_x, m.pred_on, reinterpret_cast<uint64_t*>(out)};
    const int gu = grid_for(c, b.G, WAVES * UNPACK_PG);
    if (c->diff_op)
      k_dec_unpack<1><<<gu, BLOCK, 0, s>>>(ua, m.gdesc, enc);
    else
      k_dec_unpack<0><<<gu, BLOCK, 0, s>>>(ua, m.gdesc, enc);
  }
  if (hist_out) {
    HistArgs ha{m.cm, reinterpret_cast<const uint64_t*>(ref), m.mdir, hist_in ? hist_in->h1 : nullptr,
                hist_in ? hist_in->hlen : nullptr, hist_out->h1, hist_out->h2, hist_out->hlen, hist_out->cap,
                pw != nullptr};
    k_hist_out<<<g, BLOCK, 0, s>>>(ha);
  }
  TA_LAUNCH_CHECK();
  return TA_OK;
}
