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
//   k_enc_setup   one block: message headers, record counts, hash sizes and
//                 their prefixes
//   k_clear_tab   empty hash table, flags
//   k_enc_insert  every C and R record: validate, insert its uid into the
//                 segment's open-addressing table (duplicates detected on both
//                 sides); XOR of reference uids per segment
//   k_enc_match   every R slot: matched C record (same uid and header word)
//   k_scan x2     packed (count << 34 | words) prefixes over R slots (matched)
//                 and C records (new)
//   k_enc_seg2    one block: per segment sizes, section layout, C' headers
//   k_enc_mdir    matched-record directory (C word, R word, residual start)
//   k_enc_xor     one wave per 64-word residual group: C xor X, C' words,
//                 bitmap, length nibbles and significant bytes assembled in
//                 LDS; a look-back over group block sizes places the blocks
//   k_enc_fin     one block: encoding offsets and headers
//   k_enc_fixed   presence bitmaps, word bitmaps, block size tables, new
//                 record sizes, C' offsets of new records
//   k_newcopy     new records into the encoding and into C'
// The decoder mirrors these steps.
#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_predict.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int PK = 34;  // packed scan value: count << 34 | words
constexpr uint64_t WMASK = (1ull << PK) - 1;
constexpr int XG = 4;                 // groups per wave in the xor/unpack kernels
constexpr int TILE_G = WAVES * XG;    // groups per tile
constexpr int BLK_MAX = 544;          // 32 nibble bytes + 512 significant bytes
constexpr uint32_t ANY_ERR = (1u << ERR_INVALID) | (1u << ERR_CAPACITY) | (1u << ERR_CORRUPT) | (1u << ERR_REF) |
                             (1u << ERR_INTERNAL);

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
};

struct MDir {
  uint64_t cword;   // encoder: C record word index in cur; decoder: unused
  uint64_t rword;   // R record word index in ref
  uint64_t dstart;  // global residual word position of the record
  uint64_t g;       // global reference slot
};

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
__device__ inline void seg_xor(uint64_t* fold_base, size_t stride_words, int64_t s, bool active, uint64_t v) {
  uint64_t pending = __ballot(active);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int64_t s0 = __shfl(s, leader, WAVE);
    const bool mine = active && s == s0;
    const uint64_t part = wave_xor(mine ? v : 0);
    if (lane_id() == leader) atomicXor((unsigned long long*)(fold_base + stride_words * s0), (unsigned long long)part);
    pending &= ~__ballot(mine);
  }
}

struct Common {
  int64_t nseg;
  Seg* seg;
  uint64_t* cpre;  // [nseg+1] record prefixes (C / encoding new records)
  uint64_t* rpre;  // [nseg+1] reference slot prefixes
  uint64_t* gpre;  // [nseg+1] residual group prefixes
  uint64_t* ppre;  // [nseg+1] presence word prefixes
  uint64_t* npre;  // [nseg+1] new record prefixes
  int64_t* meta;   // [0] C records [1] R records [2] hash slots [3] groups [4] presence words [5] matched
                   // [6] new records [7] new words [8] C+R records
  uint32_t* status;
};

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

__global__ __launch_bounds__(1024) void k_enc_setup(Common cm, const uint8_t* cur, int64_t cur_len,
                                                    const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                                                    const int64_t* ref_off, ClearFirst cf) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry[3];
  BlockScan1024 bs{s_w};
  do_clear_first(cf);
  if (threadIdx.x < 3) s_carry[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < cm.nseg; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    uint64_t nc = 0, nr = 0, hs = 0;
    if (s < cm.nseg) {
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
      hs = pow2ceil(2 * (nc + nr));
      g.hsize = hs;
      g.fold = 0;
      g.mode = 0;
    }
    uint64_t t0, t1, t2;
    const uint64_t e0 = bs.excl(nc, &t0), e1 = bs.excl(nr, &t1), e2 = bs.excl(hs, &t2);
    if (s < cm.nseg) {
      cm.cpre[s] = s_carry[0] + e0;
      cm.rpre[s] = s_carry[1] + e1;
      cm.seg[s].hbase = s_carry[2] + e2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry[0] += t0;
      s_carry[1] += t1;
      s_carry[2] += t2;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cm.cpre[cm.nseg] = s_carry[0];
    cm.rpre[cm.nseg] = s_carry[1];
    cm.meta[0] = s_carry[0];
    cm.meta[1] = s_carry[1];
    cm.meta[2] = s_carry[2];
    cm.meta[8] = s_carry[0] + s_carry[1];
  }
}

__global__ __launch_bounds__(BLOCK) void k_clear_tab(Common cm, Entry* tab, uint8_t* cflag) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t H = cm.meta[2], Ct = cm.meta[0];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < H; i += stride) {
    tab[i].key = 0;
    tab[i].ci = NONE;
    tab[i].ri = NONE;
  }
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < Ct; i += stride) cflag[i] = 0;
}

__global__ __launch_bounds__(BLOCK) void k_enc_insert(Common cm, const uint8_t* cur, const uint8_t* ref, Entry* tab,
                                                      uint32_t* cwords, uint32_t* rwords, uint32_t* rslot) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Ct = cm.meta[0], total = cm.meta[8];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  // whole waves iterate together so the per-segment XOR fold can use the wave
  const int64_t start = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t rounds = (total + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t g = start + it * stride;
    const bool active = g < total;
    const bool isC = g < Ct;
    int64_t s = 0;
    uint64_t uid = 0;
    bool okr = false;
    if (active) {
      const uint64_t loc = isC ? (uint64_t)g : (uint64_t)(g - Ct);
      s = seg_of(isC ? cm.cpre : cm.rpre, cm.nseg, loc);
      const Seg& sg = cm.seg[s];
      const uint64_t i = loc - (isC ? cm.cpre[s] : cm.rpre[s]);
      const uint8_t* m = isC ? cur + sg.cmsg : ref + sg.rmsg;
      const uint32_t n = (uint32_t)(isC ? sg.nc : sg.nr);
      const uint64_t rw = isC ? sg.rwc : sg.rwr;
      uint32_t o;
      uint64_t hdr;
      if (tam1_record(m, n, rw, (uint32_t)i, &o, &hdr)) {
        uid = ld64(tam1_records(m, n) + 8 * (uint64_t)o);
        okr = uid != 0;
      }
      if (!okr) {
        fail(cm.status, ERR_INVALID);
      } else {
        const uint64_t H = sg.hsize, hb = sg.hbase;
        uint64_t h = mix64(uid) & (H - 1);
        uint32_t slot = NONE;
        for (uint64_t probe = 0; probe < H; ++probe) {
          const unsigned long long prev = atomicCAS(&tab[hb + h].key, 0ull, (unsigned long long)uid);
          if (prev == 0ull || prev == (unsigned long long)uid) {
            uint32_t* ip = isC ? &tab[hb + h].ci : &tab[hb + h].ri;
            if (atomicCAS(ip, NONE, (uint32_t)i) != NONE) fail(cm.status, ERR_INVALID);  // duplicate uid
            slot = (uint32_t)h;
            break;
          }
          h = (h + 1) & (H - 1);
        }
        const uint32_t words = (uint32_t)(hdr >> 32);
        if (isC) {
          cwords[g] = words;
        } else {
          rwords[g - Ct] = words;
          rslot[g - Ct] = slot;
        }
      }
    }
    // per segment XOR of the reference uids (identity of the reference)
    const bool isR = active && !isC && okr;
    seg_xor(&cm.seg[0].fold, sizeof(Seg) / 8, s, isR, uid);
  }
}

__global__ __launch_bounds__(BLOCK) void k_enc_match(Common cm, const uint8_t* cur, const uint8_t* ref,
                                                     const Entry* tab, const uint32_t* rslot, int32_t* m,
                                                     uint8_t* cflag) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < Rt; g += (int64_t)gridDim.x * BLOCK) {
    const int64_t s = seg_of(cm.rpre, cm.nseg, (uint64_t)g);
    const Seg& sg = cm.seg[s];
    const uint64_t j = g - cm.rpre[s];
    const uint32_t i = tab[sg.hbase + rslot[g]].ci;
    int32_t res = -1;
    if (i != NONE) {
      const uint32_t oc = ld32(cur + sg.cmsg + 32 + 4 * (uint64_t)i);
      const uint32_t orr = ld32(ref + sg.rmsg + 32 + 4 * j);
      const uint64_t hc = ld64(cur + sg.cbody + 8 * (uint64_t)oc + 8);
      const uint64_t hr = ld64(ref + sg.rbody + 8 * (uint64_t)orr + 8);
      if (hc == hr) {
        res = (int32_t)i;
        cflag[cm.cpre[s] + i] = 1;
      }
    }
    m[g] = res;
  }
}

struct RMatchIn {  // count << 34 | words of matched reference slots
  const int32_t* m;
  const uint32_t* rwords;
  __device__ uint64_t operator()(int64_t g) const { return m[g] >= 0 ? ((1ull << PK) | rwords[g]) : 0; }
};
struct CNewIn {  // count << 34 | words of new current records
  const uint8_t* cflag;
  const uint32_t* cwords;
  __device__ uint64_t operator()(int64_t g) const { return cflag[g] ? 0 : ((1ull << PK) | cwords[g]); }
};

// Per segment layout after matching; block-wide prefixes; C' headers.
__global__ __launch_bounds__(1024) void k_enc_seg2(Common cm, const uint64_t* rscan, const uint64_t* cscan,
                                                   uint8_t* newref, int64_t newref_cap, int64_t* newref_off,
                                                   uint64_t* gex) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry[4];
  BlockScan1024 bs{s_w};
  const bool bad = (status_of(cm.status) & ANY_ERR) != 0;
  if (threadIdx.x < 4) s_carry[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < cm.nseg; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    uint64_t G = 0, fixed = 0, osize = 0, PG = 0;
    if (s < cm.nseg && !bad) {
      Seg& g = cm.seg[s];
      const uint64_t rs = rscan[cm.rpre[s]], re = rscan[cm.rpre[s + 1]];
      const uint64_t cs = cscan[cm.cpre[s]], ce = cscan[cm.cpre[s + 1]];
      g.mbase = rs >> PK;
      g.n_match = (re >> PK) - g.mbase;
      g.dbase = rs & WMASK;
      g.W = (re & WMASK) - g.dbase;
      g.nbase = cs >> PK;
      g.n_new = (ce >> PK) - g.nbase;
      g.npbase = cs & WMASK;
      g.new_words = (ce & WMASK) - g.npbase;
      G = (g.W + 63) / 64;
      PG = (g.nr + 63) / 64;
      g.G = G;
      g.PG = PG;
      fixed = 64 + 8 * PG + 8 * G + round8(G) + round8(4 * g.n_new) + 8 * g.new_words;
      g.fixed = fixed;
      osize = tam1_size(g.n_match + g.n_new, g.W + g.new_words);
    }
    uint64_t t0, t1, t2, t3;
    const uint64_t e0 = bs.excl(G, &t0), e1 = bs.excl(fixed, &t1), e2 = bs.excl(osize, &t2), e3 = bs.excl(PG, &t3);
    if (s < cm.nseg && !bad) {
      cm.gpre[s] = s_carry[0] + e0;
      cm.seg[s].fixed_excl = s_carry[1] + e1;
      cm.seg[s].oref = s_carry[2] + e2;
      newref_off[s] = (int64_t)(s_carry[2] + e2);
      cm.ppre[s] = s_carry[3] + e3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry[0] += t0;
      s_carry[1] += t1;
      s_carry[2] += t2;
      s_carry[3] += t3;
    }
    __syncthreads();
  }
  if (bad) return;
  const bool fits = s_carry[2] <= (uint64_t)newref_cap;
  if (threadIdx.x == 0) {
    cm.gpre[cm.nseg] = s_carry[0];
    cm.ppre[cm.nseg] = s_carry[3];
    newref_off[cm.nseg] = (int64_t)s_carry[2];
    cm.meta[3] = s_carry[0];
    cm.meta[4] = s_carry[3];
    cm.meta[5] = rscan[cm.meta[1]] >> PK;
    cm.meta[6] = cscan[cm.meta[0]] >> PK;
    cm.meta[7] = cscan[cm.meta[0]] & WMASK;
    cm.meta[9] = (int64_t)s_carry[1];  // fixed total
    gex[s_carry[0]] = 0;
    if (!fits) fail(cm.status, ERR_CAPACITY);
  }
  if (!fits) return;
  for (int64_t s = threadIdx.x; s < cm.nseg; s += 1024) {
    const Seg& g = cm.seg[s];
    uint8_t* o = newref + g.oref;
    const uint64_t n = g.n_match + g.n_new;
    uint64_t* h = reinterpret_cast<uint64_t*>(o);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);
    h[1] = n;
    h[2] = g.W + g.new_words;
    h[3] = 0;
    if (n & 1) *reinterpret_cast<uint32_t*>(o + 32 + 4 * n) = 0;
  }
}

// Directory of matched records; C' offsets of matched records.
__global__ __launch_bounds__(BLOCK) void k_enc_mdir(Common cm, const uint8_t* cur, const uint8_t* ref,
                                                    const int32_t* m, const uint64_t* rscan, MDir* mdir,
                                                    uint8_t* newref) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < Rt; g += (int64_t)gridDim.x * BLOCK) {
    const int32_t i = m[g];
    if (i < 0) continue;
    const int64_t s = seg_of(cm.rpre, cm.nseg, (uint64_t)g);
    const Seg& sg = cm.seg[s];
    const uint64_t j = g - cm.rpre[s];
    const uint64_t k = rscan[g] >> PK;
    const uint64_t d = rscan[g] & WMASK;
    MDir e;
    e.cword = sg.cbody / 8 + ld32(cur + sg.cmsg + 32 + 4 * (uint64_t)i);
    e.rword = sg.rbody / 8 + ld32(ref + sg.rmsg + 32 + 4 * j);
    e.dstart = d;
    e.g = (uint64_t)g;
    mdir[k] = e;
    *reinterpret_cast<uint32_t*>(newref + sg.oref + 32 + 4 * (k - sg.mbase)) = (uint32_t)(d - sg.dbase);
  }
}

// Record of each lane of a 64-word residual window starting at global
// residual position dq0 inside segment sg: index into mdir.
__device__ inline uint64_t window_record(const MDir* mdir, uint64_t kbeg, uint64_t kend, uint64_t dq0) {
  // k0: last matched record of the segment starting at or before dq0 (uniform)
  uint64_t lo = kbeg, hi = kend;
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (mdir[mid].dstart <= dq0) lo = mid;
    else hi = mid;
  }
  const uint64_t k0 = lo;
  const int l = lane_id();
  const uint64_t kk = k0 + 1 + (uint64_t)l;
  uint64_t bit = 0;
  if (kk < kend) {
    const uint64_t rel = mdir[kk].dstart - dq0;
    if (rel < 64) bit = 1ull << rel;
  }
  const uint64_t starts = wave_or(bit);
  return k0 + (uint64_t)__popcll(starts & lanemask_le(l));
}

// Assemble the block of one group in LDS.  Returns the block size in bytes.
__device__ inline uint32_t build_block(uint64_t D, uint8_t* blk, uint64_t* bitmap_out) {
  const int l = lane_id();
  const uint64_t bm = __ballot(D != 0);
  const uint32_t len = D ? (uint32_t)(8 - (__clzll((long long)D) >> 3)) : 0u;
  const uint32_t popc = (uint32_t)__popcll(bm);
  const uint32_t nib = (popc + 1) / 2;
  const uint64_t sig_incl = wave_incl_scan(len);
  const uint64_t sig_tot = uniform64(__shfl(sig_incl, 63, WAVE));
  const uint32_t size = (uint32_t)round8(nib + sig_tot);
  // zero the block
  uint64_t* b64 = reinterpret_cast<uint64_t*>(blk);
  for (uint32_t k = l; k < size / 8; k += WAVE) b64[k] = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  const uint32_t t = (uint32_t)__popcll(bm & lanemask_lt(l));
  const uint64_t after = bm & ~lanemask_le(l);
  const int nl = after ? (__ffsll((unsigned long long)after) - 1) : l;
  const uint32_t len_next = (uint32_t)__shfl((int)len, nl, WAVE);
  if (D && !(t & 1)) blk[t / 2] = (uint8_t)(len | ((after ? len_next : 0u) << 4));
  if (D) {
    const uint32_t so = nib + (uint32_t)(sig_incl - len);
    for (uint32_t b = 0; b < len; ++b) blk[so + b] = (uint8_t)(D >> (8 * b));
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  *bitmap_out = bm;
  return size;
}

struct XorArgs {
  Common cm;
  const uint64_t* cur;
  const uint64_t* ref;
  const MDir* mdir;
  uint8_t* enc;
  int64_t enc_cap;
  uint64_t* newref;
  uint64_t* bm;     // [groups] word bitmaps
  uint8_t* gsz;     // [groups] block sizes / 8
  uint64_t* gex;    // [groups+1] exclusive prefix of block bytes
  const PredW* pw;  // learned mode: predictor (nullptr: plain)
  const uint64_t* pred_x;  // learned: predicted words 2..5 per matched record [k][4]
  const uint8_t* pred_on;  // learned: record k predicted
  LookBack lb;
};

__global__ __launch_bounds__(BLOCK) void k_enc_xor(XorArgs a) {
  __shared__ uint64_t s_blk[TILE_G][BLK_MAX / 8];
  __shared__ uint32_t s_size[TILE_G];
  __shared__ uint64_t s_pre[TILE_G];
  __shared__ uint32_t s_ticket;
  __shared__ uint64_t s_excl, s_agg;
  lb_clear_next(a.lb);
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Gt = cm.meta[3];
  const int64_t ntiles = (Gt + TILE_G - 1) / TILE_G;
  const int l = lane_id(), wv = wave_id();
  for (;;) {
    const uint32_t t = lb_take_ticket(a.lb, &s_ticket);
    if ((int64_t)t >= ntiles) break;
    for (int x = 0; x < XG; ++x) {
      const int loc = wv * XG + x;
      const int64_t gg = (int64_t)t * TILE_G + loc;
      if (gg >= Gt) {
        if (l == 0) s_size[loc] = 0;
        continue;
      }
      const int64_t s = seg_of(cm.gpre, cm.nseg, (uint64_t)gg);
      const Seg& sg = cm.seg[s];
      const uint64_t lg = (uint64_t)gg - cm.gpre[s];
      const uint64_t q = 64 * lg + (uint64_t)l;
      const uint64_t dq0 = sg.dbase + 64 * lg;
      const uint64_t k = window_record(a.mdir, sg.mbase, sg.mbase + sg.n_match, dq0);
      uint64_t D = 0;
      if (q < sg.W) {
        const MDir e = a.mdir[k];
        const uint64_t w = dq0 + (uint64_t)l - e.dstart;
        const uint64_t c = a.cur[e.cword + w];
        uint64_t x_ = a.ref[e.rword + w];
        if (sg.mode == 1 && w >= 2 && w < 6 && a.pred_on[k]) x_ = a.pred_x[4 * k + (w - 2)];
        D = c ^ x_;
        a.newref[(sg.oref + 32 + 8 * ((sg.n_match + sg.n_new + 1) / 2)) / 8 + q] = c;
      }
      uint64_t bm;
      const uint32_t size = build_block(D, reinterpret_cast<uint8_t*>(s_blk[loc]), &bm);
      if (l == 0) {
        s_size[loc] = size;
        a.bm[gg] = bm;
        a.gsz[gg] = (uint8_t)(size / 8);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t run = 0;
      for (int i = 0; i < TILE_G; ++i) {
        s_pre[i] = run;
        run += s_size[i];
      }
      s_agg = run;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
      const uint64_t e = lb_exclusive(a.lb, t, s_agg);
      if (threadIdx.x == 0) s_excl = e;
    }
    __syncthreads();
    for (int x = 0; x < XG; ++x) {
      const int loc = wv * XG + x;
      const int64_t gg = (int64_t)t * TILE_G + loc;
      if (gg >= Gt) continue;
      const uint64_t V = s_excl + s_pre[loc];
      if (l == 0) a.gex[gg] = V;
      const uint32_t size = s_size[loc];
      if (!size) continue;
      const int64_t s = seg_of(cm.gpre, cm.nseg, (uint64_t)gg);
      const Seg& sg = cm.seg[s];
      const uint64_t at = sg.fixed_excl + sg.fixed + V;
      if (at + size > (uint64_t)a.enc_cap) {
        if (l == 0) fail(cm.status, ERR_CAPACITY);
        continue;
      }
      uint64_t* dst = reinterpret_cast<uint64_t*>(a.enc + at);
      for (uint32_t w = l; w < size / 8; w += WAVE) dst[w] = s_blk[loc][w];
    }
    if ((int64_t)t == ntiles - 1 && threadIdx.x == 0) a.gex[Gt] = s_excl + s_agg;
    __syncthreads();
  }
}

// Encoding offsets and headers.
__global__ __launch_bounds__(1024) void k_enc_fin(Common cm, const uint64_t* gex, uint8_t* enc, int64_t enc_cap,
                                                  int64_t* enc_off, uint8_t* modes) {
  if (status_of(cm.status) & ANY_ERR) return;
  const uint64_t total = (uint64_t)cm.meta[9] + gex[cm.meta[3]];
  const bool fits = total <= (uint64_t)enc_cap;
  if (threadIdx.x == 0) {
    enc_off[cm.nseg] = (int64_t)total;
    if (!fits) fail(cm.status, ERR_CAPACITY);
  }
  for (int64_t s = threadIdx.x; s < cm.nseg; s += 1024) {
    Seg& g = cm.seg[s];
    const uint64_t off = g.fixed_excl + gex[cm.gpre[s]];
    g.encm = off;
    enc_off[s] = (int64_t)off;
    if (modes) modes[s] = (uint8_t)g.mode;
    if (!fits) continue;
    uint64_t* h = reinterpret_cast<uint64_t*>(enc + off);
    h[0] = (uint64_t)TAD1_MAGIC | (1ull << 32) | ((uint64_t)g.mode << 48) | (1ull << 56);
    h[1] = g.nr | (g.n_match << 32);
    h[2] = g.n_new;
    h[3] = g.rwr;
    h[4] = g.fold;
    h[5] = g.W;
    h[6] = g.new_words;
    h[7] = gex[cm.gpre[s + 1]] - gex[cm.gpre[s]];
  }
}

// Presence bitmaps (one wave per 64 reference slots), word bitmaps and block
// size tables (per group), new record sizes and C' offsets (per C record).
__global__ __launch_bounds__(BLOCK) void k_enc_fixed(Common cm, const int32_t* m, const uint8_t* cflag,
                                                     const uint32_t* cwords, const uint64_t* cscan,
                                                     const uint64_t* bm, const uint8_t* gsz, uint8_t* enc,
                                                     int64_t enc_cap, uint8_t* newref) {
  if (status_of(cm.status) & ANY_ERR) return;
  // presence items first, padded to whole blocks so that every wave of the
  // range works on one presence word; then groups, then C records
  const int64_t A = (64 * cm.meta[4] + BLOCK - 1) / BLOCK * BLOCK, B = cm.meta[3], Cn = cm.meta[0];
  const int64_t total = A + B + Cn;
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  const int l = lane_id();
  for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < total; base += stride) {
    const int64_t it = base + threadIdx.x;
    if (base < A) {  // whole waves: presence words (A is a multiple of 64, BLOCK too)
      const int64_t pw = (base + 64 * wave_id()) / 64;
      bool bit = false;
      int64_t s = 0;
      if (pw < cm.meta[4]) {
        s = seg_of(cm.ppre, cm.nseg, (uint64_t)pw);
        const uint64_t j = 64 * (pw - cm.ppre[s]) + (uint64_t)l;
        bit = j < cm.seg[s].nr && m[cm.rpre[s] + j] >= 0;
      }
      const uint64_t word = __ballot(bit);
      if (pw < cm.meta[4] && l == 0) {
        const Seg& g = cm.seg[s];
        *reinterpret_cast<uint64_t*>(enc + g.encm + 64 + 8 * (pw - cm.ppre[s])) = word;
      }
      continue;
    }
    if (it >= total) continue;
    if (it < A + B) {
      const int64_t gg = it - A;
      const int64_t s = seg_of(cm.gpre, cm.nseg, (uint64_t)gg);
      const Seg& g = cm.seg[s];
      const uint64_t lg = gg - cm.gpre[s];
      uint8_t* sec = enc + g.encm + 64 + 8 * g.PG;
      *reinterpret_cast<uint64_t*>(sec + 8 * lg) = bm[gg];
      sec += 8 * g.G;
      sec[lg] = gsz[gg];
      if (lg == g.G - 1)
        for (uint64_t b = g.G; b < round8(g.G); ++b) sec[b] = 0;
    } else {
      const int64_t gc = it - A - B;
      if (cflag[gc]) continue;
      const int64_t s = seg_of(cm.cpre, cm.nseg, (uint64_t)gc);
      const Seg& g = cm.seg[s];
      const uint64_t r = (cscan[gc] >> PK) - g.nbase;
      const uint64_t np = (cscan[gc] & WMASK) - g.npbase;
      uint8_t* ns = enc + g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G);
      *reinterpret_cast<uint32_t*>(ns + 4 * r) = cwords[gc];
      if (r == g.n_new - 1 && (g.n_new & 1)) *reinterpret_cast<uint32_t*>(ns + 4 * (r + 1)) = 0;
      *reinterpret_cast<uint32_t*>(newref + g.oref + 32 + 4 * (g.n_match + r)) = (uint32_t)(g.W + np);
    }
  }
}

// New records, word by word: from C into the encoding and C'.
__global__ __launch_bounds__(BLOCK) void k_enc_newcopy(Common cm, const uint64_t* cscan, const uint8_t* cflag,
                                                       const uint8_t* cur, uint8_t* enc, uint8_t* newref) {
  if (status_of(cm.status) & ANY_ERR) return;
  const uint64_t NW = (uint64_t)cm.meta[7];
  const int64_t Cn = cm.meta[0];
  for (uint64_t q = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; q < NW; q += (uint64_t)gridDim.x * BLOCK) {
    // last C record whose new-word prefix is <= q: a new record holding q
    int64_t lo = 0, hi = Cn;
    while (hi - lo > 1) {
      const int64_t mid = lo + (hi - lo) / 2;
      if ((cscan[mid] & WMASK) <= q) lo = mid;
      else hi = mid;
    }
    const int64_t gc = lo;
    const int64_t s = seg_of(cm.cpre, cm.nseg, (uint64_t)gc);
    const Seg& g = cm.seg[s];
    const uint64_t i = gc - cm.cpre[s];
    const uint64_t w = q - (cscan[gc] & WMASK);
    const uint64_t qs = q - g.npbase;  // word within the segment's new records
    const uint32_t o = ld32(cur + g.cmsg + 32 + 4 * i);
    const uint64_t v = ld64(cur + g.cbody + 8 * ((uint64_t)o + w));
    const uint64_t nsz = round8(4 * g.n_new);
    *reinterpret_cast<uint64_t*>(enc + g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + nsz + 8 * qs) = v;
    const uint64_t n = g.n_match + g.n_new;
    *reinterpret_cast<uint64_t*>(newref + g.oref + 32 + 8 * ((n + 1) / 2) + 8 * (g.W + qs)) = v;
  }
}

// =============================================================================
// Decoder
// =============================================================================
__global__ __launch_bounds__(1024) void k_dec_setup(Common cm, const uint8_t* enc, int64_t enc_len,
                                                    const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                                                    const int64_t* ref_off, bool have_pred, int64_t out_cap,
                                                    int64_t* out_off, uint8_t* out, ClearFirst cf) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry[5];
  BlockScan1024 bs{s_w};
  do_clear_first(cf);
  if (threadIdx.x < 5) s_carry[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < cm.nseg; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    uint64_t nr = 0, G = 0, nn = 0, osz = 0, PG = 0;
    if (s < cm.nseg) {
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
        if (magic != TAD1_MAGIC || ver != 1 || packer != 1 || mode > 1 || (h[2] >> 32) != 0) code = ERR_CORRUPT;
        else if (mode == 1 && !have_pred) code = ERR_INVALID;
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
          }
        }
      }
      if (code) {
        fail(cm.status, code);
        nr = G = nn = osz = PG = 0;
      }
    }
    uint64_t t0, t1, t2, t3, t4;
    const uint64_t e0 = bs.excl(nr, &t0), e1 = bs.excl(G, &t1), e2 = bs.excl(nn, &t2), e3 = bs.excl(osz, &t3),
                   e4 = bs.excl(PG, &t4);
    if (s < cm.nseg) {
      cm.rpre[s] = s_carry[0] + e0;
      cm.gpre[s] = s_carry[1] + e1;
      cm.npre[s] = s_carry[2] + e2;
      cm.seg[s].oref = s_carry[3] + e3;
      out_off[s] = (int64_t)(s_carry[3] + e3);
      cm.ppre[s] = s_carry[4] + e4;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry[0] += t0;
      s_carry[1] += t1;
      s_carry[2] += t2;
      s_carry[3] += t3;
      s_carry[4] += t4;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cm.rpre[cm.nseg] = s_carry[0];
    cm.gpre[cm.nseg] = s_carry[1];
    cm.npre[cm.nseg] = s_carry[2];
    cm.ppre[cm.nseg] = s_carry[4];
    out_off[cm.nseg] = (int64_t)s_carry[3];
    cm.meta[1] = s_carry[0];
    cm.meta[3] = s_carry[1];
    cm.meta[6] = s_carry[2];
    cm.meta[4] = s_carry[4];
    if (s_carry[3] > (uint64_t)out_cap) fail(cm.status, ERR_CAPACITY);
  }
}

__global__ __launch_bounds__(BLOCK) void k_dec_rslots(Common cm, const uint8_t* enc, const uint8_t* ref,
                                                      uint32_t* rwords, uint8_t* rmatch) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  const int64_t start = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t rounds = (Rt + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t g = start + it * stride;
    const bool active = g < Rt;
    int64_t s = 0;
    uint64_t uid = 0;
    bool ok = false;
    if (active) {
      s = seg_of(cm.rpre, cm.nseg, (uint64_t)g);
      const Seg& sg = cm.seg[s];
      const uint64_t j = g - cm.rpre[s];
      uint32_t o;
      uint64_t hdr;
      const uint8_t* m = ref + sg.rmsg;
      if (tam1_record(m, (uint32_t)sg.nr, sg.rwr, (uint32_t)j, &o, &hdr)) {
        uid = ld64(tam1_records(m, (uint32_t)sg.nr) + 8 * (uint64_t)o);
        ok = uid != 0;
      }
      if (!ok) fail(cm.status, ERR_INVALID);
      const uint64_t pw = ld64(enc + sg.encm + 64 + 8 * (j / 64));
      rmatch[g] = (uint8_t)((pw >> (j & 63)) & 1);
      rwords[g] = (uint32_t)(hdr >> 32);
    }
    // XOR of the reference uids, compared with the encoding's later
    seg_xor(&cm.seg[0].rfold, sizeof(Seg) / 8, s, active && ok, uid);
  }
}

struct DMatchIn {
  const uint8_t* rmatch;
  const uint32_t* rwords;
  __device__ uint64_t operator()(int64_t g) const { return rmatch[g] ? ((1ull << PK) | rwords[g]) : 0; }
};
struct DNewIn {  // words of new records, from the encodings' size tables
  Common cm;
  const uint8_t* enc;
  __device__ uint64_t operator()(int64_t r) const {
    const int64_t s = seg_of(cm.npre, cm.nseg, (uint64_t)r);
    const Seg& g = cm.seg[s];
    const uint64_t k = r - cm.npre[s];
    const uint32_t sz = ld32(enc + g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + 4 * k);
    if (sz < 2) {
      fail(cm.status, ERR_CORRUPT);
      return 2;
    }
    return sz;
  }
};
struct DGroupIn {  // group block bytes
  Common cm;
  const uint8_t* enc;
  __device__ uint64_t operator()(int64_t gg) const {
    const int64_t s = seg_of(cm.gpre, cm.nseg, (uint64_t)gg);
    const Seg& g = cm.seg[s];
    return 8 * (uint64_t)enc[g.encm + 64 + 8 * g.PG + 8 * g.G + (gg - cm.gpre[s])];
  }
};


__global__ __launch_bounds__(1024) void k_dec_seg2(Common cm, const uint64_t* rscan, const uint64_t* nscan,
                                                   const uint64_t* gex, uint8_t* out) {
  if (status_of(cm.status) & ANY_ERR) return;
  for (int64_t s = threadIdx.x; s < cm.nseg; s += 1024) {
    Seg& g = cm.seg[s];
    const uint64_t rs = rscan[cm.rpre[s]], re = rscan[cm.rpre[s + 1]];
    g.mbase = rs >> PK;
    g.dbase = rs & WMASK;
    const uint64_t nm = (re >> PK) - g.mbase, W = (re & WMASK) - g.dbase;
    g.npbase = nscan[cm.npre[s]];
    const uint64_t nw = nscan[cm.npre[s + 1]] - g.npbase;
    const uint64_t var = gex[cm.gpre[s + 1]] - gex[cm.gpre[s]];
    if (g.rfold != g.fold) fail(cm.status, ERR_REF);
    if (nm != g.n_match || W != g.W || nw != g.new_words || var != g.var) fail(cm.status, ERR_CORRUPT);
  }
  if (threadIdx.x == 0) cm.meta[7] = (int64_t)nscan[cm.meta[6]];
  __syncthreads();
  if (status_of(cm.status) & ANY_ERR) return;
  for (int64_t s = threadIdx.x; s < cm.nseg; s += 1024) {
    const Seg& g = cm.seg[s];
    uint8_t* o = out + g.oref;
    const uint64_t n = g.n_match + g.n_new;
    uint64_t* h = reinterpret_cast<uint64_t*>(o);
    h[0] = (uint64_t)TAM1_MAGIC | (1ull << 32);
    h[1] = n;
    h[2] = g.W + g.new_words;
    h[3] = 0;
    if (n & 1) *reinterpret_cast<uint32_t*>(o + 32 + 4 * n) = 0;
  }
}

__global__ __launch_bounds__(BLOCK) void k_dec_mdir(Common cm, const uint8_t* ref, const uint8_t* rmatch,
                                                    const uint64_t* rscan, MDir* mdir, uint8_t* out) {
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Rt = cm.meta[1];
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < Rt; g += (int64_t)gridDim.x * BLOCK) {
    if (!rmatch[g]) continue;
    const int64_t s = seg_of(cm.rpre, cm.nseg, (uint64_t)g);
    const Seg& sg = cm.seg[s];
    const uint64_t j = g - cm.rpre[s];
    const uint64_t k = rscan[g] >> PK;
    const uint64_t d = rscan[g] & WMASK;
    MDir e;
    e.cword = 0;
    e.rword = sg.rbody / 8 + ld32(ref + sg.rmsg + 32 + 4 * j);
    e.dstart = d;
    e.g = (uint64_t)g;
    mdir[k] = e;
    *reinterpret_cast<uint32_t*>(out + sg.oref + 32 + 4 * (k - sg.mbase)) = (uint32_t)(d - sg.dbase);
  }
}

struct UnpackArgs {
  Common cm;
  const uint8_t* enc;
  const uint64_t* ref;
  const MDir* mdir;
  const uint64_t* gex;
  uint64_t* out;
  const uint64_t* pred_x;
  const uint8_t* pred_on;
};

// One wave per 64-word group: read the block, rebuild the residual words, xor
// with X and write C'.  Every length, size and padding byte is checked.
__global__ __launch_bounds__(BLOCK) void k_dec_unpack(UnpackArgs a) {
  __shared__ uint64_t s_blk[WAVES][BLK_MAX / 8];
  const Common& cm = a.cm;
  if (status_of(cm.status) & ANY_ERR) return;
  const int64_t Gt = cm.meta[3];
  const int l = lane_id(), wv = wave_id();
  uint8_t* blk = reinterpret_cast<uint8_t*>(s_blk[wv]);
  const int64_t nwaves = (int64_t)gridDim.x * WAVES;
  for (int64_t gg = (int64_t)blockIdx.x * WAVES + wv; gg < Gt; gg += nwaves) {
    const int64_t s = seg_of(cm.gpre, cm.nseg, (uint64_t)gg);
    const Seg& sg = cm.seg[s];
    const uint64_t lg = (uint64_t)gg - cm.gpre[s];
    const uint8_t* e = a.enc + sg.encm;
    const uint64_t bitmap = ld64(e + 64 + 8 * sg.PG + 8 * lg);
    const uint32_t size = 8u * e[64 + 8 * sg.PG + 8 * sg.G + lg];
    bool bad = size > BLK_MAX;
    if (!bad) {
      const uint64_t boff = sg.fixed + (a.gex[gg] - a.gex[cm.gpre[s]]);
      for (uint32_t w = l; w < size / 8; w += WAVE) s_blk[wv][w] = ld64(e + boff + 8 * w);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const bool bit = (bitmap >> l) & 1;
    const uint32_t popc = (uint32_t)__popcll(bitmap);
    const uint32_t nib = (popc + 1) / 2;
    const uint32_t t = (uint32_t)__popcll(bitmap & lanemask_lt(l));
    uint32_t len = 0;
    if (bit && !bad) len = (blk[t / 2] >> (4 * (t & 1))) & 15u;
    bool lbad = bit && (len < 1 || len > 8);
    const uint64_t sig_incl = wave_incl_scan(len);
    const uint64_t end = nib + uniform64(__shfl(sig_incl, 63, WAVE));
    if (end > size || round8(end) != size) bad = true;
    uint64_t D = 0;
    if (bit && !bad && !lbad) {
      const uint32_t so = nib + (uint32_t)(sig_incl - len);
      for (uint32_t b = 0; b < len; ++b) D |= (uint64_t)blk[so + b] << (8 * b);
      if ((D >> (8 * (len - 1))) == 0) lbad = true;
    }
    if (!bad) {
      if (end + (uint64_t)l < size && blk[end + l] != 0) lbad = true;   // padding bytes
      if (l == 0 && (popc & 1) && (blk[popc / 2] >> 4) != 0) lbad = true;  // unused high nibble
    }
    const uint64_t q = 64 * lg + (uint64_t)l;
    const uint64_t dq0 = sg.dbase + 64 * lg;
    const uint64_t k = window_record(a.mdir, sg.mbase, sg.mbase + sg.n_match, dq0);
    if (q < sg.W && !bad) {
      const MDir r = a.mdir[k];
      const uint64_t w = dq0 + (uint64_t)l - r.dstart;
      uint64_t x = a.ref[r.rword + w];
      if (sg.mode == 1 && w >= 2 && w < 6 && a.pred_on[k]) x = a.pred_x[4 * k + (w - 2)];
      if (w < 2 && D != 0) lbad = true;  // a matched record keeps its uid and header
      const uint64_t n = sg.n_match + sg.n_new;
      a.out[(sg.oref + 32 + 8 * ((n + 1) / 2)) / 8 + q] = D ^ x;
    }
    if (__ballot(lbad) || bad) {
      if (l == 0) fail(cm.status, ERR_CORRUPT);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// New records, word by word, from the encoding into C'; their offsets.
__global__ __launch_bounds__(BLOCK) void k_dec_newcopy(Common cm, const uint64_t* nscan, const uint8_t* enc,
                                                       uint8_t* out) {
  if (status_of(cm.status) & ANY_ERR) return;
  const uint64_t NW = (uint64_t)cm.meta[7];
  const int64_t Nn = cm.meta[6];
  for (uint64_t q = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; q < NW; q += (uint64_t)gridDim.x * BLOCK) {
    const int64_t r = last_le<uint64_t>(nscan, 0, Nn, q);
    const int64_t s = seg_of(cm.npre, cm.nseg, (uint64_t)r);
    const Seg& g = cm.seg[s];
    const uint64_t k = r - cm.npre[s];
    const uint64_t w = q - nscan[r];
    const uint64_t qs = q - g.npbase;
    const uint64_t size = nscan[r + 1] - nscan[r];
    const uint8_t* src = enc + g.encm + 64 + 8 * g.PG + 8 * g.G + round8(g.G) + round8(4 * g.n_new);
    const uint64_t v = ld64(src + 8 * qs);
    if ((w == 0 && v == 0) || (w == 1 && (v >> 32) != size)) fail(cm.status, ERR_CORRUPT);
    const uint64_t n = g.n_match + g.n_new;
    *reinterpret_cast<uint64_t*>(out + g.oref + 32 + 8 * ((n + 1) / 2) + 8 * (g.W + qs)) = v;
    if (w == 0) *reinterpret_cast<uint32_t*>(out + g.oref + 32 + 4 * (g.n_match + k)) = (uint32_t)(g.W + nscan[r] - g.npbase);
  }
}

// ---------------------------------------------------------------------------
struct Mem {
  Common cm;
  Entry* tab;
  uint32_t* cwords;
  uint32_t* rwords;
  uint32_t* rslot;
  int32_t* m;
  uint8_t* cflag;   // encoder: matched C records; decoder: matched R slots
  uint64_t* rscan;
  uint64_t* cscan;  // encoder: new C records; decoder: new record words
  MDir* mdir;
  uint64_t* bm;
  uint8_t* gsz;
  uint64_t* gex;
  uint64_t* pred_x;
  uint8_t* pred_on;
};

struct Bounds {
  int64_t C, R, H, G;
};

Mem carve(Arena& ar, int64_t nseg, const Bounds& b) {
  Mem m;
  m.cm.nseg = nseg;
  m.cm.seg = ar.take<Seg>(nseg + 1);
  m.cm.cpre = ar.take<uint64_t>(nseg + 1);
  m.cm.rpre = ar.take<uint64_t>(nseg + 1);
  m.cm.gpre = ar.take<uint64_t>(nseg + 1);
  m.cm.ppre = ar.take<uint64_t>(nseg + 1);
  m.cm.npre = ar.take<uint64_t>(nseg + 1);
  m.cm.meta = ar.take<int64_t>(16);
  m.cm.status = nullptr;
  m.tab = ar.take<Entry>(b.H);
  m.cwords = ar.take<uint32_t>(b.C);
  m.rwords = ar.take<uint32_t>(b.R);
  m.rslot = ar.take<uint32_t>(b.R);
  m.m = ar.take<int32_t>(b.R);
  m.cflag = ar.take<uint8_t>(std::max(b.C, b.R));
  m.rscan = ar.take<uint64_t>(b.R + 1);
  m.cscan = ar.take<uint64_t>(std::max(b.C, b.R) + 1);
  m.mdir = ar.take<MDir>(b.R);
  m.bm = ar.take<uint64_t>(b.G);
  m.gsz = ar.take<uint8_t>(b.G);
  m.gex = ar.take<uint64_t>(b.G + 1);
  m.pred_x = ar.take<uint64_t>(4 * b.R);
  m.pred_on = ar.take<uint8_t>(b.R);
  return m;
}

Bounds enc_bounds(int64_t nseg, int64_t cur_len, int64_t ref_len) {
  Bounds b;
  b.C = cur_len / 20 + 1;
  b.R = ref_len / 20 + 1;
  b.H = 4 * (b.C + b.R) + 2 * nseg + 1;
  b.G = ref_len / 512 + nseg + 1;
  return b;
}
Bounds dec_bounds(int64_t nseg, int64_t enc_len, int64_t ref_len) {
  Bounds b;
  b.C = enc_len / 20 + 1;  // new records
  b.R = ref_len / 20 + 1;
  b.H = 1;
  b.G = ref_len / 512 + nseg + 1;
  return b;
}

}  // namespace

namespace ta {
size_t encode_scratch(int64_t nseg, int64_t cur_len, int64_t ref_len, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  const Bounds b = enc_bounds(nseg, cur_len, ref_len);
  carve(ar, nseg, b);
  *tiles = ceil_div(std::max(b.C, b.R) + 1, SCAN_TILE) + ceil_div(b.G, TILE_G) + 2;
  return ar.used + 256;
}
size_t decode_scratch(int64_t nseg, int64_t enc_len, int64_t ref_len, int64_t out_cap, int64_t* tiles) {
  (void)out_cap;
  Arena ar{nullptr, 0, 0};
  const Bounds b = dec_bounds(nseg, enc_len, ref_len);
  carve(ar, nseg, b);
  *tiles = ceil_div(std::max(std::max(b.C, b.R), b.G) + 1, SCAN_TILE) + 2;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_delta_encode(ta_ctx* c, int64_t nseg, const uint8_t* cur, int64_t cur_len,
                                     const int64_t* cur_off, const uint8_t* ref, int64_t ref_len,
                                     const int64_t* ref_off, const ta_predictor* pred, const ta_history* hist_in,
                                     ta_history* hist_out, uint8_t* enc, int64_t enc_cap, int64_t* enc_off,
                                     uint8_t* newref, int64_t newref_cap, int64_t* newref_off, uint8_t* modes,
                                     void* stream) {
  if (!c || nseg < 0 || !cur_off || !ref_off || !enc_off || !newref_off || cur_len < 0 || ref_len < 0 ||
      enc_cap < 0 || newref_cap < 0 || (cur_len && !cur) || (ref_len && !ref) || (enc_cap && !enc) ||
      (newref_cap && !newref) || (pred && !hist_in))
    return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (nseg == 0) {
    TA_HIP(hipMemsetAsync(enc_off, 0, 8, s));
    TA_HIP(hipMemsetAsync(newref_off, 0, 8, s));
    return TA_OK;
  }
  if (cur_len / 20 + 1 >= (1ll << 28) || cur_len / 8 >= (1ll << 34) || ref_len / 20 + 1 >= (1ll << 28) ||
      ref_len / 8 >= (1ll << 34))
    return TA_ERR_INVALID;  // packed scan fields: < 2^28 records, < 2^34 words
  int64_t tiles;
  ta_status st = ensure_scratch(c, encode_scratch(nseg, cur_len, ref_len, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const Bounds b = enc_bounds(nseg, cur_len, ref_len);
  Mem m = carve(ar, nseg, b);
  m.cm.status = c->d_status;
  const int g = c->grid;
  k_enc_setup<<<1, 1024, 0, s>>>(m.cm, cur, cur_len, cur_off, ref, ref_len, ref_off, clear_first(c));
  k_clear_tab<<<g, BLOCK, 0, s>>>(m.cm, m.tab, m.cflag);
  k_enc_insert<<<g, BLOCK, 0, s>>>(m.cm, cur, ref, m.tab, m.cwords, m.rwords, m.rslot);
  k_enc_match<<<g, BLOCK, 0, s>>>(m.cm, cur, ref, m.tab, m.rslot, m.m, m.cflag);
  k_scan<RMatchIn><<<grid_for(c, b.R + 1, SCAN_TILE), BLOCK, 0, s>>>(RMatchIn{m.m, m.rwords}, m.cm.meta + 1, m.rscan,
                                                                     lookback(c, 0));
  k_scan<CNewIn><<<grid_for(c, b.C + 1, SCAN_TILE), BLOCK, 0, s>>>(CNewIn{m.cflag, m.cwords}, m.cm.meta + 0, m.cscan,
                                                                   lookback(c, 1));
  k_enc_seg2<<<1, 1024, 0, s>>>(m.cm, m.rscan, m.cscan, newref, newref_cap, newref_off, m.gex);
  k_enc_mdir<<<g, BLOCK, 0, s>>>(m.cm, cur, ref, m.m, m.rscan, m.mdir, newref);
  {
    Timed tm(c, "encode_xor", s);
    XorArgs xa{m.cm,  reinterpret_cast<const uint64_t*>(cur), reinterpret_cast<const uint64_t*>(ref), m.mdir, enc,
               enc_cap, reinterpret_cast<uint64_t*>(newref), m.bm, m.gsz, m.gex, nullptr, m.pred_x, m.pred_on,
               lookback(c, 2)};
    k_enc_xor<<<grid_for(c, b.G, TILE_G), BLOCK, 0, s>>>(xa);
  }
  k_enc_fin<<<1, 1024, 0, s>>>(m.cm, m.gex, enc, enc_cap, enc_off, modes);
  k_enc_fixed<<<g, BLOCK, 0, s>>>(m.cm, m.m, m.cflag, m.cwords, m.cscan, m.bm, m.gsz, enc, enc_cap, newref);
  k_enc_newcopy<<<g, BLOCK, 0, s>>>(m.cm, m.cscan, m.cflag, cur, enc, newref);
  (void)hist_out;
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_delta_decode(ta_ctx* c, int64_t nseg, const uint8_t* enc, int64_t enc_len,
                                     const int64_t* enc_off, const uint8_t* ref, int64_t ref_len,
                                     const int64_t* ref_off, const ta_predictor* pred, const ta_history* hist_in,
                                     ta_history* hist_out, uint8_t* out, int64_t out_cap, int64_t* out_off,
                                     void* stream) {
  if (!c || nseg < 0 || !enc_off || !ref_off || !out_off || enc_len < 0 || ref_len < 0 || out_cap < 0 ||
      (enc_len && !enc) || (ref_len && !ref) || (out_cap && !out) || (pred && !hist_in))
    return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (nseg == 0) {
    TA_HIP(hipMemsetAsync(out_off, 0, 8, s));
    return TA_OK;
  }
  if (enc_len / 8 >= (1ll << 34) || ref_len / 20 + 1 >= (1ll << 28) || ref_len / 8 >= (1ll << 34))
    return TA_ERR_INVALID;
  int64_t tiles;
  ta_status st = ensure_scratch(c, decode_scratch(nseg, enc_len, ref_len, out_cap, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  const Bounds b = dec_bounds(nseg, enc_len, ref_len);
  Mem m = carve(ar, nseg, b);
  m.cm.status = c->d_status;
  const int g = c->grid;
  k_dec_setup<<<1, 1024, 0, s>>>(m.cm, enc, enc_len, enc_off, ref, ref_len, ref_off, pred != nullptr, out_cap,
                                 out_off, out, clear_first(c));
  k_dec_rslots<<<g, BLOCK, 0, s>>>(m.cm, enc, ref, m.rwords, m.cflag);
  k_scan<DMatchIn><<<grid_for(c, b.R + 1, SCAN_TILE), BLOCK, 0, s>>>(DMatchIn{m.cflag, m.rwords}, m.cm.meta + 1,
                                                                     m.rscan, lookback(c, 0));
  k_scan<DNewIn><<<grid_for(c, b.C + 1, SCAN_TILE), BLOCK, 0, s>>>(DNewIn{m.cm, enc}, m.cm.meta + 6, m.cscan,
                                                                   lookback(c, 1));
  k_scan<DGroupIn><<<grid_for(c, b.G + 1, SCAN_TILE), BLOCK, 0, s>>>(DGroupIn{m.cm, enc}, m.cm.meta + 3, m.gex,
                                                                     lookback(c, 2));
  k_dec_seg2<<<1, 1024, 0, s>>>(m.cm, m.rscan, m.cscan, m.gex, out);
  k_dec_mdir<<<g, BLOCK, 0, s>>>(m.cm, ref, m.cflag, m.rscan, m.mdir, out);
  {
    Timed tm(c, "decode_unpack", s);
    UnpackArgs ua{m.cm, enc, reinterpret_cast<const uint64_t*>(ref), m.mdir, m.gex, reinterpret_cast<uint64_t*>(out),
                  m.pred_x, m.pred_on};
    k_dec_unpack<<<grid_for(c, b.G, WAVES), BLOCK, 0, s>>>(ua);
  }
  k_dec_newcopy<<<g, BLOCK, 0, s>>>(m.cm, m.cscan, enc, out);
  (void)hist_out;
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_predictor_load(ta_ctx* c, const void* blob, size_t len, ta_predictor** out) {
  (void)c;
  (void)blob;
  (void)len;
  (void)out;
  return TA_ERR_INVALID;
}
extern "C" void ta_predictor_free(ta_predictor* p) { (void)p; }
