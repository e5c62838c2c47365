// ta_migrate.hip -- the store after one exchange of migrants (Sec. 2.1,
// "Agent Migration"; records as serialized in Sec. 2.2.1).
//
// Agents that left their partition's box are selected by ta_select_migrants
// (the aura kernels with an exact direction match) and serialized by
// ta_serialize.  ta_migrate_apply then builds the new store in one pass over
// the old one: partition q holds the agents of q that stay inside box q, in
// store order, then the records of the messages addressed to q (ascending
// message, record order) unpacked into the columns.
//
// Kernels:
//   k_mig_setup        partition table and message headers checked; records
//                      per message
//   k_scan_cols        record prefix over the messages
//   k_scan<KeepIn>     agents that stay (flag and prefix)
//   k_scan<KeepBehIn>  behaviour bytes of the agents that stay
//   k_scan<RecIn>      every record checked; behaviour bytes of the records
//                      that are taken in
//   k_mig_part         one block per partition: the newcomer slots of each
//                      message addressed to it, the partition's result sizes
//   k_scan_cols        partition starts of the result (agents, behaviour bytes)
//   k_mig_keep         agents that stay: every column and behaviour bytes
//   k_mig_unpack       records unpacked into the columns
#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

struct MigScratch {
  uint8_t* kflag;    // [n] agent stays in its box
  uint64_t* kscan;   // [n+1] agents that stay, before i
  uint64_t* kbscan;  // [n+1] their behaviour bytes, before i
  uint64_t* mrec;    // [nseg+1] records of message s (0 when its header is bad)
  uint64_t* mrw;     // [nseg+1] record words of message s
  uint64_t* mpre;    // [nseg+1] records before message s
  uint64_t* rbscan;  // [rec_cap+1] behaviour bytes taken in, before record r
  uint64_t* mbase;   // [nseg+1] first newcomer slot of message s in its partition
  uint64_t* mbbase;  // [nseg+1] its first behaviour byte among the partition's newcomers
  uint64_t* cols;    // [2][P+1] agents and behaviour bytes of each result partition
  uint64_t* keptn;   // [P+1] agents that stay, per partition
  uint64_t* keptb;   // [P+1] their behaviour bytes
  uint64_t* obpre;   // [P+1] behaviour byte starts of the result's partitions
  int64_t* meta;     // [0] records of all messages, [1] agents in partitions
};

struct StoreOut {
  uint64_t* uid;
  uint16_t* cls;
  uint16_t* nb;
  uint64_t* f64;  // fp64 columns moved as raw 64-bit words
  int64_t fs;
  int32_t* i32;
  int64_t is;
  int64_t* beh_off;
  uint8_t* beh;
};

int64_t rec_bound(int64_t msgs_len) { return msgs_len / 16 + 1; }  // records take >= 16 bytes

MigScratch carve(Arena& ar, int64_t n, int64_t P, int64_t nseg, int64_t msgs_len) {
  MigScratch m;
  m.kflag = ar.take<uint8_t>(n + 8);
  m.kscan = ar.take<uint64_t>(n + 1);
  m.kbscan = ar.take<uint64_t>(n + 1);
  m.mrec = ar.take<uint64_t>(nseg + 1);
  m.mrw = ar.take<uint64_t>(nseg + 1);
  m.mpre = ar.take<uint64_t>(nseg + 1);
  m.rbscan = ar.take<uint64_t>(rec_bound(msgs_len) + 1);
  m.mbase = ar.take<uint64_t>(nseg + 1);
  m.mbbase = ar.take<uint64_t>(nseg + 1);
  m.cols = ar.take<uint64_t>(2 * (P + 1));
  m.keptn = ar.take<uint64_t>(P + 1);
  m.keptb = ar.take<uint64_t>(P + 1);
  m.obpre = ar.take<uint64_t>(P + 1);
  m.meta = ar.take<int64_t>(4);
  return m;
}

__global__ __launch_bounds__(BLOCK) void k_mig_setup(const int64_t* part_off, int32_t P, int64_t n_agents,
                                                     const uint8_t* msgs, int64_t msgs_len, const int64_t* msg_off,
                                                     int64_t nseg, const int32_t* dest, MigScratch sc, ClearFirst cf,
                                                     uint32_t* status) {
  do_clear_first(cf);
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (int64_t)gridDim.x * BLOCK;
  if (tid == 0) {
    const bool ok = part_off[0] == 0 && part_off[P] >= 0 && part_off[P] <= n_agents;
    if (!ok) fail(status, ERR_INVALID);
    sc.meta[1] = ok ? part_off[P] : 0;  // nothing is read past the store when the table is bad
  }
  for (int64_t p = tid; p < P; p += stride)
    if (part_off[p + 1] < part_off[p]) fail(status, ERR_INVALID);
  for (int64_t s = tid; s < nseg; s += stride) {
    const int64_t a = msg_off[s], b = msg_off[s + 1];
    uint32_t n = 0;
    uint64_t rw = 0;
    bool ok = a >= 0 && b >= a && b <= msgs_len && !(a & 7) && dest[s] < P;
    if (ok) ok = tam1_header(msgs + a, b - a, &n, &rw);
    if (!ok) {
      fail(status, ERR_INVALID);
      n = 0;
      rw = 0;
    }
    sc.mrec[s] = n;
    sc.mrw[s] = rw;
  }
}

// Agent i stays when its position is inside its partition's box on every
// axis (lo <= x < hi; a NaN coordinate counts as inside, as it is selected
// for no direction).
struct KeepIn {
  const uint64_t* f64;  // raw words of the fp64 columns
  int64_t stride;
  const uint64_t* part_off;
  int32_t P;
  const double* boxes;
  uint8_t* kflag;
  int64_t lo = 0, hi = 0;
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(part_off, 0, P, (uint64_t)first);
    hi = wave_last_le<uint64_t>(part_off, lo, P, (uint64_t)last);
  }
  __device__ uint64_t operator()(int64_t i) const {
    const int64_t p = last_le<uint64_t>(part_off, lo, hi + 1, (uint64_t)i);
    const double* b = boxes + 6 * p;
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = __builtin_bit_cast(double, f64[a * stride + i]);
      in = in && !(x < b[a]) && !(x >= b[3 + a]);
    }
    return in ? 1u : 0u;
  }
  // All rounds' coordinates are loaded before any test; a wave inside one
  // partition (the common case) reads its box once.
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    int64_t ic[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      ic[r] = i < n ? i : n - 1;
    }
    if (lo == hi) {  // uniform
      const double* b = boxes + 6 * lo;
      double x[R][3];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) x[r][a] = __builtin_bit_cast(double, f64[a * stride + ic[r]]);
      const double b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3], b4 = b[4], b5 = b[5];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool in = !(x[r][0] < b0) && !(x[r][0] >= b3) && !(x[r][1] < b1) && !(x[r][1] >= b4) &&
                        !(x[r][2] < b2) && !(x[r][2] >= b5);
        v[r] = (wbase + r * WAVE + l < n && in) ? 1u : 0u;
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = wbase + r * WAVE + l < n ? (*this)(ic[r]) : 0u;
    }
  }
  __device__ void emit(int64_t i, uint64_t, uint64_t v) const { kflag[i] = (uint8_t)v; }
};

struct KeepBehIn {
  static constexpr int ROUNDS = 16;  // tiles of 8192 agents: half the tickets and look-backs (76 -> 63 us over 1e7)
  const uint8_t* kflag;
  const int64_t* beh_off;
  uint32_t* status;
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    uint8_t f[R];
    int64_t a[R], b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l, ic = i < n ? i : n - 1;
      f[r] = kflag[ic];
      a[r] = beh_off[ic];
      b[r] = beh_off[ic + 1];
    }
    __builtin_amdgcn_sched_barrier(0);
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool keep = wbase + r * WAVE + l < n && f[r];
      const bool ok = !(a[r] & 7) && b[r] >= a[r] && !((b[r] - a[r]) & 7);
      bad = bad || (keep && !ok);
      v[r] = keep && ok ? (uint64_t)(b[r] - a[r]) : 0;
    }
    if (bad) fail(status, ERR_INVALID);
  }
};

// Record r of all messages: checked (offsets, size, non-zero uid, class,
// room for the class's fixed part); value = its behaviour bytes when its
// message is taken in.
struct RecIn {
  const uint8_t* msgs;
  const int64_t* msg_off;
  const uint64_t* mpre;
  const uint64_t* mrec;
  const uint64_t* mrw;
  const int32_t* dest;
  int64_t nseg;
  const uint16_t* nf;
  const uint16_t* ni;
  uint32_t ncls;
  uint32_t* status;
  int64_t lo = 0, hi = 0;
  __device__ void wave_begin(int64_t first, int64_t last) {
    lo = wave_last_le<uint64_t>(mpre, 0, nseg, (uint64_t)first);
    hi = wave_last_le<uint64_t>(mpre, lo, nseg, (uint64_t)last);
  }
  // All rounds in stages: message, then its descriptors, then the offsets,
  // then the record words, then the class.
  template <int R>
  __device__ void values(int64_t wbase, int64_t n, uint64_t* v) const {
    const int l = lane_id();
    int64_t s[R], rc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = wbase + r * WAVE + l;
      rc[r] = i < n ? i : n - 1;
      s[r] = last_le<uint64_t>(mpre, lo, hi + 1, (uint64_t)rc[r]);
    }
    const uint8_t* m[R];
    uint32_t nn[R];
    uint64_t rw[R], p0[R];
    int32_t d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      m[r] = msgs + msg_off[s[r]];
      nn[r] = (uint32_t)mrec[s[r]];
      rw[r] = mrw[s[r]];
      p0[r] = mpre[s[r]];
      d[r] = dest[s[r]];
    }
    __builtin_amdgcn_sched_barrier(0);
    Tam1Loc loc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) loc[r] = tam1_locate(m[r], nn[r], rw[r], (uint32_t)(rc[r] - (int64_t)p0[r]));
    __builtin_amdgcn_sched_barrier(0);
    uint64_t uid[R], hdr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tam1_words(m[r], nn[r], loc[r], &uid[r], &hdr[r]);
    __builtin_amdgcn_sched_barrier(0);
    uint32_t c[R];
    uint64_t fx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      c[r] = (uint32_t)(hdr[r] & 0xFFFF);
      const uint32_t cc = c[r] < ncls ? c[r] : 0;
      fx[r] = 2 + (uint64_t)nf[cc] + ((uint64_t)ni[cc] + 1) / 2;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t words = hdr[r] >> 32;
      const bool ok = tam1_valid(loc[r], hdr[r]) && uid[r] != 0 && c[r] < ncls && words >= fx[r];
      const bool live = wbase + r * WAVE + l < n;
      bad = bad || (live && !ok);
      v[r] = live && ok && d[r] >= 0 ? 8 * (words - fx[r]) : 0;
    }
    if (bad) fail(status, ERR_INVALID);
  }
};

// One block per result partition q: over all messages, a block scan of the
// records (and behaviour bytes) of those addressed to q gives each one its
// first newcomer slot; the partition's sizes go to the column scan.
__global__ __launch_bounds__(1024) void k_mig_part(const int64_t* part_off, int32_t P, const int32_t* dest,
                                                   int64_t nseg, MigScratch sc, uint32_t* status) {
  __shared__ uint64_t s_a[16], s_b[16];
  if (status_of(status) & ANY_ERR) return;
  const int t = threadIdx.x, wv = t / WAVE;
  for (int64_t q = blockIdx.x; q < P; q += gridDim.x) {
    uint64_t carry_a = 0, carry_b = 0;
    for (int64_t s0 = 0; s0 < nseg; s0 += 1024) {
      const int64_t s = s0 + t;
      const bool mine = s < nseg && dest[s] == q;
      const uint64_t a = mine ? sc.mrec[s] : 0;
      const uint64_t b = mine ? sc.rbscan[sc.mpre[s + 1]] - sc.rbscan[sc.mpre[s]] : 0;
      const uint64_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
      if (lane_id() == WAVE - 1) {
        s_a[wv] = ia;
        s_b[wv] = ib;
      }
      __syncthreads();
      uint64_t pa = 0, pb = 0, ta = 0, tb = 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        pa += i < wv ? s_a[i] : 0;
        pb += i < wv ? s_b[i] : 0;
        ta += s_a[i];
        tb += s_b[i];
      }
      if (mine) {
        sc.mbase[s] = carry_a + pa + ia - a;
        sc.mbbase[s] = carry_b + pb + ib - b;
      }
      carry_a += ta;
      carry_b += tb;
      __syncthreads();
    }
    if (t == 0) {
      const uint64_t kn = sc.kscan[part_off[q + 1]] - sc.kscan[part_off[q]];
      const uint64_t kb = sc.kbscan[part_off[q + 1]] - sc.kbscan[part_off[q]];
      sc.keptn[q] = kn;
      sc.keptb[q] = kb;
      sc.cols[q] = kn + carry_a;
      sc.cols[P + 1 + q] = kb + carry_b;
    }
  }
}

// Agents that stay: MK_U rounds of 64 consecutive agents per wave (their
// partitions found once per wave).  Every agent's flag, prefixes and
// behaviour range are loaded first, then each column is moved MK_U agents at
// a time (loads of all rounds before their stores, indices clamped so no
// load sits behind a branch), fp64 columns as raw words; behaviour bytes last.
constexpr int MK_U = 4;
__global__ __launch_bounds__(BLOCK) void k_mig_keep(ta_agents in, const uint64_t* part_off, int32_t P, int nfc,
                                                    int nic, MigScratch sc, const uint64_t* opre, StoreOut out,
                                                    uint32_t* status) {
  if (status_of(status) & ANY_ERR) return;
  const int64_t n = sc.meta[1];
  const uint64_t* f64 = reinterpret_cast<const uint64_t*>(in.f64);
  const int l = lane_id();
  constexpr int64_t SPAN = (int64_t)WAVE * MK_U;
  for (int64_t b0 = ((int64_t)blockIdx.x * WAVES + wave_id()) * SPAN; b0 < n; b0 += (int64_t)gridDim.x * WAVES * SPAN) {
    const int64_t last = b0 + SPAN - 1 < n ? b0 + SPAN - 1 : n - 1;
    const int64_t lo = wave_last_le<uint64_t>(part_off, 0, P, (uint64_t)b0);
    const int64_t hi = wave_last_le<uint64_t>(part_off, lo, P, (uint64_t)last);
    int64_t ic[MK_U];
    uint64_t j[MK_U], bb[MK_U];
    int64_t ba[MK_U], be[MK_U];
    bool keep[MK_U];
#pragma unroll
    for (int u = 0; u < MK_U; ++u) {
      const int64_t i = b0 + (int64_t)u * WAVE + l;
      ic[u] = i < n ? i : n - 1;
      const int64_t q = last_le<uint64_t>(part_off, lo, hi + 1, (uint64_t)ic[u]);
      keep[u] = i < n && sc.kflag[ic[u]];
      j[u] = opre[q] + sc.kscan[ic[u]] - sc.kscan[part_off[q]];
      bb[u] = sc.obpre[q] + sc.kbscan[ic[u]] - sc.kbscan[part_off[q]];
      ba[u] = in.beh_off[ic[u]];
      be[u] = in.beh_off[ic[u] + 1];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      uint64_t uid[MK_U];
      uint16_t cl[MK_U], nb[MK_U];
#pragma unroll
      for (int u = 0; u < MK_U; ++u) {
        uid[u] = in.uid[ic[u]];
        cl[u] = in.cls[ic[u]];
        nb[u] = in.nb[ic[u]];
      }
#pragma unroll
      for (int u = 0; u < MK_U; ++u)
        if (keep[u]) {
          out.uid[j[u]] = uid[u];
          out.cls[j[u]] = cl[u];
          out.nb[j[u]] = nb[u];
          out.beh_off[j[u]] = (int64_t)bb[u];
        }
    }
    for (int k = 0; k < nfc; ++k) {
      uint64_t v[MK_U];
#pragma unroll
      for (int u = 0; u < MK_U; ++u) v[u] = f64[k * in.f64_stride + ic[u]];
#pragma unroll
      for (int u = 0; u < MK_U; ++u)
        if (keep[u]) out.f64[k * out.fs + j[u]] = v[u];
    }
    for (int k = 0; k < nic; ++k) {
      int32_t v[MK_U];
#pragma unroll
      for (int u = 0; u < MK_U; ++u) v[u] = in.i32[k * in.i32_stride + ic[u]];
#pragma unroll
      for (int u = 0; u < MK_U; ++u)
        if (keep[u]) out.i32[k * out.is + j[u]] = v[u];
    }
    // Behaviour bytes.  When every agent of the wave's span stays and the span
    // lies in one partition, its bytes are one range on both sides: the wave
    // copies it lane-parallel, MK_U words per lane in flight.  Otherwise each
    // lane copies its own agents' words.
    bool span_kept = true;
#pragma unroll
    for (int u = 0; u < MK_U; ++u) span_kept = span_kept && (b0 + (int64_t)u * WAVE + l > last || keep[u]);
    if (lo == hi && __ballot(!span_kept) == 0) {
      const int64_t lu = (last - b0) / WAVE, ll = (last - b0) % WAVE;  // round and lane of the span's last agent
      const uint64_t s0 = readlane64((uint64_t)ba[0], 0), d0 = readlane64(bb[0], 0);
      uint64_t s1 = s0;
#pragma unroll
      for (int u = 0; u < MK_U; ++u)
        if (u == lu) s1 = readlane64((uint64_t)be[u], (int)ll);
      const int64_t nw = (int64_t)(s1 - s0) / 8;
      const uint64_t* src = reinterpret_cast<const uint64_t*>(in.beh + s0);
      uint64_t* dst = reinterpret_cast<uint64_t*>(out.beh + d0);
      for (int64_t w0 = l; w0 < nw; w0 += (int64_t)MK_U * WAVE) {
        uint64_t v[MK_U];
#pragma unroll
        for (int u = 0; u < MK_U; ++u) {
          const int64_t w = w0 + (int64_t)u * WAVE;
          v[u] = src[w < nw ? w : nw - 1];
        }
#pragma unroll
        for (int u = 0; u < MK_U; ++u) {
          const int64_t w = w0 + (int64_t)u * WAVE;
          if (w < nw) dst[w] = v[u];
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < MK_U; ++u) {
        if (!keep[u]) continue;
        const int64_t nw = (be[u] - ba[u]) / 8;
        const uint64_t* src = reinterpret_cast<const uint64_t*>(in.beh + ba[u]);
        uint64_t* dst = reinterpret_cast<uint64_t*>(out.beh + bb[u]);
        for (int64_t w = 0; w < nw; ++w) dst[w] = src[w];
      }
    }
  }
}

// Records taken in: uid, class, behaviour count, the class's fields and
// attributes (zeros in the other columns), the rest of the record as
// behaviour bytes.
__global__ __launch_bounds__(BLOCK) void k_mig_unpack(const uint8_t* msgs, const int64_t* msg_off, const int32_t* dest,
                                                      int64_t nseg, int32_t P, const uint16_t* nf, const uint16_t* ni,
                                                      int nfc, int nic, MigScratch sc, const uint64_t* opre,
                                                      StoreOut out, uint32_t* status) {
  if (status_of(status) & ANY_ERR) return;
  const int64_t Rt = sc.meta[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) out.beh_off[opre[P]] = (int64_t)sc.obpre[P];
  const int l = lane_id();
  for (int64_t r0 = ((int64_t)blockIdx.x * WAVES + wave_id()) * WAVE; r0 < Rt; r0 += (int64_t)gridDim.x * BLOCK) {
    const int64_t r = r0 + l, last = r0 + WAVE - 1 < Rt ? r0 + WAVE - 1 : Rt - 1;
    const int64_t s = wave_seg(sc.mpre, nseg, (uint64_t)(r < Rt ? r : Rt - 1), (uint64_t)r0, (uint64_t)last);
    if (r >= Rt) continue;
    const int32_t q = dest[s];
    if (q < 0) continue;
    const uint8_t* m = msgs + msg_off[s];
    const uint32_t n = (uint32_t)sc.mrec[s];
    const uint64_t i = (uint64_t)r - sc.mpre[s];
    uint32_t o;
    uint64_t uid, hdr;
    tam1_record(m, n, sc.mrw[s], (uint32_t)i, &o, &uid, &hdr);  // checked by the record scan
    const uint64_t* rec = reinterpret_cast<const uint64_t*>(tam1_records(m, n)) + o;
    const uint32_t c = (uint32_t)(hdr & 0xFFFF);
    const int fc = nf[c], ic = ni[c];
    const uint64_t fixed = 2 + (uint64_t)fc + (uint64_t)(ic + 1) / 2, words = hdr >> 32;
    const uint64_t j = opre[q] + sc.keptn[q] + sc.mbase[s] + i;
    const uint64_t bb = sc.obpre[q] + sc.keptb[q] + sc.mbbase[s] + (sc.rbscan[r] - sc.rbscan[sc.mpre[s]]);
    out.uid[j] = uid;
    out.cls[j] = (uint16_t)c;
    out.nb[j] = (uint16_t)(hdr >> 16);
    for (int k = 0; k < nfc; ++k) out.f64[k * out.fs + j] = k < fc ? rec[2 + k] : 0;
    const uint32_t* at = reinterpret_cast<const uint32_t*>(rec + 2 + fc);
    for (int k = 0; k < nic; ++k) out.i32[k * out.is + j] = k < ic ? (int32_t)at[k] : 0;
    out.beh_off[j] = (int64_t)bb;
    uint64_t* dst = reinterpret_cast<uint64_t*>(out.beh + bb);
    for (uint64_t w = 0; w < words - fixed; ++w) dst[w] = rec[fixed + w];
  }
}

}  // namespace

namespace ta {
size_t migrate_scratch(int64_t n_agents, int64_t P, int64_t nseg, int64_t msgs_len, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  carve(ar, n_agents, P, nseg, msgs_len);
  *tiles = std::max(ceil_div(n_agents + 1, SCAN_TILE), ceil_div(rec_bound(msgs_len) + 1, SCAN_TILE)) + 1;
  return ar.used + 256;
}
}  // namespace ta

extern "C" ta_status ta_migrate_apply(ta_ctx* c, const ta_agents* in, int32_t P, const int64_t* part_off,
                                      const double* boxes, const uint8_t* msgs, int64_t msgs_len,
                                      const int64_t* msg_off, int64_t nseg, const int32_t* msg_part,
                                      const ta_store* out, int64_t* part_off_out, int64_t* sizes_out,
                                      void* stream) {
  if (!c || !in || !out || P < 1 || !part_off || !boxes || !part_off_out || !sizes_out || nseg < 0 ||
      (nseg > 0 && (!msg_off || !msg_part)) || msgs_len < 0 || (msgs_len > 0 && !msgs) || in->n < 0 ||
      in->f64_stride < in->n || in->i32_stride < in->n ||
      (in->n > 0 && (!in->uid || !in->cls || !in->nb || !in->f64 || !in->beh_off || (c->max_i && !in->i32))) ||
      out->cap < 0 || out->beh_cap < 0 || out->f64_stride < out->cap || out->i32_stride < out->cap ||
      !out->beh_off || (out->cap > 0 && (!out->uid || !out->cls || !out->nb || !out->f64 || (c->max_i && !out->i32))) ||
      (out->beh_cap > 0 && !out->beh))
    return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  int64_t tiles;
  ta_status st = ensure_scratch(c, migrate_scratch(in->n, P, nseg, msgs_len, &tiles), tiles);
  if (st) return st;
  Arena ar{c->scratch, c->scratch_cap, 0};
  MigScratch sc = carve(ar, in->n, P, nseg, msgs_len);
  const int64_t n = in->n, rb = rec_bound(msgs_len);
  const uint64_t* po = reinterpret_cast<const uint64_t*>(part_off);
  k_mig_setup<<<grid_for(c, std::max<int64_t>(P, nseg) + 1, BLOCK), BLOCK, 0, s>>>(
      part_off, P, n, msgs, msgs_len, msg_off, nseg, msg_part, sc, clear_first(c, ceil_div(n + 1, SCAN_TILE)),
      c->d_status);
  if (nseg > 0) {
    ColScan cs{};
    cs.in[0] = sc.mrec;
    cs.out[0] = sc.mpre;
    cs.cap[0] = ~0ull;
    cs.meta_idx[0] = 0;
    cs.meta = sc.meta;
    cs.status = c->d_status;
    cs.n = nseg;
    k_scan_cols<<<1, 1024, 0, s>>>(cs);
  } else {
    st = zero_i64(sc.meta, 1, s);
    if (st) return st;
  }
  k_scan<KeepIn><<<grid_for(c, n + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(
      KeepIn{reinterpret_cast<const uint64_t*>(in->f64), in->f64_stride, po, P, boxes, sc.kflag}, sc.meta + 1, n,
      sc.kscan, lookback(c, 0));
  k_scan<KeepBehIn><<<grid_for(c, n + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(KeepBehIn{sc.kflag, in->beh_off, c->d_status},
                                                                        sc.meta + 1, n, sc.kbscan, lookback(c, 1));
  k_scan<RecIn><<<grid_for(c, rb + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(
      RecIn{msgs, msg_off, sc.mpre, sc.mrec, sc.mrw, msg_part, nseg, c->d_nf, c->d_ni, c->n_classes, c->d_status},
      sc.meta + 0, rb, sc.rbscan, lookback(c, 2));
  k_mig_part<<<grid_for(c, P, 1), 1024, 0, s>>>(part_off, P, msg_part, nseg, sc, c->d_status);
  {
    ColScan cs{};
    cs.in[0] = sc.cols;
    cs.in[1] = sc.cols + P + 1;
    cs.out[0] = reinterpret_cast<uint64_t*>(part_off_out);
    cs.out[1] = sc.obpre;
    cs.cap[0] = (uint64_t)out->cap;
    cs.cap[1] = (uint64_t)out->beh_cap;
    cs.meta_idx[0] = 0;
    cs.meta_idx[1] = 1;
    cs.meta = sizes_out;
    cs.status = c->d_status;
    cs.n = P;
    k_scan_cols<<<2, 1024, 0, s>>>(cs);  // one block per column
  }
  const StoreOut so{out->uid, out->cls, out->nb, reinterpret_cast<uint64_t*>(out->f64), out->f64_stride, out->i32,
                    out->i32_stride, out->beh_off, out->beh};
  const uint64_t* opre = reinterpret_cast<const uint64_t*>(part_off_out);
  {
    Timed tm(c, "migrate_keep", s);
    k_mig_keep<<<grid_for(c, n, BLOCK * MK_U), BLOCK, 0, s>>>(*in, po, P, c->max_f, c->max_i, sc, opre, so,
                                                             c->d_status);
  }
  k_mig_unpack<<<grid_for(c, rb, BLOCK), BLOCK, 0, s>>>(msgs, msg_off, msg_part, nseg, P, c->d_nf, c->d_ni, c->max_f,
                                                       c->max_i, sc, opre, so, c->d_status);
  TA_LAUNCH_CHECK();
  return TA_OK;
}
