// ta_select.hip -- aura selection (Sec. 2.1, "Aura Update").
//
// An agent is copied to the neighbour in direction d when its interaction
// region reaches into that neighbour's box: on every axis where d points down
// its coordinate is below lo+w, on every axis where d points up it is at or
// above hi-w.  Per agent this is a 6-bit code (below lo+w / at or above hi-w
// per axis); direction d needs the bits of its nonzero components.
//
// Kernels (all partitions in one launch each):
//   k_sel_prep    one block: tiles per partition and their prefix
//   k_sel_count   per 2048-agent tile: the 6-bit codes (1 byte/agent), the
//                 number of members per direction and whether it has any
//   k_scan        look-back exclusive scan of the counts, laid out
//                 [partition][direction][tile], which yields every tile's
//                 output position in segment order
//   k_sel_scatter per tile with members: stable compaction of store indices
//                 into the segments, and the segment offsets
#include <mutex>

#include "ta_internal.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace {

#ifndef TA_SEL_IPT
#define TA_SEL_IPT 8
#endif
constexpr int SEL_IPT = TA_SEL_IPT;  // agents per thread and tile
static_assert(BLOCK * SEL_IPT < 4096, "a tile's count per direction must fit a 12-bit field");
constexpr int SEL_TILE = BLOCK * SEL_IPT;

struct DirTable {
  uint8_t req[26];  // code bits direction k requires
};

// Membership of a 6-bit code in a direction: the aura takes every direction
// whose bits the code has (an agent near a corner goes to three faces, three
// edges and the corner); a migrant (EXACT) goes to the one direction whose
// bits are exactly its code.
template <bool EXACT>
__device__ inline bool member(uint32_t code, uint32_t req) {
  if constexpr (EXACT) return code == req;
  else return (code & req) == req;
}

struct SelScratch {
  uint8_t* code;       // [n_agents]
  int64_t* tile_off;   // [P+1]
  uint32_t* cnt;       // [cnt_cap]
  uint64_t* cnt_pre;   // [cnt_cap+1]
  uint8_t* tany;       // [tiles] 1 when some agent of the tile goes to some direction
  int64_t* meta;       // [0] tiles, [1] count entries
};

__global__ __launch_bounds__(1024) void k_sel_prep(const int64_t* part_off, int32_t P, int32_t ndirs, int64_t n_agents,
                                                   SelScratch sc, ClearFirst cf, uint32_t* status) {
  __shared__ uint64_t s_w[16];
  __shared__ int64_t s_carry;
  __shared__ int s_bad;
  do_clear_first(cf);
  if (threadIdx.x == 0) {
    s_carry = 0;
    s_bad = part_off[0] != 0 || part_off[P] > n_agents;
  }
  __syncthreads();
  for (int64_t p0 = 0; p0 < P; p0 += 1024) {
    const int64_t p = p0 + threadIdx.x;
    uint64_t nt = 0;
    if (p < P) {
      const int64_t len = part_off[p + 1] - part_off[p];
      if (len < 0) s_bad = 1;
      else nt = (uint64_t)((len + SEL_TILE - 1) / SEL_TILE);
    }
    const uint64_t incl = wave_incl_scan(nt);
    if (lane_id() == 63) s_w[threadIdx.x / 64] = incl;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      pre += (i < (int)(threadIdx.x / 64)) ? s_w[i] : 0;
      tot += s_w[i];
    }
    if (p < P) sc.tile_off[p] = s_carry + (int64_t)(pre + incl - nt);
    __syncthreads();
    if (threadIdx.x == 0) s_carry += (int64_t)tot;
    __syncthreads();
  }
  __syncthreads();
  if (s_bad) {
    // invalid partition table: no tiles, every segment empty
    for (int64_t p = threadIdx.x; p <= P; p += 1024) sc.tile_off[p] = 0;
    if (threadIdx.x == 0) {
      fail(status, ERR_INVALID);
      sc.meta[0] = 0;
      sc.meta[1] = 0;
    }
    return;
  }
  if (threadIdx.x == 0) {
    sc.tile_off[P] = s_carry;
    sc.meta[0] = s_carry;
    sc.meta[1] = s_carry * ndirs;
  }
}

struct TileInfo {
  int64_t p, lt, nt, a0, a1;
};

__device__ inline TileInfo tile_info(const SelScratch& sc, const int64_t* part_off, int32_t P, int64_t t) {
  TileInfo ti;
  ti.p = last_le<int64_t>(sc.tile_off, 0, P, t);
  ti.lt = t - sc.tile_off[ti.p];
  ti.nt = sc.tile_off[ti.p + 1] - sc.tile_off[ti.p];
  ti.a0 = part_off[ti.p] + ti.lt * SEL_TILE;
  const int64_t e = part_off[ti.p + 1];
  ti.a1 = ti.a0 + SEL_TILE < e ? ti.a0 + SEL_TILE : e;
  return ti;
}

template <int NDIRS, bool EXACT>
__global__ __launch_bounds__(BLOCK) void k_sel_count(const double* f64, int64_t stride, const int64_t* part_off,
                                                     const double* boxes, double w, int32_t P, DirTable dt,
                                                     SelScratch sc) {
  __shared__ uint32_t s_cnt[WAVES][NDIRS];
  const int64_t ntiles = sc.meta[0];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileInfo ti = tile_info(sc, part_off, P, t);
    const double* box = boxes + 6 * ti.p;
    const double tlo0 = box[0] + w, tlo1 = box[1] + w, tlo2 = box[2] + w;
    const double thi0 = box[3] - w, thi1 = box[4] - w, thi2 = box[5] - w;
    uint32_t cnt[NDIRS];
#pragma unroll
    for (int d = 0; d < NDIRS; ++d) cnt[d] = 0;
    // every coordinate of the tile loaded before the first code (agents past
    // the tile read its last agent, unused)
    double x[SEL_IPT], y[SEL_IPT], z[SEL_IPT];
#pragma unroll
    for (int k = 0; k < SEL_IPT; ++k) {
      const int64_t i = ti.a0 + (int64_t)k * BLOCK + threadIdx.x;
      const int64_t ic = i < ti.a1 ? i : ti.a1 - 1;
      x[k] = f64[ic];
      y[k] = f64[stride + ic];
      z[k] = f64[2 * stride + ic];
    }
#pragma unroll
    for (int k = 0; k < SEL_IPT; ++k) {
      const int64_t i = ti.a0 + (int64_t)k * BLOCK + threadIdx.x;
      uint32_t code = 0;
      if (i < ti.a1) {
        code = (uint32_t)(x[k] < tlo0) | ((uint32_t)(x[k] >= thi0) << 1) | ((uint32_t)(y[k] < tlo1) << 2) |
               ((uint32_t)(y[k] >= thi1) << 3) | ((uint32_t)(z[k] < tlo2) << 4) | ((uint32_t)(z[k] >= thi2) << 5);
        sc.code[i] = (uint8_t)code;
      }
      if (__ballot(code != 0) == 0) continue;
#pragma unroll
      for (int d = 0; d < NDIRS; ++d) cnt[d] += (uint32_t)__popcll(__ballot(member<EXACT>(code, dt.req[d])));
    }
    if (lane_id() == 0) {
#pragma unroll
      for (int d = 0; d < NDIRS; ++d) s_cnt[wave_id()][d] = cnt[d];
    }
    __syncthreads();
    if (threadIdx.x < NDIRS) {  // (the first wave's lanes)
      const int d = threadIdx.x;
      uint32_t sum = 0;
#pragma unroll
      for (int wv = 0; wv < WAVES; ++wv) sum += s_cnt[wv][d];
      sc.cnt[sc.tile_off[ti.p] * NDIRS + d * ti.nt + ti.lt] = sum;
      const uint64_t nz = __ballot(sum != 0);
      if (d == 0) sc.tany[t] = nz != 0 ? 1 : 0;
    }
    __syncthreads();
  }
}

struct CntIn {
  const uint32_t* a;
  __device__ uint64_t operator()(int64_t i) const { return a[i]; }
};

// Per-direction thread counts (<= 8) packed 5 to a word in 12-bit fields, so a
// block-wide exclusive scan of NW words gives all directions at once (block
// totals <= 2048 < 4096: no field overflows into the next).  Two tables per
// block, indexed by an agent's 6-bit code, turn counting into lookups: the
// packed increments of the directions the code belongs to, and those
// directions as a bit mask; a wave then scatters only into the directions
// some of its agents belong to.  Held to five waves per SIMD (96 registers
// and an 8-byte spill; at 97 it ran at four, 31.5 instead of 28 us over 1e7
// agents).
template <int NDIRS, bool EXACT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_sel_scatter(const int64_t* part_off, int32_t P, DirTable dt, SelScratch sc,
                                                       int32_t* idx_out, int64_t idx_cap, int64_t* seg_off,
                                                       uint32_t* status) {
  constexpr int NW = (NDIRS + 4) / 5;
  __shared__ uint64_t s_w[WAVES][NW];
  // (256 rows: any byte value indexes inside the tables; codes are 6-bit, rows
  // 64 and up stay empty)
  __shared__ uint64_t s_inc[256][NW];  // per code: +1 in the field of every direction it belongs to
  __shared__ uint32_t s_dm[256];      // per code: its directions, one bit each
  __shared__ uint32_t s_wm[WAVES];    // per wave: directions some of its agents belong to
  __shared__ uint32_t s_req[NDIRS];   // code bits each direction requires
  __shared__ int64_t s_base[NDIRS];   // per direction: the tile's first output position
  const int64_t nseg = (int64_t)P * NDIRS;
  const int64_t gstride = (int64_t)gridDim.x * BLOCK;
  for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s <= nseg; s += gstride) {
    int64_t pos;
    if (s == nseg) {
      pos = (int64_t)sc.cnt_pre[sc.meta[1]];
      if (pos > idx_cap) fail(status, ERR_CAPACITY);
    } else {
      const int64_t p = s / NDIRS, d = s % NDIRS;
      const int64_t nt = sc.tile_off[p + 1] - sc.tile_off[p];
      pos = (int64_t)sc.cnt_pre[sc.tile_off[p] * NDIRS + d * nt];
    }
    seg_off[s] = pos;
  }
  for (int c = threadIdx.x; c < 256; c += BLOCK) {
    uint64_t inc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) inc[j] = 0;
    uint32_t dm = 0;
#pragma unroll
    for (int d = 0; d < NDIRS; ++d) {
      if (c && c < 64 && member<EXACT>(c, dt.req[d])) {
        inc[d / 5] += 1ull << (12 * (d % 5));
        dm |= 1u << d;
      }
    }
#pragma unroll
    for (int j = 0; j < NW; ++j) s_inc[c][j] = inc[j];
    s_dm[c] = dm;
  }
  if (threadIdx.x < NDIRS) s_req[threadIdx.x] = dt.req[threadIdx.x];
  __syncthreads();
  const int l = lane_id(), wv = wave_id();
  const int64_t ntiles = sc.meta[0];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    // (the same in the whole block) a tile none of whose agents is selected
    // writes nothing: it skips its loads, scan and barriers
    if (!uniform32(sc.tany[t])) continue;
    const TileInfo ti = tile_info(sc, part_off, P, t);
    const int64_t cbase = sc.tile_off[ti.p] * NDIRS + ti.lt;
    // every direction's output position loaded at once, ahead of the scan,
    // so that the direction loop below waits on no global load
    if (threadIdx.x < NDIRS) s_base[threadIdx.x] = (int64_t)sc.cnt_pre[cbase + (int64_t)threadIdx.x * ti.nt];
    const int64_t i0 = ti.a0 + (int64_t)threadIdx.x * SEL_IPT;
    uint32_t code[SEL_IPT];
    uint64_t packed[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) packed[j] = 0;
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < SEL_IPT; ++k) {
      code[k] = (i0 + k < ti.a1) ? sc.code[i0 + k] : 0u;
      any |= code[k];
    }
    // most waves (agents away from the box faces) select nothing: they skip
    // the per-direction counts and only join the block scan with zeros
    const bool wave_any = __ballot(any != 0) != 0;
    uint32_t lmask = 0;
    if (wave_any) {
#pragma unroll
      for (int k = 0; k < SEL_IPT; ++k) {
#pragma unroll
        for (int j = 0; j < NW; ++j) packed[j] += s_inc[code[k]][j];
        lmask |= s_dm[code[k]];
      }
    }
    // block exclusive scan of the packed words
    uint64_t incl[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) incl[j] = wave_incl_scan64(packed[j]);
    if (l == WAVE - 1) {
#pragma unroll
      for (int j = 0; j < NW; ++j) s_w[wv][j] = incl[j];
    }
    if (l == 0) s_wm[wv] = 0;
    __syncthreads();
    uint64_t pre[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      uint64_t off = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) off += (w < wv) ? s_w[w][j] : 0;
      pre[j] = off + incl[j] - packed[j];
    }
    if (lmask) atomicOr(&s_wm[wv], lmask);
    __syncthreads();
    const uint32_t wm = uniform32(s_wm[wv]);
    // the wave's directions, one at a time: the packed word of five
    // directions by a static index, its directions present by a uniform loop
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      for (uint32_t mm = (wm >> (5 * j)) & 31u; mm; mm &= mm - 1) {
        const int b = __builtin_ctz(mm), d = 5 * j + b, sh = 12 * b;
        const uint64_t mine = (packed[j] >> sh) & 0xFFF;
        if (!mine) continue;
        const uint32_t req = s_req[d];
        int64_t pos = s_base[d] + (int64_t)((pre[j] >> sh) & 0xFFF);
#pragma unroll
        for (int k = 0; k < SEL_IPT; ++k) {
          if (code[k] && member<EXACT>(code[k], req)) {
            if (pos < idx_cap) idx_out[pos] = (int32_t)(i0 + k);
            ++pos;
          }
        }
      }
    }
    __syncthreads();  // s_w and s_wm are reused by the next tile
  }
}

DirTable make_dirs(int ndirs) {
  DirTable dt{};
  int n = 0;
  for (int c = 0; c < 27; ++c) {
    if (c == 13) continue;
    const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
    const int nz = (d[0] != 0) + (d[1] != 0) + (d[2] != 0);
    if (ndirs == 6 && nz != 1) continue;
    uint8_t req = 0;
    for (int a = 0; a < 3; ++a) {
      if (d[a] == -1) req |= (uint8_t)(1u << (2 * a));
      if (d[a] == +1) req |= (uint8_t)(1u << (2 * a + 1));
    }
    dt.req[n++] = req;
  }
  return dt;
}

struct Sizes {
  int64_t ntiles, cnt_cap;
};
Sizes sel_sizes(int64_t n, int64_t P, int ndirs) {
  Sizes z;
  z.ntiles = ceil_div(n, SEL_TILE) + P;
  z.cnt_cap = z.ntiles * ndirs;
  return z;
}

SelScratch carve(Arena& ar, int64_t n, int64_t P, int ndirs) {
  const Sizes z = sel_sizes(n, P, ndirs);
  SelScratch sc;
  sc.code = ar.take<uint8_t>(n + 8);
  sc.tile_off = ar.take<int64_t>(P + 1);
  sc.cnt = ar.take<uint32_t>(z.cnt_cap);
  sc.cnt_pre = ar.take<uint64_t>(z.cnt_cap + 1);
  sc.tany = ar.take<uint8_t>(z.ntiles);
  sc.meta = ar.take<int64_t>(4);
  return sc;
}

}  // namespace

namespace ta {
size_t select_scratch(int64_t n, int64_t P, int ndirs, int64_t* tiles) {
  Arena ar{nullptr, 0, 0};
  carve(ar, n, P, ndirs);
  *tiles = ceil_div(sel_sizes(n, P, ndirs).cnt_cap + 1, SCAN_TILE) + 1;
  return ar.used + 256;
}
}  // namespace ta

namespace {
// The selection's kernels on scratch carved from `ar`; cf and lb0 clear and
// use the look-back flags of its one scan.
template <bool EXACT>
ta_status select_launch(ta_ctx* c, const ta_agents* ag, int32_t P, const int64_t* part_off, const double* boxes,
                        double w, int32_t ndirs, int32_t* idx_out, int64_t idx_cap, int64_t* seg_off_out,
                        hipStream_t s, Arena ar, const ClearFirst& cf, const LookBack& lb0) {
  SelScratch sc = carve(ar, ag->n, P, ndirs);
  const DirTable dt = make_dirs(ndirs);
  const int64_t cnt_cap = sel_sizes(ag->n, P, ndirs).cnt_cap;
  const int g = grid_for(c, sel_sizes(ag->n, P, ndirs).ntiles, 1);
  k_sel_prep<<<1, 1024, 0, s>>>(part_off, P, ndirs, ag->n, sc, cf, c->d_status);
  {
    Timed tm(c, "select_count", s);
    if (ndirs == 26)
      k_sel_count<26, EXACT><<<g, BLOCK, 0, s>>>(ag->f64, ag->f64_stride, part_off, boxes, w, P, dt, sc);
    else
      k_sel_count<6, EXACT><<<g, BLOCK, 0, s>>>(ag->f64, ag->f64_stride, part_off, boxes, w, P, dt, sc);
  }
  k_scan<CntIn><<<grid_for(c, cnt_cap + 1, SCAN_TILE), SCAN_BLOCK, 0, s>>>(CntIn{sc.cnt}, sc.meta + 1, cnt_cap, sc.cnt_pre,
                                                                      lb0);
  {
    Timed tm(c, "select_scatter", s);
    const int gs = grid_for(c, std::max<int64_t>(sel_sizes(ag->n, P, ndirs).ntiles, ceil_div(P * ndirs + 1, BLOCK)), 1);
    if (ndirs == 26)
      k_sel_scatter<26, EXACT><<<gs, BLOCK, 0, s>>>(part_off, P, dt, sc, idx_out, idx_cap, seg_off_out, c->d_status);
    else
      k_sel_scatter<6, EXACT><<<gs, BLOCK, 0, s>>>(part_off, P, dt, sc, idx_out, idx_cap, seg_off_out, c->d_status);
  }
  TA_LAUNCH_CHECK();
  return TA_OK;
}

template <bool EXACT>
ta_status select_impl(ta_ctx* c, const ta_agents* ag, int32_t P, const int64_t* part_off, const double* boxes,
                      double w, int32_t ndirs, int32_t* idx_out, int64_t idx_cap, int64_t* seg_off_out,
                      void* stream) {
  use_family(c, FAM_SELECT);
  int64_t tiles;
  ta_status st = ensure_scratch(c, select_scratch(ag->n, P, ndirs, &tiles), tiles);
  if (st) return st;
  const int64_t cnt_cap = sel_sizes(ag->n, P, ndirs).cnt_cap;
  return select_launch<EXACT>(c, ag, P, part_off, boxes, w, ndirs, idx_out, idx_cap, seg_off_out,
                              (hipStream_t)stream, Arena{c->scratch, c->scratch_cap, 0},
                              clear_first(c, ceil_div(cnt_cap + 1, SCAN_TILE)), lookback(c, 0));
}

// ---- selection without allocation ---------------------------------------------
// Scratch of ta_select_aura_static, one copy per device for the whole
// process: the per-agent codes, per-tile counts and their prefix, two
// look-back flag arrays and their tickets.  Sized for STATIC_AGENTS agents
// in STATIC_PARTS partitions with 26 directions (about 20.6 MB needed).
constexpr int64_t STATIC_AGENTS = int64_t(1) << 24;
constexpr int64_t STATIC_PARTS = 4096;
constexpr size_t STATIC_BYTES = size_t(22) << 20;
static __device__ __align__(256) uint8_t scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[MAX_DEVICES];  // device address of `scratch` on each device (null: not looked up)

// The carve of the static scratch: selection arrays, then the flags and
// tickets; returns the bytes used.
struct StaticLayout {
  uint64_t* flags[2];
  uint32_t* tickets;
  int64_t nflags;
  size_t used;
};
StaticLayout static_layout(uint8_t* base, int64_t n, int64_t P, int ndirs) {
  Arena ar{base, STATIC_BYTES, 0};
  carve(ar, n, P, ndirs);
  StaticLayout L;
  L.nflags = ceil_div(sel_sizes(n, P, ndirs).cnt_cap + 1, SCAN_TILE) + 1;
  L.flags[0] = ar.take<uint64_t>(L.nflags);
  L.flags[1] = ar.take<uint64_t>(L.nflags);
  L.tickets = ar.take<uint32_t>(2);
  L.used = ar.used;
  return L;
}
}  // namespace

namespace ta {
// Once per device, with that device current (called by ta_create): the
// device address of the static scratch.
ta_status static_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return TA_ERR_HIP;
  // the documented guarantee: every store of up to STATIC_AGENTS agents in
  // up to STATIC_PARTS partitions fits
  if (static_layout(nullptr, STATIC_AGENTS, STATIC_PARTS, 26).used > STATIC_BYTES) return TA_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_ptr[device]) return TA_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TA_ERR_HIP;
  g_static_ptr[device] = ptr;
  return TA_OK;
}
}  // namespace ta

extern "C" ta_status ta_select_aura_static(ta_ctx* c, const ta_agents* ag, int32_t P, const int64_t* part_off,
                                           const double* boxes, double w, int32_t ndirs, int32_t* idx_out,
                                           int64_t idx_cap, int64_t* seg_off_out, void* stream) {
  if (!c || !ag || P < 1 || (ndirs != 6 && ndirs != 26) || !part_off || !boxes || !seg_off_out || idx_cap < 0 ||
      (idx_cap > 0 && !idx_out) || ag->n < 0 || ag->n > INT32_MAX || (ag->n > 0 && !ag->f64) ||
      ag->f64_stride < ag->n || !(w == w))
    return TA_ERR_INVALID;
  void* base;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    base = c->device >= 0 && c->device < MAX_DEVICES ? g_static_ptr[c->device] : nullptr;
  }
  if (!base) return TA_ERR_HIP;
  // sizes beyond the array: rejected before anything is enqueued
  if (static_layout(nullptr, ag->n, P, ndirs).used > STATIC_BYTES) return TA_ERR_CAPACITY;
  use_family(c, FAM_SELECT);
  const StaticLayout L = static_layout(static_cast<uint8_t*>(base), ag->n, P, ndirs);
  const int64_t cnt_cap = sel_sizes(ag->n, P, ndirs).cnt_cap;
  // the first kernel zeroes the flags and ticket the scan uses (the array
  // keeps the previous call's contents); the scan zeroes the other pair
  const ClearFirst cf{L.flags[0], L.tickets, ceil_div(cnt_cap + 1, SCAN_TILE) + 1};
  LookBack lb;
  lb.flags = L.flags[0];
  lb.ticket = L.tickets;
  lb.clear_flags = L.flags[1];
  lb.clear_ticket = L.tickets + 1;
  lb.clear_n = L.nflags;
  lb.status = c->d_status;
  return select_launch<false>(c, ag, P, part_off, boxes, w, ndirs, idx_out, idx_cap, seg_off_out,
                              (hipStream_t)stream, Arena{static_cast<uint8_t*>(base), STATIC_BYTES, 0}, cf, lb);
}

extern "C" ta_status ta_select_aura(ta_ctx* c, const ta_agents* ag, int32_t P, const int64_t* part_off,
                                    const double* boxes, double w, int32_t ndirs, int32_t* idx_out, int64_t idx_cap,
                                    int64_t* seg_off_out, void* stream) {
  if (!c || !ag || P < 1 || (ndirs != 6 && ndirs != 26) || !part_off || !boxes || !seg_off_out || idx_cap < 0 ||
      (idx_cap > 0 && !idx_out) || ag->n < 0 || ag->n > INT32_MAX || (ag->n > 0 && !ag->f64) ||
      ag->f64_stride < ag->n || !(w == w))
    return TA_ERR_INVALID;
  return select_impl<false>(c, ag, P, part_off, boxes, w, ndirs, idx_out, idx_cap, seg_off_out, stream);
}

// Migrants: the aura kernels with thresholds at the box faces (w = 0; lo + 0
// and hi - 0 are lo and hi exactly) and an exact direction match, so that
// each agent outside its box lands in one of the 26 segments.
extern "C" ta_status ta_select_migrants(ta_ctx* c, const ta_agents* ag, int32_t P, const int64_t* part_off,
                                        const double* boxes, int32_t* idx_out, int64_t idx_cap, int64_t* seg_off_out,
                                        void* stream) {
  if (!c || !ag || P < 1 || !part_off || !boxes || !seg_off_out || idx_cap < 0 || (idx_cap > 0 && !idx_out) ||
      ag->n < 0 || ag->n > INT32_MAX || (ag->n > 0 && !ag->f64) || ag->f64_stride < ag->n)
    return TA_ERR_INVALID;
  return select_impl<true>(c, ag, P, part_off, boxes, 0.0, 26, idx_out, idx_cap, seg_off_out, stream);
}
