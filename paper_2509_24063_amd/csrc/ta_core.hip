// ta_core.hip -- context lifecycle, scratch memory, status word, message view
// and validation, kernel timing.
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "ta_internal.hpp"
#include "ta_msg.hpp"
#include "ta_scratch.hpp"

using namespace ta;

namespace ta {

int persistent_blocks(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return 2048;
  return std::max(256, p.multiProcessorCount * 8);
}

ta_status ensure_scratch(ta_ctx* c, size_t bytes, int64_t tiles) {
  if (c->capturing && (bytes > c->scratch_cap || tiles > c->lb_cap)) return TA_ERR_CAPACITY;
  if (bytes > c->scratch_cap) {
    TA_HIP(hipDeviceSynchronize());
    if (c->scratch) TA_HIP(hipFree(c->scratch));
    c->scratch = nullptr;
    c->scratch_cap = 0;
    size_t cap = std::max(bytes + bytes / 4, (size_t)1 << 20);
    TA_HIP(hipMalloc(&c->scratch, cap));
    c->scratch_cap = cap;
  }
  if (tiles > c->lb_cap) {
    TA_HIP(hipDeviceSynchronize());
    for (int k = 0; k < 2; ++k) {
      if (c->d_lb[k]) TA_HIP(hipFree(c->d_lb[k]));
      c->d_lb[k] = nullptr;
    }
    int64_t cap = std::max<int64_t>(tiles + tiles / 4, 1024);
    for (int k = 0; k < 2; ++k) {
      TA_HIP(hipMalloc(&c->d_lb[k], sizeof(uint64_t) * cap));
      TA_HIP(hipMemset(c->d_lb[k], 0, sizeof(uint64_t) * cap));
    }
    c->lb_cap = cap;
  }
  return TA_OK;
}

LookBack lookback(ta_ctx* c, int k) {
  LookBack lb;
  lb.flags = c->d_lb[k & 1];
  lb.ticket = c->d_tickets + (k & 1);
  lb.clear_flags = c->d_lb[(k + 1) & 1];
  lb.clear_ticket = c->d_tickets + ((k + 1) & 1);
  lb.clear_n = c->lb_cap;
  lb.status = c->d_status;
  return lb;
}

ClearFirst clear_first(ta_ctx* c, int64_t tiles) {
  return ClearFirst{c->d_lb[0], c->d_tickets, tiles + 1 < c->lb_cap ? tiles + 1 : c->lb_cap};
}

__global__ void k_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

ta_status zero_i64(int64_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return TA_OK;
  k_zero_i64<<<(int)std::min<int64_t>(ceil_div(n, BLOCK), 1024), BLOCK, 0, s>>>(p, n);
  TA_LAUNCH_CHECK();
  return TA_OK;
}

// Is `name` one of the comma-separated names of `list`?
static bool listed(const std::string& list, const char* name) {
  const size_t n = strlen(name);
  for (size_t at = 0; at <= list.size();) {
    size_t end = list.find(',', at);
    if (end == std::string::npos) end = list.size();
    if (end - at == n && list.compare(at, n, name) == 0) return true;
    at = end + 1;
  }
  return false;
}

Timed::Timed(ta_ctx* ctx, const char* nm, hipStream_t stream) : c(ctx), s(stream), name(nm) {
  on = !c->timed.empty() && listed(c->timed, nm);
  if (on) {
    // (no system-scope fence when an event completes: the timestamps are all
    // that is wanted, and the fence lengthens the gap around the kernels)
    (void)hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
    (void)hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
    (void)hipEventRecord(a, s);
  }
}
Timed::~Timed() {
  if (on) {
    (void)hipEventRecord(b, s);
    c->events.push_back({name, a, b});
  }
}

}  // namespace ta

// ---------------------------------------------------------------------------
extern "C" ta_status ta_create(ta_ctx** out, uint32_t n_classes, const uint16_t* n_f64, const uint16_t* n_i32) {
  if (!out || n_classes == 0 || n_classes > 256 || !n_f64 || !n_i32) return TA_ERR_INVALID;
  for (uint32_t k = 0; k < n_classes; ++k)
    if (n_f64[k] > 64 || n_i32[k] > 64) return TA_ERR_INVALID;
  ta_ctx* c = new ta_ctx();
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return TA_ERR_HIP;
  }
  c->grid = c->grid_default = persistent_blocks(c->device);
  for (int f = 0; f < N_FAMILIES; ++f) c->fam_grid[f] = c->grid_default;
  {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, c->device) == hipSuccess) c->cus = p.multiProcessorCount;
  }
  c->n_classes = n_classes;
  for (uint32_t k = 0; k < n_classes; ++k) {
    c->max_f = std::max(c->max_f, n_f64[k]);
    c->max_i = std::max(c->max_i, n_i32[k]);
  }
  bool ok = hipMalloc(&c->d_nf, 2 * 256) == hipSuccess && hipMalloc(&c->d_ni, 2 * 256) == hipSuccess &&
            hipMalloc(&c->d_status, 64) == hipSuccess && hipMalloc(&c->d_tickets, 64) == hipSuccess;
  if (ok) {
    uint16_t nf[256] = {0}, ni[256] = {0};
    memcpy(nf, n_f64, 2 * n_classes);
    memcpy(ni, n_i32, 2 * n_classes);
    ok = hipMemcpy(c->d_nf, nf, 512, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_ni, ni, 512, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(c->d_status, 0, 64) == hipSuccess && hipMemset(c->d_tickets, 0, 64) == hipSuccess;
  }
  if (ok) ok = ensure_scratch(c, 1 << 20, 1024) == TA_OK;
  if (ok) ok = static_scratch_init(c->device) == TA_OK;
  if (!ok) {
    ta_destroy(c);
    return TA_ERR_HIP;
  }
  *out = c;
  return TA_OK;
}

extern "C" ta_status ta_destroy(ta_ctx* c) {
  if (!c) return TA_OK;
  // every step is attempted; the first failure is reported
  bool ok = hipDeviceSynchronize() == hipSuccess;
  for (void* p : {(void*)c->d_nf, (void*)c->d_ni, (void*)c->d_status, (void*)c->d_tickets, (void*)c->d_lb[0],
                  (void*)c->d_lb[1], (void*)c->scratch})
    ok = hipFree(p) == hipSuccess && ok;
  for (auto& e : c->events) {
    ok = hipEventDestroy(e.a) == hipSuccess && ok;
    ok = hipEventDestroy(e.b) == hipSuccess && ok;
  }
  delete c;
  return ok ? TA_OK : TA_ERR_HIP;
}

extern "C" ta_status ta_reserve(ta_ctx* c, int64_t max_agents, int64_t max_segments, int64_t max_records,
                                int64_t max_msg_bytes) {
  if (!c || max_agents < 0 || max_segments < 0 || max_records < 0 || max_msg_bytes < 0) return TA_ERR_INVALID;
  int64_t tiles = 0, t;
  size_t need = 0;
  need = std::max(need, select_scratch(max_agents, max_segments, 26, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, serialize_scratch(max_segments, max_records, &t));
  tiles = std::max(tiles, t);
  c->rec_cap = max_records;
  need = std::max(need, encode_scratch(max_segments, max_msg_bytes, max_msg_bytes, c->rec_cap, false, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, decode_scratch(max_segments, max_msg_bytes, max_msg_bytes, max_msg_bytes, c->rec_cap, false, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, validate_scratch(max_segments, max_msg_bytes, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, migrate_scratch(max_agents, max_segments, max_segments, max_msg_bytes, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, grow_scratch(max_records, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, compact_scratch(max_segments, max_msg_bytes, &t));
  tiles = std::max(tiles, t);
  return ensure_scratch(c, need, tiles);
}

extern "C" ta_status ta_status_poll(ta_ctx* c, void* stream) {
  if (!c) return TA_ERR_INVALID;
  uint32_t bits = 0;
  TA_HIP(hipStreamSynchronize((hipStream_t)stream));
  TA_HIP(hipMemcpy(&bits, c->d_status, 4, hipMemcpyDeviceToHost));
  TA_HIP(hipMemset(c->d_status, 0, 4));
  if (bits & (1u << ERR_INVALID)) return TA_ERR_INVALID;
  if (bits & (1u << ERR_REF)) return TA_ERR_REF_MISMATCH;
  if (bits & (1u << ERR_CORRUPT)) return TA_ERR_CORRUPT;
  if (bits & (1u << ERR_CAPACITY)) return TA_ERR_CAPACITY;
  if (bits) return TA_ERR_HIP;
  return TA_OK;
}

extern "C" int64_t ta_serialize_bound(int64_t nseg, int64_t nrec, int64_t max_words) {
  return 32 * nseg + 8 * ((nrec + 1) / 2 + nseg) + 8 * nrec * max_words;
}

extern "C" ta_status ta_set_difference_op(ta_ctx* c, int32_t op) {
  if (!c || op < 0 || op > 1) return TA_ERR_INVALID;
  c->diff_op = (uint32_t)op;
  return TA_OK;
}

extern "C" int64_t ta_delta_bound(int64_t nseg, int64_t cur_len, int64_t ref_len) {
  // headers and paddings per segment; presence bitmap (reference records are
  // >= 20 bytes each); word bitmaps and size tables of the residual (its words
  // are words of current records); new record sizes (4 bytes per record of
  // >= 16 bytes); the new records and the group blocks, which never exceed
  // 68/64 of the residual bytes they pack.
  return 96 * nseg + ref_len / 64 + cur_len / 64 + cur_len / 512 + cur_len / 4 + cur_len + cur_len / 16 + 64;
}

// ---------------------------------------------------------------------------
extern "C" ta_status ta_view(uint8_t* msg, int64_t len, const void* header, ta_view_t* out, void* stream) {
  if (!msg || !out || len < 32) return TA_ERR_INVALID;
  uint8_t hdr[40] = {0};
  if (header) {
    memcpy(hdr, header, 32);  // the caller's copy: msg itself is not read
  } else {
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, msg) == hipSuccess && attr.type == hipMemoryTypeDevice) on_device = true;
    (void)hipGetLastError();
    if (on_device) {
      // ordered after the work already enqueued on `stream`
      hipStream_t s = (hipStream_t)stream;
      TA_HIP(hipMemcpyAsync(hdr, msg, 32, hipMemcpyDeviceToHost, s));
      TA_HIP(hipStreamSynchronize(s));
    } else {
      memcpy(hdr, msg, 32);
    }
  }
  uint32_t magic, n, pad;
  uint16_t ver, flags;
  uint64_t rw, reserved;
  memcpy(&magic, hdr, 4);
  memcpy(&ver, hdr + 4, 2);
  memcpy(&flags, hdr + 6, 2);
  memcpy(&n, hdr + 8, 4);
  memcpy(&pad, hdr + 12, 4);
  memcpy(&rw, hdr + 16, 8);
  memcpy(&reserved, hdr + 24, 8);
  if (magic != TAM1_MAGIC || ver != 1 || flags != 0 || pad != 0 || reserved != 0) return TA_ERR_INVALID;
  if ((uint64_t)n > (uint64_t)len / 4 || rw > (uint64_t)len / 8 || rw < 2 * (uint64_t)n) return TA_ERR_INVALID;
  if (32 + 8 * (((uint64_t)n + 1) / 2) + 8 * rw != (uint64_t)len) return TA_ERR_INVALID;
  out->n = n;
  out->rec_words = (int64_t)rw;
  out->off = reinterpret_cast<const uint32_t*>(msg + 32);
  out->records = msg + 32 + 8 * (((uint64_t)n + 1) / 2);
  return TA_OK;
}

// ---- full validation ---------------------------------------------------------
namespace {

// one block: per segment header check, record counts and their prefix
__global__ __launch_bounds__(1024) void k_vv_setup(const uint8_t* msgs, const int64_t* off, int64_t nseg,
                                                   int64_t len, uint64_t* rbase, uint32_t* status) {
  __shared__ uint64_t s_carry;
  __shared__ uint64_t s_w[16];
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < nseg; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    uint64_t n_rec = 0;
    if (s < nseg) {
      const int64_t a = off[s], b = off[s + 1];
      uint32_t n;
      uint64_t rw;
      if (a < 0 || b < a || b > len || (a & 7) || !tam1_header(msgs + a, b - a, &n, &rw)) {
        fail(status, ERR_INVALID);
      } else {
        n_rec = n;
      }
    }
    // block exclusive scan over 1024 threads (16 waves)
    const uint64_t incl = wave_incl_scan(n_rec);
    if (lane_id() == 63) s_w[threadIdx.x / 64] = incl;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      pre += (i < (int)(threadIdx.x / 64)) ? s_w[i] : 0;
      tot += s_w[i];
    }
    if (s < nseg) rbase[s] = s_carry + pre + incl - n_rec;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) rbase[nseg] = s_carry;
}

__global__ __launch_bounds__(BLOCK) void k_vv_records(const uint8_t* msgs, const int64_t* off, int64_t nseg,
                                                      const uint64_t* rbase, uint32_t* status) {
  if (status_of(status) & (1u << ERR_INVALID)) return;
  const int64_t total = (int64_t)rbase[nseg];
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < total; g += (int64_t)gridDim.x * BLOCK) {
    const int64_t s = last_le<uint64_t>(rbase, 0, nseg, (uint64_t)g);
    const uint8_t* m = msgs + off[s];
    const uint32_t n = ld32(m + 8);
    const uint64_t rw = ld64(m + 16);
    uint32_t o;
    uint64_t uid, hdr;
    if (!tam1_record(m, n, rw, (uint32_t)(g - (int64_t)rbase[s]), &o, &uid, &hdr) || uid == 0) fail(status, ERR_INVALID);
  }
}

}  // namespace

namespace ta {
size_t validate_scratch(int64_t nseg, int64_t len, int64_t* tiles) {
  *tiles = 0;
  (void)len;
  return sizeof(uint64_t) * (size_t)(nseg + 1) + 256;
}
}  // namespace ta

extern "C" ta_status ta_view_validate(ta_ctx* c, const uint8_t* msgs, const int64_t* msg_off, int64_t nseg,
                                      int64_t msgs_len, void* stream) {
  if (!c || nseg < 0 || (nseg > 0 && (!msgs || !msg_off))) return TA_ERR_INVALID;
  if (nseg == 0) return TA_OK;
  c->grid = c->grid_default;
  int64_t tiles;
  ta_status st = ensure_scratch(c, validate_scratch(nseg, msgs_len, &tiles), tiles);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena ar{c->scratch, c->scratch_cap, 0};
  uint64_t* rbase = ar.take<uint64_t>(nseg + 1);
  k_vv_setup<<<1, 1024, 0, s>>>(msgs, msg_off, nseg, msgs_len, rbase, c->d_status);
  k_vv_records<<<c->grid, BLOCK, 0, s>>>(msgs, msg_off, nseg, rbase, c->d_status);
  TA_LAUNCH_CHECK();
  return TA_OK;
}

// ---- timing -----------------------------------------------------------------
extern "C" ta_status ta_time_kernel(ta_ctx* c, const char* name) {
  if (!c) return TA_ERR_INVALID;
  c->timed = name ? name : "";
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.clear();
  return TA_OK;
}

// Launches and summed milliseconds of the recorded events whose family is
// `name` (every family when name is null); those events are released.
static ta_status collect(ta_ctx* c, const char* name, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return TA_ERR_INVALID;
  double ms = 0;
  int64_t k = 0;
  std::vector<ta_ctx::TimedLaunch> keep;
  for (auto& e : c->events) {
    if (name && e.name != name) {
      keep.push_back(e);
      continue;
    }
    TA_HIP(hipEventSynchronize(e.b));
    float t = 0;
    TA_HIP(hipEventElapsedTime(&t, e.a, e.b));
    ms += t;
    ++k;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.swap(keep);
  *launches = k;
  *total_ms = ms;
  return TA_OK;
}

extern "C" ta_status ta_kernel_time(ta_ctx* c, int64_t* launches, double* total_ms) {
  return collect(c, nullptr, launches, total_ms);
}

extern "C" ta_status ta_kernel_time_of(ta_ctx* c, const char* name, int64_t* launches, double* total_ms) {
  if (!name) return TA_ERR_INVALID;
  return collect(c, name, launches, total_ms);
}
