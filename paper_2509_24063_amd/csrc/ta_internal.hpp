// ta_internal.hpp -- host-side context shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/teraagent.h"
#include "ta_device.hpp"

struct ta_predictor {
  int device;
  void* dev;  // device copy of the weights (ta::PredW)
};

namespace ta {

// Persistent grid: enough resident blocks to fill the chip several times
// over; every kernel loops over its work with a grid stride or a ticket.
int persistent_blocks(int device);

struct Arena {
  uint8_t* base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  T* take(int64_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + used);
    used += sizeof(T) * (size_t)(count > 0 ? count : 1);
    return p;
  }
};

}  // namespace ta

// Kernel families with their own launch grid (tuned by ta_tune).
enum { FAM_SELECT = 0, FAM_SERIALIZE = 1, FAM_ENCODE = 2, FAM_DECODE = 3, N_FAMILIES = 4 };

struct ta_ctx {
  int device = 0;
  int cus = 256;
  int grid = 2048;                  // grid of the call in progress
  int grid_default = 2048;          // persistent grid: the chip filled several times over
  int fam_grid[N_FAMILIES] = {2048, 2048, 2048, 2048};
  bool capturing = false;           // a graph capture is in progress: no allocation
  int64_t rec_cap = 0;              // records per message side the delta scratch holds (0: from the sizes)
  uint32_t diff_op = 0;             // difference operator of encode and decode: 0 XOR, 1 byte-wise subtraction
  uint32_t n_classes = 0;
  uint16_t* d_nf = nullptr;  // device copies of the schema
  uint16_t* d_ni = nullptr;
  uint16_t max_f = 0, max_i = 0;
  uint32_t* d_status = nullptr;
  uint32_t* d_tickets = nullptr;  // ticket pair for the look-back ping-pong
  uint64_t* d_lb[2] = {nullptr, nullptr};
  int64_t lb_cap = 0;  // tiles per flag array
  uint8_t* scratch = nullptr;
  size_t scratch_cap = 0;
  // training-window tap of the encoder (null: off)
  int32_t* tap_in = nullptr;
  float* tap_tgt = nullptr;
  int64_t tap_cap = 0;
  unsigned long long* tap_count = nullptr;
  // timing of kernel families: `timed` is a comma-separated list of names;
  // every launch of a listed family leaves (family, start, end) events
  std::string timed;
  struct TimedLaunch {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<TimedLaunch> events;
};

namespace ta {

// Make sure the scratch arena holds `bytes` and the look-back arrays hold
// `tiles` tiles.  Returns TA_ERR_HIP on allocation failure.
ta_status ensure_scratch(ta_ctx* c, size_t bytes, int64_t tiles);

// Look-back descriptor for the k-th look-back kernel of a call (k = 0, 1, 2,
// ...): uses array k%2 and clears array (k+1)%2 for the next one.  The first
// kernel of a call that has look-back kernels must clear array 0 itself
// (clear_first()).
LookBack lookback(ta_ctx* c, int k);
// What the first kernel of a call clears: ticket 0 and the first `tiles`
// entries of array 0 (at least what the call's first look-back kernel uses;
// every later look-back kernel clears the whole other array).
struct ClearFirst {
  uint64_t* flags;
  uint32_t* ticket;
  int64_t n;
};
ClearFirst clear_first(ta_ctx* c, int64_t tiles);

__device__ inline void do_clear_first(const ClearFirst& cf) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cf.n; i += stride) cf.flags[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *cf.ticket = 0;
}

// Kernel timing: brackets launches of the named family with events.
struct Timed {
  ta_ctx* c;
  hipStream_t s;
  bool on;
  const char* name;
  hipEvent_t a{}, b{};
  Timed(ta_ctx* ctx, const char* name, hipStream_t stream);
  ~Timed();
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline void use_family(ta_ctx* c, int f) { c->grid = c->fam_grid[f]; }

// Looks up, once per device, the device address of the static scratch of
// ta_select_aura_static (with `device` current).
ta_status static_scratch_init(int device);

// Zero n int64 values on the stream with a kernel (graph-capture safe).
ta_status zero_i64(int64_t* p, int64_t n, hipStream_t s);
inline int grid_for(ta_ctx* c, int64_t items, int per_block) {
  int64_t g = ceil_div(items > 0 ? items : 1, per_block);
  if (g > c->grid) g = c->grid;
  return (int)g;
}

#define TA_HIP(call)                                  \
  do {                                                \
    if ((call) != hipSuccess) return TA_ERR_HIP;      \
  } while (0)
#define TA_LAUNCH_CHECK() TA_HIP(hipGetLastError())

}  // namespace ta
