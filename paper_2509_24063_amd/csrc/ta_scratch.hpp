// ta_scratch.hpp -- device scratch needed by each call (bytes, and look-back
// tiles through *tiles), from the host-known bounds of that call.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ta {
size_t select_scratch(int64_t n_agents, int64_t P, int ndirs, int64_t* tiles);
size_t serialize_scratch(int64_t nseg, int64_t idx_cap, int64_t* tiles);
// rec_cap > 0: at most rec_cap records per side (current, reference, new)
size_t encode_scratch(int64_t nseg, int64_t cur_len, int64_t ref_len, int64_t rec_cap, bool learned,
                      int64_t* tiles);
size_t decode_scratch(int64_t nseg, int64_t enc_len, int64_t ref_len, int64_t out_cap, int64_t rec_cap,
                      bool learned, int64_t* tiles);
size_t validate_scratch(int64_t nseg, int64_t len, int64_t* tiles);
size_t migrate_scratch(int64_t n_agents, int64_t P, int64_t nseg, int64_t msgs_len, int64_t* tiles);
size_t grow_scratch(int64_t n, int64_t* tiles);
size_t compact_scratch(int64_t nseg, int64_t cap, int64_t* tiles);
}  // namespace ta
