// ta_msg.hpp -- device-side reading of TAM1 messages.
#pragma once
#include "ta_device.hpp"

namespace ta {

__device__ inline uint64_t round8(uint64_t b) { return (b + 7) & ~uint64_t(7); }
__device__ inline uint64_t tam1_size(uint64_t n, uint64_t rw) { return 32 + 8 * ((n + 1) / 2) + 8 * rw; }

// Header and size identity of one message of len bytes.
__device__ inline bool tam1_header(const uint8_t* m, int64_t len, uint32_t* n_out, uint64_t* rw_out) {
  if (len < 32) return false;
  if (ld32(m) != TAM1_MAGIC || *reinterpret_cast<const uint16_t*>(m + 4) != 1 ||
      *reinterpret_cast<const uint16_t*>(m + 6) != 0)
    return false;
  if (ld32(m + 12) != 0 || ld64(m + 24) != 0) return false;
  const uint64_t n = ld32(m + 8), rw = ld64(m + 16);
  if (n > (uint64_t)len / 4 || rw > (uint64_t)len / 8) return false;
  if (tam1_size(n, rw) != (uint64_t)len) return false;
  if (n == 0 && rw != 0) return false;
  if (rw < 2 * n) return false;  // every record has at least 2 words
  if ((n & 1) && ld32(m + 32 + 4 * n) != 0) return false;
  *n_out = (uint32_t)n;
  *rw_out = rw;
  return true;
}

__device__ inline const uint8_t* tam1_records(const uint8_t* m, uint32_t n) { return m + 32 + 8 * ((n + 1) / 2); }

// Record i of a message whose header passed tam1_header: offsets form the
// running sum of record sizes (checked locally against the next offset),
// every record has at least 2 words.  Returns the record's word offset.
__device__ inline bool tam1_record(const uint8_t* m, uint32_t n, uint64_t rw, uint32_t i, uint32_t* off_out,
                                   uint64_t* hdr_out) {
  const uint8_t* offs = m + 32;
  const uint32_t o = ld32(offs + 4 * (uint64_t)i);
  if (i == 0 && o != 0) return false;
  if ((uint64_t)o + 2 > rw) return false;
  const uint64_t hdr = ld64(tam1_records(m, n) + 8 * (uint64_t)o + 8);
  const uint64_t words = hdr >> 32;
  if (words < 2) return false;
  const uint64_t next = (i + 1 < n) ? (uint64_t)ld32(offs + 4 * ((uint64_t)i + 1)) : rw;
  if ((uint64_t)o + words != next) return false;
  *off_out = o;
  *hdr_out = hdr;
  return true;
}

}  // namespace ta
