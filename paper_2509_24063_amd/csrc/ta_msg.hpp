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
// every record has at least 2 words.  Reading one takes two dependent steps,
// kept apart so that a caller can issue the first step's loads for several
// records before any second step: tam1_locate loads the record's offset and
// the next one (branch-free), tam1_words loads the record's uid (word 0) and
// header word (word 1) -- from record 0 when the offset is out of range,
// which tam1_valid reports -- and tam1_valid checks them.
struct Tam1Loc {
  uint32_t o;
  uint64_t next;
  bool o_ok;
};
__device__ inline Tam1Loc tam1_locate(const uint8_t* m, uint32_t n, uint64_t rw, uint32_t i) {
  const uint32_t* offs = reinterpret_cast<const uint32_t*>(m + 32);
  Tam1Loc r;
  r.o = offs[i];
  const uint32_t o1 = offs[i + 1 < n ? i + 1 : i];  // (always loaded: no branch around a load)
  r.next = i + 1 < n ? (uint64_t)o1 : rw;
  r.o_ok = (i != 0 || r.o == 0) && (uint64_t)r.o + 2 <= rw;
  return r;
}
// The record's two words (loads only) ...
__device__ inline void tam1_words(const uint8_t* m, uint32_t n, const Tam1Loc& r, uint64_t* uid_out,
                                  uint64_t* hdr_out) {
  const uint64_t* rec = reinterpret_cast<const uint64_t*>(tam1_records(m, n)) + (r.o_ok ? r.o : 0u);
  *uid_out = rec[0];
  *hdr_out = rec[1];
}
// ... and the checks on them.
__device__ inline bool tam1_valid(const Tam1Loc& r, uint64_t hdr) {
  const uint64_t words = hdr >> 32;
  return r.o_ok && words >= 2 && (uint64_t)r.o + words == r.next;
}
__device__ inline bool tam1_fetch(const uint8_t* m, uint32_t n, const Tam1Loc& r, uint64_t* uid_out,
                                  uint64_t* hdr_out) {
  tam1_words(m, n, r, uid_out, hdr_out);
  return tam1_valid(r, *hdr_out);
}
// Both steps for one record; gives its word offset too.
__device__ inline bool tam1_record(const uint8_t* m, uint32_t n, uint64_t rw, uint32_t i, uint32_t* off_out,
                                   uint64_t* uid_out, uint64_t* hdr_out) {
  const Tam1Loc r = tam1_locate(m, n, rw, i);
  *off_out = r.o;
  return tam1_fetch(m, n, r, uid_out, hdr_out);
}

}  // namespace ta
