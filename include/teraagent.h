/*
 * teraagent.h -- C ABI of the MI355X aura-exchange library (libteraagent.so).
 *
 * One GPU holds one rank's share of space (one or many partition boxes).  Each
 * iteration the library
 *   1. selects the aura agents of every partition for each neighbour
 *      direction                                   (ta_select_aura),
 *   2. serializes them into flat, in-place usable TAM1 messages
 *                                                  (ta_serialize, ta_view),
 *   3. delta-encodes every message against the previous iteration's message
 *      of the same neighbour pair                  (ta_delta_encode),
 *   4. decodes and applies the encoding on the receive side
 *                                                  (ta_delta_decode),
 * and moves the agents that left their partition's box to the partition that
 * owns their new position (ta_select_migrants, ta_serialize,
 * ta_migrate_apply).
 * Paper: Sec. 2.1 (aura update, agent migration), Sec. 2.2 / 2.2.1 (TA IO serialization and
 * single-pass deserialization), Sec. 2.3 (delta encoding against a reference
 * shared by sender and receiver).
 *
 * Conventions for every call:
 *  - Pointers marked "device" are HIP device pointers (e.g. a torch CUDA
 *    tensor's data_ptr()); "host" pointers are ordinary memory.  The caller
 *    owns every buffer it passes.  Device buffers must be 8-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work and return without synchronising; results are valid once the
 *    stream has reached them.
 *  - Counts produced on the device stay on the device; nothing in the
 *    exchange calls syncs the host, so an iteration can be captured in a
 *    HIP graph once the context has been sized with ta_reserve.
 *  - Errors found on the host (bad arguments) are returned at once.  Errors
 *    that depend on data (corrupt encodings, wrong reference, duplicate or
 *    zero uid, output larger than its capacity) are recorded in the
 *    context's device status word and read by ta_status_poll.  After such
 *    an error the outputs of that call are unspecified, but nothing is ever
 *    written outside the buffers and capacities passed in.
 *  - Several errors in one call are reported with the precedence
 *    TA_ERR_INVALID, TA_ERR_REF_MISMATCH, TA_ERR_CORRUPT, TA_ERR_CAPACITY.
 *  - A context is used by one host thread and one stream at a time.
 *
 * Wire formats (little-endian, every record and section 8-byte aligned,
 * every pad byte zero):
 *
 *  TAM1 message (Sec. 2.2.1; offsets stand in for the paper's pointer
 *  markers so a GPU can address record i directly):
 *    u32 magic "TAM1" | u16 version 1 | u16 flags 0 | u32 n | u32 0 |
 *    u64 rec_words | u64 0 | u32 off[n] (record i starts at word off[i] of
 *    the record area; off[0]=0, off[i+1]=off[i]+words_i), padded to 8 |
 *    record area (rec_words words).
 *  Record: u64 uid (non-zero) | u16 class, u16 behaviour count, u32 record
 *    words | the class's fp64 fields (0..2 position, 3 diameter) | its int32
 *    attributes, padded to 8 | behaviour blocks verbatim (u32 class,
 *    u32 payload bytes (multiple of 8), payload).  The class id stands in
 *    for the vtable pointer.
 *
 *  TAD1 encoding of a current message C against a reference R (Sec. 2.3):
 *    64-byte header: u32 magic "TAD1" | u16 version 1 | u8 mode (0 plain,
 *    1 learned, 2 mixed) | u8 packer (1) | u32 n_ref | u32 n_match | u32 n_new |
 *    u32 operator (0 XOR, 1 byte-wise subtraction) | u64 ref_words |
 *    u64 XOR of all reference uids | u64 W |
 *    u64 new_words | u64 var_bytes;
 *    presence bitmap (ceil(n_ref/64) u64; bit j: reference slot j matched);
 *    word bitmap (ceil(W/64) u64; bit q: residual word q non-zero);
 *    group block sizes (ceil(W/64) u8, bytes/8; in mode 2 bit 7 set marks a
 *    group whose residual is against the learned X), padded to 8;
 *    new record sizes (n_new u32 words), padded to 8;
 *    new records verbatim (new_words words);
 *    group blocks (var_bytes): for each group of 64 residual words, one
 *    4-bit length per non-zero word (bytes up to its highest non-zero byte;
 *    two per byte, low nibble first), then those low-order bytes of each
 *    non-zero word, padded to a multiple of 8 bytes.
 *  A reference slot is matched when C holds a record with the same uid and
 *  the same header word.  The residual combines the matched current
 *  records, taken in reference order, with X by XOR (operator 0) or by
 *  byte-wise subtraction modulo 256 (operator 1).  X is the reference record
 *  (plain) or the reference record with words 2..5 replaced by the predictor's
 *  estimate (learned; in mixed mode per 64-word group, as flagged).  C' = matched records in reference order followed by
 *  the new records in C order; it is returned to the sender and rebuilt by
 *  the receiver, and it is the next reference of both.
 */
#ifndef TERAAGENT_H
#define TERAAGENT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TA_OK = 0,
  TA_ERR_INVALID = 1,      /* bad argument, bad message, zero or duplicate uid */
  TA_ERR_CAPACITY = 2,     /* an output buffer is too small */
  TA_ERR_CORRUPT = 3,      /* a TAD1 encoding is damaged */
  TA_ERR_REF_MISMATCH = 4, /* a TAD1 encoding was made against another reference */
  TA_ERR_HIP = 5           /* a HIP runtime call failed */
} ta_status;

typedef struct ta_ctx ta_ctx;

/* Agent store: struct of arrays, all partitions concatenated, all device. */
typedef struct {
  int64_t n;               /* number of agents */
  const uint64_t *uid;     /* [n] */
  const uint16_t *cls;     /* [n] class id, < n_classes */
  const uint16_t *nb;      /* [n] behaviour block count */
  const double *f64;       /* field k of agent i at f64[k * f64_stride + i] */
  int64_t f64_stride;      /* >= n */
  const int32_t *i32;      /* attribute k of agent i at i32[k * i32_stride + i] */
  int64_t i32_stride;      /* >= n */
  const int64_t *beh_off;  /* [n+1] byte offsets into beh, multiples of 8 */
  const uint8_t *beh;      /* behaviour blocks of agent i: beh[beh_off[i] .. beh_off[i+1]) */
} ta_agents;

/* Read-only description of one TAM1 message (see ta_view). */
typedef struct {
  int64_t n;               /* records */
  int64_t rec_words;       /* 8-byte words in the record area */
  const uint32_t *off;     /* n word offsets (same memory space as the message) */
  uint8_t *records;        /* record area; record i at records + 8 * off[i] */
} ta_view_t;

/* Create a context for a class schema: class c has n_f64[c] fp64 fields and
 * n_i32[c] int32 attributes (host arrays of n_classes entries, n_classes <=
 * 256, n_f64[c] <= 64, n_i32[c] <= 64).  Uses the current HIP device. */
ta_status ta_create(ta_ctx **out, uint32_t n_classes, const uint16_t *n_f64, const uint16_t *n_i32);

/* Release the context and its device scratch memory (after waiting for the
 * device).  Null is accepted (TA_OK).  The context is gone afterwards even
 * when a HIP call failed on the way; that failure is returned as
 * TA_ERR_HIP. */
ta_status ta_destroy(ta_ctx *ctx);

/* Pre-size the device scratch memory for calls with at most max_agents
 * agents in the store, max_segments segments, idx_cap <= max_records and
 * message buffers (cur_len, ref_len, enc_len, out_cap, ...) of at most
 * max_msg_bytes bytes.  Calls that need more grow the scratch memory
 * themselves (which allocates and synchronises); calls within the reserved
 * sizes allocate nothing and may be captured in a HIP graph.
 * max_records > 0 also caps the records per side (current, reference, new)
 * that ta_delta_encode / ta_delta_decode size their scratch for, instead of
 * the bound the byte sizes give (20 bytes per record); a call with more
 * records then fails with TA_ERR_CAPACITY.  max_records = 0 removes the cap. */
ta_status ta_reserve(ta_ctx *ctx, int64_t max_agents, int64_t max_segments, int64_t max_records,
                     int64_t max_msg_bytes);

/* Wait for `stream`, read and clear the device status word: TA_OK or the
 * highest-precedence data-dependent error of the calls since the last poll. */
ta_status ta_status_poll(ta_ctx *ctx, void *stream);

/* Aura selection (Sec. 2.1, "Aura Update").
 * P partitions; partition p holds agents [part_off[p], part_off[p+1]) of the
 * store (part_off: device int64[P+1]) and owns the half-open box boxes[6p ..
 * 6p+5] = lo0 lo1 lo2 hi0 hi1 hi2 (device double[6P]).  ndirs is 6 (face
 * neighbours) or 26 (faces, edges, corners).  With thresholds lo+w and hi-w
 * (each one fp64 operation), an agent belongs to direction (dx,dy,dz) when on
 * every axis with d=-1 its coordinate is < lo+w and on every axis with d=+1
 * it is >= hi-w.  Segment s = p*ndirs + k, k-th direction in ascending order
 * of (dx+1) + 3(dy+1) + 9(dz+1).
 * Output: idx_out (device int32[idx_cap]) store indices, segment by segment,
 * ascending within a segment; seg_off_out (device int64[P*ndirs+1]) segment
 * starts.  More than idx_cap selections -> TA_ERR_CAPACITY (seg_off_out still
 * holds the needed sizes).  Agents beyond 2^31-1 are not supported. */
ta_status ta_select_aura(ta_ctx *ctx, const ta_agents *agents, int32_t P, const int64_t *part_off,
                         const double *boxes, double w, int32_t ndirs, int32_t *idx_out, int64_t idx_cap,
                         int64_t *seg_off_out, void *stream);

/* Aura selection that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Arguments, results and errors are those
 * of ta_select_aura, whose kernels it runs; its scratch memory (agent
 * codes, per-tile counts and their prefix, look-back flags) is a static
 * device array of 22 MiB that the library holds on every device it runs on
 * until the process ends, instead of the context's scratch, which it never
 * grows.  Every store of at most 2^24 agents in at most 4096 partitions fits;
 * a larger one is rejected with TA_ERR_CAPACITY before anything is
 * enqueued.  All calls on one device share the array and find the previous
 * call's contents in it (each call clears what it needs): calls that
 * overlap on one device, on any streams or contexts, race and give
 * unspecified results.  The status word is the context's. */
ta_status ta_select_aura_static(ta_ctx *ctx, const ta_agents *agents, int32_t P, const int64_t *part_off,
                                const double *boxes, double w, int32_t ndirs, int32_t *idx_out, int64_t idx_cap,
                                int64_t *seg_off_out, void *stream);

/* Migrant selection (Sec. 2.1, "Agent Migration"): the agents that left
 * their partition's box, by the neighbour box they moved into.  Per axis an
 * agent's offset is -1 when its coordinate is < lo, +1 when >= hi, 0
 * otherwise; an agent with a nonzero offset belongs to exactly that one of the
 * 26 directions (not to the directions of its faces or edges, unlike the
 * aura), agents inside their box to none.  A NaN coordinate counts as inside.
 * Arguments, segment order (s = p*26 + k) and outputs as for ta_select_aura
 * with ndirs = 26; the segments are serialized by ta_serialize and taken in
 * by ta_migrate_apply.  More than idx_cap migrants -> TA_ERR_CAPACITY
 * (seg_off_out still holds the needed sizes). */
ta_status ta_select_migrants(ta_ctx *ctx, const ta_agents *agents, int32_t P, const int64_t *part_off,
                             const double *boxes, int32_t *idx_out, int64_t idx_cap, int64_t *seg_off_out,
                             void *stream);

/* Record keys: the uid and header word of every record of a message set,
 * in record order (message 0's records, then message 1's, ...): key[2i] =
 * uid, key[2i+1] = header word of record i.  Device memory, 16-byte aligned,
 * 16 bytes per record.  They are optional companions of a message set: the
 * library writes them beside the messages it writes (ta_serialize, the C'
 * of ta_delta_encode and ta_delta_decode), and the delta calls that are
 * given the keys of their inputs read each record's uid and header from
 * them instead of from the record (16 bytes instead of the record's cache
 * lines); offsets and sizes are still checked against the messages.
 * Whoever passes keys in vouches that they describe the messages: after a
 * message has been changed where a uid or header word lives, its keys must
 * be rewritten or left out. */
typedef struct {
  const uint64_t *cur;     /* keys of the current messages (ta_delta_encode), nullable */
  const uint64_t *ref;     /* keys of the reference messages, nullable */
  uint64_t *out;           /* nullable: receives the keys of C' (newref / out) */
  int64_t out_cap;         /* records `out` holds; more C' records -> TA_ERR_CAPACITY */
} ta_keys;

/* TA IO serialization (Sec. 2.2.1, "Serialization"): one TAM1 message per
 * segment.  idx / seg_off (device) as produced by ta_select_aura, nseg
 * segments, at most idx_cap records in total.  Messages are packed densely
 * into out (device, out_cap bytes); msg_off_out (device int64[nseg+1])
 * receives their byte offsets.  A class id >= n_classes or a behaviour range
 * that is not a multiple of 8 bytes -> TA_ERR_INVALID; messages larger than
 * out_cap -> TA_ERR_CAPACITY (msg_off_out still holds the needed sizes).
 * keys_out (nullable; keys_cap >= idx_cap records) receives the records'
 * keys (see ta_keys). */
ta_status ta_serialize(ta_ctx *ctx, const ta_agents *agents, const int32_t *idx, const int64_t *seg_off,
                       int64_t nseg, int64_t idx_cap, uint8_t *out, int64_t out_cap, int64_t *msg_off_out,
                       uint64_t *keys_out, int64_t keys_cap, void *stream);

/* Upper bound of the serialized size of nrec records of at most max_words
 * words each, in nseg messages. */
int64_t ta_serialize_bound(int64_t nseg, int64_t nrec, int64_t max_words);

/* View of one TAM1 message (Sec. 2.2.1, "Deserialization"/"Mutability"):
 * O(1).  Checks the header (magic, version, zero flags and reserved fields,
 * n <= len/4, rec_words >= 2n) and the size identity
 * len == 32 + 8*ceil(n/2) + 8*rec_words, and fills *out with pointers into
 * the message itself, so records are read and updated in place.  The
 * message may be in host or device memory.  header (nullable, host): the
 * message's first 32 bytes as the caller already holds them; msg is then
 * not read, nothing is copied and nothing waits, so the call may sit
 * between captured or queued work.  header == NULL with a device message:
 * the 32 header bytes are copied on `stream` and the host waits for that
 * stream, so work enqueued on it before the call (e.g. the ta_serialize that
 * wrote the message) is complete first; work on other streams must be
 * ordered with `stream` by the caller.  The offsets and records are not
 * checked here (ta_view_validate does that).  Bad header or size ->
 * TA_ERR_INVALID. */
ta_status ta_view(uint8_t *msg, int64_t len, const void *header, ta_view_t *out, void *stream);

/* Growth of records used in place (Sec. 2.2.1, "Mutability": a record that
 * needs more room than its message gives it moves to a new block outside its
 * message, and the old block is given up).  The new blocks come from an
 * arena that follows the last message in the same device buffer: bytes
 * [msg_off[nseg], cap) of msgs, of which *arena_used (device int64, a
 * multiple of 8) are taken.  For k < n, record rec[k] of message seg[k]
 * (device arrays; (seg, rec) strictly ascending) moves to the next free
 * words[k] words of the arena (words[k] >= its size): its words are copied,
 * the rest zeroed, its header's word count set to words[k], and its offset
 * entry redirected there (offsets count 8-byte words from the message's
 * record area, so they may point past it; views see the grown record).
 * *arena_used grows by 8 * sum(words).  A listed record whose block in use
 * is not below msg_off[nseg] + *arena_used, a bad message or list, or cap >
 * 2^35 -> TA_ERR_INVALID; an arena too small -> TA_ERR_CAPACITY; in both
 * cases nothing is written.  A message with redirected offsets is read by
 * ta_view and by the caller, not by the delta encoder: ta_view_compact first. */
ta_status ta_view_grow(ta_ctx *ctx, uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg,
                       const int32_t *seg, const uint32_t *rec, const uint32_t *words, int64_t n,
                       int64_t *arena_used, void *stream);

/* Canonical copies of messages whose offsets may be redirected (Sec. 2.2.1):
 * message s of out holds the records of message s of msgs (cap bytes) in
 * order, offsets the running sum of their sizes.  out_off (device
 * int64[nseg+1]) receives the output offsets, also when they exceed out_cap
 * (-> TA_ERR_CAPACITY, nothing else written).  A bad header, or a record
 * whose block is not inside msgs -> TA_ERR_INVALID (out and out_off
 * unspecified).  Compacting a canonical message copies it unchanged. */
ta_status ta_view_compact(ta_ctx *ctx, const uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg,
                          uint8_t *out, int64_t out_cap, int64_t *out_off, void *stream);

/* Full O(n) check of nseg device messages (msgs at msg_off[s] ..
 * msg_off[s+1], 8-byte aligned, inside msgs_len bytes): every check of
 * ta_view, a zero pad entry after an odd offset table, offsets that are the
 * running sum of the record sizes from 0 to rec_words, record sizes of at
 * least 2 words, and a non-zero uid in every record (uids name one agent
 * each, Sec. 2.5; zero is reserved).  Problems -> TA_ERR_INVALID in the
 * status word. */
ta_status ta_view_validate(ta_ctx *ctx, const uint8_t *msgs, const int64_t *msg_off, int64_t nseg,
                           int64_t msgs_len, void *stream);

/* An agent store the library writes: device arrays with room for cap agents
 * (the column layout of ta_agents) and beh_cap behaviour bytes; beh_off has
 * cap+1 entries.  Base pointers 8-byte aligned. */
typedef struct {
  int64_t cap;
  uint64_t *uid;
  uint16_t *cls;
  uint16_t *nb;
  double *f64;             /* field k of agent j at f64[k * f64_stride + j], f64_stride >= cap */
  int64_t f64_stride;
  int32_t *i32;            /* attribute k of agent j at i32[k * i32_stride + j], i32_stride >= cap */
  int64_t i32_stride;
  int64_t *beh_off;        /* [cap+1] */
  uint8_t *beh;
  int64_t beh_cap;
} ta_store;

/* The store after one exchange of migrants (Sec. 2.1, "Agent Migration";
 * records as serialized in Sec. 2.2.1), built in one pass into `out` (which
 * must not overlap `in`).  Partition q of the result holds:
 *   1. the agents of input partition q (part_off, device int64[P+1]) whose
 *      position lies inside box q (boxes as for ta_select_aura; the agents
 *      ta_select_migrants does not select), in store order, with all of the
 *      schema's fp64 and int32 columns (the largest class's counts) and
 *      their behaviour bytes;
 *   2. then the records of every message s whose msg_part[s] == q (device
 *      int32[nseg]; < 0: the message is checked but not taken in), messages
 *      in ascending s, records in message order, unpacked: uid, class,
 *      behaviour count, the class's fp64 fields and int32 attributes (zero in
 *      the other columns), the rest of the record as behaviour bytes.
 * Both stores hold as many fp64 and int32 columns as the schema's largest
 * class (the columns of every kept agent are copied).
 * Messages: nseg TAM1 messages at msg_off[s] .. msg_off[s+1] of msgs (device,
 * msgs_len bytes, 8-byte aligned starts).  part_off_out (device int64[P+1])
 * receives the result's partition starts and sizes_out (device int64[2]) its
 * agent count and behaviour bytes, also when they exceed out->cap or
 * out->beh_cap (-> TA_ERR_CAPACITY, nothing else written).  A bad partition
 * table, message, record (zero uid, class >= n_classes, fewer words than the
 * class's fixed part), msg_part[s] >= P or a behaviour range of a kept agent
 * that is not whole 8-byte words -> TA_ERR_INVALID (outputs unspecified).
 * The result's beh_off[agents] is its behaviour byte count. */
ta_status ta_migrate_apply(ta_ctx *ctx, const ta_agents *in, int32_t P, const int64_t *part_off,
                           const double *boxes, const uint8_t *msgs, int64_t msgs_len, const int64_t *msg_off,
                           int64_t nseg, const int32_t *msg_part, const ta_store *out, int64_t *part_off_out,
                           int64_t *sizes_out, void *stream);

/* Predictor for learned delta encoding: an integer MLP 12 -> 64 -> 64 -> 4
 * (int8 weights, int32 accumulation) estimating the next position and
 * diameter of an agent from its last moves.  Blob (host, 5672 bytes): u32
 * magic "TAP1", u32 version 1, int8 W1[64][12], int8 W2[64][64], int8
 * W3[4][64], int32 b1[64], int32 b2[64], int32 b3[4], u8 r1, r2, r3, 5 zero
 * bytes, f64 cell; |b| <= 2^24, r <= 24, cell > 0.  Copied to the device. */
typedef struct ta_predictor ta_predictor;
ta_status ta_predictor_load(ta_ctx *ctx, const void *blob, size_t len, ta_predictor **out);
void ta_predictor_free(ta_predictor *p);

/* Evaluate the predictor on n rows of 12 int32 inputs (device, row-major; the
 * inputs the exchange forms are q(R-h1) x4, q(h1-h2) x4, neighbour count,
 * behaviour count, class, history length) into n rows of 4 int32 outputs
 * (device): integer layers with int32 accumulation, requantisation
 * floor((a + 2^(r-1)) / 2^r), ReLU clamp to [0,127] after layers 1 and 2,
 * outputs clamped to +-2^24. */
ta_status ta_predictor_eval(ta_ctx *ctx, const ta_predictor *p, const int32_t *in, int32_t *q, int64_t n,
                            void *stream);

/* Per reference slot history of the predicted words (device):
 * h1[4j..4j+3] words 2..5 of slot j's record one exchange before the
 * reference, h2 two exchanges before (raw fp64 bits), hlen[j] in {0,1,2}. */
typedef struct {
  uint64_t *h1;
  uint64_t *h2;
  uint8_t *hlen;
  int64_t cap;             /* slots the arrays hold; a learned call whose hist_in
                              holds fewer slots than its reference has records
                              fails with TA_ERR_INVALID (found on the device,
                              reported by ta_status_poll) */
} ta_history;

/* Delta encoding (Sec. 2.3) of nseg current messages against nseg
 * reference messages (same segment order).  cur/ref: device buffers of
 * cur_len/ref_len bytes holding the messages at cur_off/ref_off (device
 * int64[nseg+1]).  pred == NULL: plain mode.  Otherwise each 64-word group
 * of the residual takes the learned X when that makes its block strictly
 * smaller; a segment where no group does is plain (mode 0), one where every
 * group with a different size does is learned (mode 1), else mixed (mode 2);
 * hist_in (slots flattened in segment order, device) must then be given.  hist_out (nullable) receives the history of C';
 * its arrays must not overlap those of hist_in (else TA_ERR_INVALID).
 * Outputs: enc (device, enc_cap bytes) with the TAD1 encodings packed densely
 * at enc_off (device int64[nseg+1]); newref (device, newref_cap bytes) with
 * the C' messages at newref_off (device int64[nseg+1]); modes (nullable,
 * device uint8[nseg]) the mode chosen per segment (0, 1 or 2).  keys
 * (nullable): keys of cur and ref to read, and a buffer for the keys of C'.
 * Invalid or duplicate input -> TA_ERR_INVALID; too small outputs ->
 * TA_ERR_CAPACITY. */
ta_status ta_delta_encode(ta_ctx *ctx, int64_t nseg, const uint8_t *cur, int64_t cur_len, const int64_t *cur_off,
                          const uint8_t *ref, int64_t ref_len, const int64_t *ref_off, const ta_predictor *pred,
                          const ta_history *hist_in, ta_history *hist_out, uint8_t *enc, int64_t enc_cap,
                          int64_t *enc_off, uint8_t *newref, int64_t newref_cap, int64_t *newref_off,
                          uint8_t *modes, const ta_keys *keys, void *stream);

/* The difference operator (Sec. 2.3 leaves it open) of this context's
 * later ta_delta_encode and ta_delta_decode calls: 0 XOR (the default), 1
 * each byte subtracted modulo 256 (decoding adds it back).  The zero bytes,
 * and so every size, are those of XOR.  The operator is written into each
 * encoding (header bytes 20..23); a decoder set to another operator rejects
 * it with TA_ERR_INVALID, as both ends of a pair share it like the
 * predictor.  Other values -> TA_ERR_INVALID.  Not to be changed while calls
 * of the context are being captured into a graph. */
ta_status ta_set_difference_op(ta_ctx *ctx, int32_t op);

/* Upper bound of the encoding size for current messages of cur_len bytes
 * and a reference of ref_len bytes, nseg segments. */
int64_t ta_delta_bound(int64_t nseg, int64_t cur_len, int64_t ref_len);

/* Delta decoding (Sec. 2.3): rebuild C' of every segment from its TAD1
 * encoding (enc at enc_off, device) and the stored reference (ref at
 * ref_off, device).  Learned and mixed encodings (modes 1 and 2) need pred
 * and hist_in, else TA_ERR_INVALID.  Output: C' messages packed densely in
 * out (device, out_cap bytes) at out_off (device int64[nseg+1]); hist_out
 * (nullable) as for encoding.  Damaged encodings (mode above 2 included) ->
 * TA_ERR_CORRUPT; encodings made against another reference ->
 * TA_ERR_REF_MISMATCH; too small output -> TA_ERR_CAPACITY.  keys
 * (nullable; cur unused): keys of ref to read, and a buffer for the keys of
 * C'. */
ta_status ta_delta_decode(ta_ctx *ctx, int64_t nseg, const uint8_t *enc, int64_t enc_len, const int64_t *enc_off,
                          const uint8_t *ref, int64_t ref_len, const int64_t *ref_off, const ta_predictor *pred,
                          const ta_history *hist_in, ta_history *hist_out, uint8_t *out, int64_t out_cap,
                          int64_t *out_off, const ta_keys *keys, void *stream);

/* Timing of kernel families for measurement: name is a comma-separated list
 * of family names (NULL or "" disables timing); while it is set, every
 * launch of a listed family is bracketed by HIP events on its stream.
 * ta_kernel_time returns (after waiting for the events) the number of timed
 * launches and their summed duration in milliseconds since the last call,
 * over every family; ta_kernel_time_of the same for one family (its events
 * only).  Names: "select_count", "select_scatter", "serialize_pack",
 * "encode_match" (every encoder kernel before the residual: headers,
 * UID join, layout, directory), "encode_join" (the UID join alone),
 * "encode_groups" (residual, block sizes, offsets and blocks in one kernel;
 * in learned encodings both residuals and the smaller block), "predict"
 * (learned encodings and decodings: neighbour counts and the network),
 * "decode_unpack" (which also applies the residual to
 * the reference), "migrate_keep" (ta_migrate_apply: the agents that stay,
 * copied into the new store). */
ta_status ta_time_kernel(ta_ctx *ctx, const char *name);
ta_status ta_kernel_time(ta_ctx *ctx, int64_t *launches, double *total_ms);
ta_status ta_kernel_time_of(ta_ctx *ctx, const char *name, int64_t *launches, double *total_ms);

/* ---- One exchange iteration as a unit: batched over every partition and
 * segment, run eagerly, captured in a HIP graph, or tuned. ---- */

/* Every argument of the four calls of one iteration: ta_select_aura over P
 * partitions (segments nseg = P * ndirs), ta_serialize of the selection,
 * ta_delta_encode against the sender's reference, and (rx_out non-NULL)
 * ta_delta_decode of that encoding against the receiver's reference.  Each
 * member has the meaning, memory space and ownership of the argument of the
 * same name there (msgs/msgs_cap/msg_off are ta_serialize's out/out_cap/
 * msg_off_out and ta_delta_encode's cur/cur_len/cur_off; rx_* are
 * ta_delta_decode's ref/hist/out arguments).  The structs pointed to are
 * read during the call only. */
typedef struct {
  const ta_agents *agents;
  int32_t P;
  int32_t ndirs;
  const int64_t *part_off;
  const double *boxes;
  double w;
  int32_t *idx;
  int64_t idx_cap;
  int64_t *seg_off;
  uint8_t *msgs;
  int64_t msgs_cap;
  int64_t *msg_off;
  const ta_predictor *pred;
  const uint8_t *ref;
  int64_t ref_len;
  const int64_t *ref_off;
  const ta_history *hist_in;
  ta_history *hist_out;
  uint8_t *enc;
  int64_t enc_cap;
  int64_t *enc_off;
  uint8_t *newref;
  int64_t newref_cap;
  int64_t *newref_off;
  uint8_t *modes;
  const uint8_t *rx_ref;
  int64_t rx_ref_len;
  const int64_t *rx_ref_off;
  const ta_history *rx_hist_in;
  ta_history *rx_hist_out;
  uint8_t *rx_out;
  int64_t rx_out_cap;
  int64_t *rx_out_off;
  /* record keys (nullable each, see ta_keys): of msgs (written by
   * ta_serialize, read by ta_delta_encode), of ref, of newref (written), of
   * rx_ref, of rx_out (written); every written one holds keys_cap records */
  uint64_t *msg_keys;
  const uint64_t *ref_keys;
  uint64_t *newref_keys;
  const uint64_t *rx_ref_keys;
  uint64_t *rx_out_keys;
  int64_t keys_cap;
} ta_iteration;

/* Enqueue the iteration's calls in order; the first host-side error is
 * returned (data errors go to the status word as for the single calls). */
ta_status ta_iteration_run(ta_ctx *ctx, const ta_iteration *it, void *stream);

/* Capture the iteration into a HIP graph on `stream` (not the NULL stream).
 * The context's scratch memory is sized first, so the captured calls
 * allocate nothing; every pointer, capacity and launch shape is fixed in the
 * graph, while counts and sizes stay on the device, so the graph is valid
 * for any data that fits the capacities (e.g. a store whose partitions grow
 * and shrink within agents->n).  The graph uses the context's scratch
 * memory: replays of graphs of one context must not overlap.  Kernel timing
 * (ta_time_kernel) does not apply inside graphs. */
typedef struct ta_graph ta_graph;
ta_status ta_graph_capture(ta_ctx *ctx, const ta_iteration *it, void *stream, ta_graph **out);
ta_status ta_graph_launch(ta_graph *g, void *stream);
void ta_graph_free(ta_graph *g);

/* Launch grids of the four kernel families (select, serialize, encode,
 * decode), in blocks; ta_set_grids(ctx, NULL) restores the defaults. */
ta_status ta_get_grids(ta_ctx *ctx, int32_t *grids);
ta_status ta_set_grids(ta_ctx *ctx, const int32_t *grids);

/* Choose the launch grid of each kernel family for this iteration's shape
 * by timing it (median of `reps` runs per candidate, coordinate descent over
 * 1..16 blocks per compute unit) and keep the fastest in the context.
 * Runs the iteration repeatedly (its outputs are rewritten with the same
 * values) and synchronises.  cache_path (nullable, host text file): a
 * result for the same device and shape is read from it instead of timing,
 * and a new result is appended; *from_cache (nullable) tells which. */
ta_status ta_tune(ta_ctx *ctx, const ta_iteration *it, const char *cache_path, int32_t reps, void *stream,
                  int32_t *from_cache);

/* ---- Training of the learned predictor (an addition to the paper's
 * method, off the per-exchange path).  The network is the one
 * ta_predictor_load describes; training keeps fp32 parameters
 * theta[5252] = W1 (64x12 row-major), b1[64], W2 (64x64), b2[64], W3 (4x64),
 * b3[4], and its forward pass runs the integer network on the rounded
 * parameters (round half to even; weights clamped to [-128,127], biases to
 * +-2^24).  Loss: mean over windows of sum_k |o_k / 2^r3 - t_k|, o the
 * unrounded integer output, t the true move in quanta of 2^-12 um.
 * Backward: straight-through over every rounding, zero gradient where a
 * hidden pre-activation lies outside [0,127]. ---- */

/* Window tap: while set, every ta_delta_encode with a predictor on this
 * context also writes, for each slot it predicts (matched, >= 6 words,
 * history >= 1), that slot's 12 inputs to in_out[12 i ..] (device int32) and
 * the true move of words 2..5, (C - R) * 2^12 rounded to float32, to
 * tgt_out[4 i ..] (device float32).  *count (device uint64, zeroed by the
 * caller) advances by every window with finite targets; windows at i >= cap
 * are dropped, so *count > cap reports the overflow.  Window order is
 * unspecified.  in_out == NULL switches the tap off. */
ta_status ta_set_window_tap(ta_ctx *ctx, int32_t *in_out, float *tgt_out, int64_t cap, uint64_t *count);

typedef struct ta_trainer ta_trainer;
/* init: host float[5252]; shifts r1..r3 <= 24 and cell > 0 are written into
 * exported blobs.  Allocates the trainer's device state (parameters, Adam
 * moments, per-block gradient partials) on the context's device. */
ta_status ta_trainer_create(ta_ctx *ctx, const float *init, uint32_t r1, uint32_t r2, uint32_t r3, double cell,
                            ta_trainer **out);
void ta_trainer_free(ta_trainer *t);
/* Gradient of the loss at the current parameters over n windows (in:
 * device int32[n][12], tgt: device float32[n][4]).  grad_out (nullable,
 * device float32[5253]) receives the gradient and, last, the loss.  The sum
 * over windows runs in a fixed order: the result is deterministic. */
ta_status ta_trainer_grad(ta_ctx *ctx, ta_trainer *t, const int32_t *in, const float *tgt, int64_t n,
                          float *grad_out, void *stream);
/* One Adam step (bias-corrected, parameters clamped to the representable
 * ranges) on the gradient over n windows. */
ta_status ta_trainer_step(ta_ctx *ctx, ta_trainer *t, const int32_t *in, const float *tgt, int64_t n, float lr,
                          float beta1, float beta2, float eps, void *stream);
/* Copy the fp32 parameters to host float[5252] (synchronises the device). */
ta_status ta_trainer_params(ta_trainer *t, float *host_out);
/* Write the rounded parameters as a predictor blob (host, len == 5672) that
 * ta_predictor_load accepts (synchronises the device). */
ta_status ta_trainer_export(ta_trainer *t, void *blob, size_t len);

#ifdef __cplusplus
}
#endif
#endif
