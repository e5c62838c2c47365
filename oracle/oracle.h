/*
 * oracle.h -- plain CPU reference of the aura exchange.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only code that may load this library.  It shares no
 * source, header, table or helper with the GPU library; both implement the
 * byte formats from their written definition.
 *
 * Every function works on host memory, one segment (one neighbour message) at
 * a time, with plain loops.  Return values: 0 ok, 1 invalid input, 2 output
 * capacity too small, 3 corrupt encoding, 4 encoding made against another
 * reference.
 */
#ifndef TA_ORACLE_H
#define TA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_INVALID = 1, ORC_CAPACITY = 2, ORC_CORRUPT = 3, ORC_REF_MISMATCH = 4 };

typedef struct {
  int64_t n;
  const uint64_t *uid;
  const uint16_t *cls;
  const uint16_t *nb;
  const double *f64;
  int64_t f64_stride;
  const int32_t *i32;
  int64_t i32_stride;
  const int64_t *beh_off;
  const uint8_t *beh;
} orc_agents;

/* Integer MLP 12 -> 64 -> 64 -> 4 used as the position/diameter predictor. */
typedef struct {
  int8_t w1[64 * 12];
  int8_t w2[64 * 64];
  int8_t w3[4 * 64];
  int32_t b1[64];
  int32_t b2[64];
  int32_t b3[4];
  uint8_t r1, r2, r3;
  double cell;
} orc_mlp;

/* Per reference slot: h1[4*j..] words 2..5 of the record one exchange before
 * the reference, h2 two exchanges before, hlen how many of them exist. */
typedef struct {
  uint64_t *h1;
  uint64_t *h2;
  uint8_t *hlen;
} orc_hist;

/* Aura selection (Sec. 2.1).  Partitions [part_off[p], part_off[p+1]) of the
 * store with boxes[6p..6p+5] = lo0 lo1 lo2 hi0 hi1 hi2.  ndirs is 6 or 26.
 * Writes idx (store indices, CSR by partition, direction, store index) and
 * seg_off[P*ndirs+1]. */
int orc_select_aura(int64_t P, const int64_t *part_off, const double *f64, int64_t f64_stride,
                    const double *boxes, double w, int ndirs, int32_t *idx, int64_t idx_cap,
                    int64_t *seg_off);

/* Migrant selection (Sec. 2.1, "Agent Migration"): per partition and each of
 * the 26 directions (aura order), the agents whose position lies outside
 * their box on exactly that direction's side of each axis (x < lo: -1,
 * x >= hi: +1, else 0).  Same output layout as orc_select_aura. */
int orc_select_migrants(int64_t P, const int64_t *part_off, const double *f64, int64_t f64_stride,
                        const double *boxes, int32_t *idx, int64_t idx_cap, int64_t *seg_off);

/* TA IO serialization of every segment into one buffer (Sec. 2.2.1).
 * msg_off[nseg+1] receives the byte offset of each message. */
int orc_serialize(const orc_agents *a, int n_classes, const uint16_t *n_f64, const uint16_t *n_i32,
                  const int32_t *idx, const int64_t *seg_off, int64_t nseg, uint8_t *out, int64_t cap,
                  int64_t *msg_off);

/* Full validation of one TAM1 message (header, size identity, canonical
 * offsets, record sizes >= 2 words, non-zero uids); returns n and rec_words. */
int orc_view(const uint8_t *msg, int64_t len, int64_t *n, int64_t *rec_words);

/* Parse a predictor weight blob. */
int orc_mlp_parse(const uint8_t *blob, int64_t len, orc_mlp *out);
/* Integer forward pass of the predictor. */
void orc_mlp_forward(const orc_mlp *m, const int32_t in[12], int32_t q[4]);

/* Delta encoding of cur against ref (Sec. 2.3).  mlp == NULL: plain mode.
 * hin/hout may be NULL when mlp is NULL.  *mode_used is 0 (plain), 1
 * (learned) or 2 (mixed).  op: the difference operator, 0 XOR, 1 byte-wise
 * subtraction modulo 256. */
int orc_delta_encode(const uint8_t *cur, int64_t cur_len, const uint8_t *ref, int64_t ref_len,
                     const orc_mlp *mlp, const orc_hist *hin, orc_hist *hout, uint8_t *out,
                     int64_t cap, int64_t *out_len, uint8_t *newref, int64_t newref_cap,
                     int64_t *newref_len, int *mode_used, int op);

/* Decoding against the same reference (Sec. 2.3) with the receiver's
 * operator op; an encoding made with another operator is ORC_INVALID. */
int orc_delta_decode(const uint8_t *enc, int64_t enc_len, const uint8_t *ref, int64_t ref_len,
                     const orc_mlp *mlp, const orc_hist *hin, orc_hist *hout, uint8_t *out,
                     int64_t cap, int64_t *out_len, int op);

/* The 12 predictor inputs of every slot of ref (for training data and tests):
 * in[12*j..], and whether slot j is predicted at all (pred[j]). */
int orc_predictor_inputs(const uint8_t *ref, int64_t ref_len, const orc_hist *h, double cell,
                         int32_t *in, uint8_t *pred);

/* Mutable agent store with room for cap agents and beh_cap behaviour bytes. */
typedef struct {
  int64_t cap;
  uint64_t *uid;
  uint16_t *cls;
  uint16_t *nb;
  double *f64;
  int64_t f64_stride;
  int32_t *i32;
  int64_t i32_stride;
  int64_t *beh_off;
  uint8_t *beh;
  int64_t beh_cap;
} orc_store;

/* The store after one migration exchange (Sec. 2.1): per partition q, its
 * agents that stay inside box q, then the records of the messages s with
 * dest[s] == q (dest < 0: skipped) unpacked into the columns.  sizes[0..1] =
 * agents and behaviour bytes of the result, part_off_out[P+1] its partition
 * starts (both also on ORC_CAPACITY). */
int orc_migrate_apply(const orc_agents *in, int64_t P, const int64_t *part_off, const double *boxes,
                      int n_classes, const uint16_t *n_f64, const uint16_t *n_i32, int nf_cols, int ni_cols,
                      const uint8_t *msgs, int64_t msgs_len, const int64_t *msg_off, int64_t nseg,
                      const int32_t *dest, orc_store *out, int64_t *part_off_out, int64_t *sizes);

/* Growth of viewed records (Sec. 2.2.1 "Mutability"): record rec[k] of
 * message seg[k] ((seg, rec) strictly ascending) moves to the arena after the
 * last message (bytes [msg_off[nseg], cap), *arena_used of them taken) with
 * room for words[k] words (>= its size): words copied, the rest zero, header
 * size updated, offset redirected.  cap <= 2^35. */
int orc_view_grow(uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg, const int32_t *seg,
                  const uint32_t *rec, const uint32_t *words, int64_t n, int64_t *arena_used);

/* Canonical copies of messages whose offsets may be redirected (records in
 * order, offsets the running sum of sizes). */
int orc_view_compact(const uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg, uint8_t *out,
                     int64_t out_cap, int64_t *out_off);

#ifdef __cplusplus
}
#endif
#endif
