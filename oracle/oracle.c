/*
 * oracle.c -- plain CPU reference of the aura exchange.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Plain loops, one
 * message at a time, no blocking or fusion; libc qsort/bsearch are the only
 * library steps.  Formats (TAM1 message, TAD1 delta encoding, TAP1 predictor
 * blob) are implemented here from their written definition, independently of
 * the GPU library.
 *
 * Paper passages followed:
 *  - aura selection: Sec. 2.1 "Aura Update" (agents within the interaction
 *    distance of a neighbouring partition box are copied to that neighbour;
 *    the aura is narrower than the partition box);
 *  - serialization: Sec. 2.2.1 "Serialization" (in-order traversal copying
 *    each memory block, the vtable pointer replaced by a class id, pointers
 *    replaced by markers -- here by offsets) and "Deserialization" (one pass,
 *    no allocation besides the receive buffer);
 *  - delta encoding: Sec. 2.3 (agents found in both message and reference are
 *    moved to the reference position, vanished ones leave an empty
 *    placeholder, new ones are appended; the difference against the
 *    reference is written for matched agents; the receiver restores the
 *    message from the reference and removes the placeholders, without
 *    restoring the original order).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TAM1_MAGIC 0x314D4154u /* "TAM1" */
#define TAD1_MAGIC 0x31444154u /* "TAD1" */
#define TAP1_MAGIC 0x31504154u /* "TAP1" */

/* ---- little-endian field access (host is little-endian) ------------------ */
static uint64_t get64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint32_t get32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint16_t get16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
static void put64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void put32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }
static double as_f64(uint64_t bits) { double d; memcpy(&d, &bits, 8); return d; }
static uint64_t f64_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static int64_t round8(int64_t b) { return (b + 7) / 8 * 8; }

/* ======================================================================== */
/* Aura selection                                                            */
/* ======================================================================== */

/* Neighbour direction (dx,dy,dz) in {-1,0,1}^3 \ {0}; code = (dx+1)+3(dy+1)+9(dz+1).
 * Face mode uses the six codes with exactly one nonzero component. */
static int direction_codes(int ndirs, int *codes) {
  int n = 0;
  for (int c = 0; c < 27; ++c) {
    if (c == 13) continue;
    int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = c / 9 - 1;
    int nonzero = (dx != 0) + (dy != 0) + (dz != 0);
    if (ndirs == 26 || nonzero == 1) codes[n++] = c;
  }
  return n;
}

int orc_select_aura(int64_t P, const int64_t *part_off, const double *f64, int64_t f64_stride,
                    const double *boxes, double w, int ndirs, int32_t *idx, int64_t idx_cap,
                    int64_t *seg_off) {
  int codes[26];
  if (ndirs != 6 && ndirs != 26) return ORC_INVALID;
  direction_codes(ndirs, codes);
  int64_t count = 0;
  for (int64_t p = 0; p < P; ++p) {
    const double *lo = boxes + 6 * p, *hi = boxes + 6 * p + 3;
    /* an agent is within w of the lower (upper) neighbour along axis a when
     * x < lo+w (x >= hi-w); each threshold is one fp64 operation */
    double thr_lo[3], thr_hi[3];
    for (int a = 0; a < 3; ++a) {
      thr_lo[a] = lo[a] + w;
      thr_hi[a] = hi[a] - w;
    }
    for (int k = 0; k < ndirs; ++k) {
      int d[3] = {codes[k] % 3 - 1, (codes[k] / 3) % 3 - 1, codes[k] / 9 - 1};
      seg_off[p * ndirs + k] = count;
      for (int64_t i = part_off[p]; i < part_off[p + 1]; ++i) {
        int member = 1;
        for (int a = 0; a < 3; ++a) {
          double x = f64[a * f64_stride + i];
          if (d[a] == -1 && !(x < thr_lo[a])) member = 0;
          if (d[a] == +1 && !(x >= thr_hi[a])) member = 0;
        }
        if (member) {
          if (count < idx_cap) idx[count] = (int32_t)i;
          ++count;
        }
      }
    }
  }
  seg_off[P * ndirs] = count;
  return count > idx_cap ? ORC_CAPACITY : ORC_OK;
}

/* ======================================================================== */
/* Migrant selection (Sec. 2.1, "Agent Migration")                           */
/* ======================================================================== */
/*
 * An agent of partition p whose position lies outside box p belongs to the
 * rank that owns the neighbouring box it moved into.  Per axis its offset is
 * -1 when x < lo, +1 when x >= hi and 0 otherwise; the triple of offsets is
 * one of the 26 directions (in the 26-direction order of the aura
 * selection), or (0,0,0) for an agent that stays.
 */
static int axis_offset(double x, double lo, double hi) {
  if (x < lo) return -1;
  if (x >= hi) return +1;
  return 0;
}

int orc_select_migrants(int64_t P, const int64_t *part_off, const double *f64, int64_t f64_stride,
                        const double *boxes, int32_t *idx, int64_t idx_cap, int64_t *seg_off) {
  int codes[26];
  direction_codes(26, codes);
  int64_t count = 0;
  for (int64_t p = 0; p < P; ++p) {
    const double *lo = boxes + 6 * p, *hi = boxes + 6 * p + 3;
    for (int k = 0; k < 26; ++k) {
      int d[3] = {codes[k] % 3 - 1, (codes[k] / 3) % 3 - 1, codes[k] / 9 - 1};
      seg_off[p * 26 + k] = count;
      for (int64_t i = part_off[p]; i < part_off[p + 1]; ++i) {
        int same = 1;
        for (int a = 0; a < 3; ++a)
          if (axis_offset(f64[a * f64_stride + i], lo[a], hi[a]) != d[a]) same = 0;
        if (same) {
          if (count < idx_cap) idx[count] = (int32_t)i;
          ++count;
        }
      }
    }
  }
  seg_off[P * 26] = count;
  return count > idx_cap ? ORC_CAPACITY : ORC_OK;
}

/* ======================================================================== */
/* Serialization into TAM1 messages                                          */
/* ======================================================================== */
/*
 * TAM1 message: 32-byte header {u32 magic "TAM1", u16 version 1, u16 flags 0,
 * u32 n, u32 0, u64 rec_words, u64 0}; n u32 word offsets (record i starts at
 * word off[i] of the record area; canonical = running sum of record sizes),
 * zero-padded to 8 bytes; the record area of rec_words 8-byte words.
 *
 * Record: word 0 uid; word 1 = u16 class | u16 behaviour count << 16 |
 * u32 record words << 32; the class's fp64 fields; its int32 attributes, with
 * a zero pad to 8 bytes; then the agent's behaviour blocks verbatim (each
 * u32 class, u32 payload bytes, payload).
 */
static int64_t record_words(const orc_agents *a, int n_classes, const uint16_t *n_f64,
                            const uint16_t *n_i32, int64_t i, int *err) {
  if (i < 0 || i >= a->n) { *err = 1; return 0; }
  uint16_t c = a->cls[i];
  if (c >= n_classes) { *err = 1; return 0; }
  int64_t beh_bytes = a->beh_off[i + 1] - a->beh_off[i];
  if (beh_bytes < 0 || beh_bytes % 8 != 0 || a->beh_off[i] % 8 != 0) { *err = 1; return 0; }
  return 2 + n_f64[c] + (n_i32[c] + 1) / 2 + beh_bytes / 8;
}

int orc_serialize(const orc_agents *a, int n_classes, const uint16_t *n_f64, const uint16_t *n_i32,
                  const int32_t *idx, const int64_t *seg_off, int64_t nseg, uint8_t *out, int64_t cap,
                  int64_t *msg_off) {
  int64_t pos = 0;
  int err = 0, overflow = 0;
  for (int64_t s = 0; s < nseg; ++s) {
    int64_t first = seg_off[s], n = seg_off[s + 1] - seg_off[s];
    int64_t rec_words = 0;
    for (int64_t r = 0; r < n; ++r) rec_words += record_words(a, n_classes, n_f64, n_i32, idx[first + r], &err);
    if (err) return ORC_INVALID;
    int64_t size = 32 + 8 * ((n + 1) / 2) + 8 * rec_words;
    msg_off[s] = pos;
    if (pos + size > cap) {
      overflow = 1;
      pos += size;
      continue;
    }
    uint8_t *m = out + pos;
    memset(m, 0, (size_t)size);
    put32(m + 0, TAM1_MAGIC);
    put16(m + 4, 1);
    put16(m + 6, 0);
    put32(m + 8, (uint32_t)n);
    put64(m + 16, (uint64_t)rec_words);
    uint8_t *offs = m + 32;
    uint8_t *recs = m + 32 + 8 * ((n + 1) / 2);
    int64_t at = 0; /* word position of the next record */
    for (int64_t r = 0; r < n; ++r) {
      int64_t i = idx[first + r];
      uint16_t c = a->cls[i];
      int64_t words = record_words(a, n_classes, n_f64, n_i32, i, &err);
      put32(offs + 4 * r, (uint32_t)at);
      uint8_t *rec = recs + 8 * at;
      put64(rec, a->uid[i]);
      put64(rec + 8, (uint64_t)c | ((uint64_t)a->nb[i] << 16) | ((uint64_t)words << 32));
      uint8_t *f = rec + 16;
      for (int k = 0; k < n_f64[c]; ++k) {
        memcpy(f, &a->f64[k * a->f64_stride + i], 8);
        f += 8;
      }
      for (int k = 0; k < n_i32[c]; ++k) {
        memcpy(f, &a->i32[k * a->i32_stride + i], 4);
        f += 4;
      }
      if (n_i32[c] % 2) f += 4; /* zero pad */
      int64_t bb = a->beh_off[i + 1] - a->beh_off[i];
      memcpy(f, a->beh + a->beh_off[i], (size_t)bb);
      at += words;
    }
    pos += size;
  }
  msg_off[nseg] = pos;
  return overflow ? ORC_CAPACITY : ORC_OK;
}

/* ======================================================================== */
/* View: full validation of a TAM1 message                                   */
/* ======================================================================== */
/* Header and size identity, the offsets as the running sum of record sizes
 * (at least two words each), and a non-zero uid in every record: uids name
 * one agent each (Sec. 2.5) and the record format reserves zero. */
int orc_view(const uint8_t *msg, int64_t len, int64_t *n_out, int64_t *rw_out) {
  if (len < 32) return ORC_INVALID;
  if (get32(msg) != TAM1_MAGIC || get16(msg + 4) != 1 || get16(msg + 6) != 0) return ORC_INVALID;
  if (get32(msg + 12) != 0 || get64(msg + 24) != 0) return ORC_INVALID;
  int64_t n = get32(msg + 8);
  uint64_t rw = get64(msg + 16);
  if (n > len / 4 || rw > (uint64_t)len / 8) return ORC_INVALID;
  if (rw < 2 * (uint64_t)n) return ORC_INVALID; /* records have at least 2 words */
  int64_t table = 8 * ((n + 1) / 2);
  if (32 + table + 8 * (int64_t)rw != len) return ORC_INVALID;
  if (n % 2 && get32(msg + 32 + 4 * n) != 0) return ORC_INVALID;
  const uint8_t *recs = msg + 32 + table;
  uint64_t expect = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (get32(msg + 32 + 4 * i) != expect) return ORC_INVALID;
    if (expect + 2 > rw) return ORC_INVALID;
    uint64_t words = get64(recs + 8 * expect + 8) >> 32;
    if (words < 2 || words > rw - expect) return ORC_INVALID;
    if (get64(recs + 8 * expect) == 0) return ORC_INVALID;
    expect += words;
  }
  if (expect != rw) return ORC_INVALID;
  *n_out = n;
  *rw_out = (int64_t)rw;
  return ORC_OK;
}

typedef struct {
  int64_t n, rec_words;
  const uint8_t *recs;
  const uint8_t *offs;
} msg_t;

static int open_msg(const uint8_t *m, int64_t len, msg_t *out) {
  int st = orc_view(m, len, &out->n, &out->rec_words);
  if (st) return st;
  out->offs = m + 32;
  out->recs = m + 32 + 8 * ((out->n + 1) / 2);
  return ORC_OK;
}
static const uint8_t *record(const msg_t *m, int64_t i) { return m->recs + 8 * (int64_t)get32(m->offs + 4 * i); }
static int64_t rec_words_of(const uint8_t *rec) { return (int64_t)(get64(rec + 8) >> 32); }

/* ======================================================================== */
/* Predictor                                                                 */
/* ======================================================================== */
/*
 * TAP1 blob: u32 magic "TAP1", u32 version 1, int8 W1[64][12], int8 W2[64][64],
 * int8 W3[4][64], int32 b1[64], int32 b2[64], int32 b3[4], u8 r1, r2, r3,
 * 5 zero bytes, f64 cell.  Total 5672 bytes.  |b| <= 2^24, r <= 24, cell > 0.
 */
int orc_mlp_parse(const uint8_t *blob, int64_t len, orc_mlp *m) {
  if (len != 5672) return ORC_INVALID;
  if (get32(blob) != TAP1_MAGIC || get32(blob + 4) != 1) return ORC_INVALID;
  const uint8_t *p = blob + 8;
  memcpy(m->w1, p, 768); p += 768;
  memcpy(m->w2, p, 4096); p += 4096;
  memcpy(m->w3, p, 256); p += 256;
  for (int i = 0; i < 64; ++i) m->b1[i] = (int32_t)get32(p + 4 * i);
  p += 256;
  for (int i = 0; i < 64; ++i) m->b2[i] = (int32_t)get32(p + 4 * i);
  p += 256;
  for (int i = 0; i < 4; ++i) m->b3[i] = (int32_t)get32(p + 4 * i);
  p += 16;
  m->r1 = p[0]; m->r2 = p[1]; m->r3 = p[2];
  p += 8;
  m->cell = as_f64(get64(p));
  for (int i = 0; i < 64; ++i)
    if (llabs((long long)m->b1[i]) > (1 << 24) || llabs((long long)m->b2[i]) > (1 << 24)) return ORC_INVALID;
  for (int i = 0; i < 4; ++i)
    if (llabs((long long)m->b3[i]) > (1 << 24)) return ORC_INVALID;
  if (m->r1 > 24 || m->r2 > 24 || m->r3 > 24) return ORC_INVALID;
  if (!(m->cell > 0) || !isfinite(m->cell)) return ORC_INVALID;
  return ORC_OK;
}

/* floor((v + 2^(r-1)) / 2^r): requantisation with round-half-up. */
static int64_t requant(int64_t v, int r) {
  int64_t half = r > 0 ? ((int64_t)1 << (r - 1)) : 0;
  int64_t t = v + half;
  int64_t d = (int64_t)1 << r;
  int64_t q = t / d;
  if (t % d != 0 && t < 0) q -= 1; /* floor for negatives */
  return q;
}
static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

void orc_mlp_forward(const orc_mlp *m, const int32_t in[12], int32_t q[4]) {
  int64_t h1[64], h2[64];
  for (int o = 0; o < 64; ++o) {
    int64_t acc = m->b1[o];
    for (int i = 0; i < 12; ++i) acc += (int64_t)m->w1[o * 12 + i] * in[i];
    h1[o] = clampi(requant(acc, m->r1), 0, 127);
  }
  for (int o = 0; o < 64; ++o) {
    int64_t acc = m->b2[o];
    for (int i = 0; i < 64; ++i) acc += (int64_t)m->w2[o * 64 + i] * h1[i];
    h2[o] = clampi(requant(acc, m->r2), 0, 127);
  }
  for (int o = 0; o < 4; ++o) {
    int64_t acc = m->b3[o];
    for (int i = 0; i < 64; ++i) acc += (int64_t)m->w3[o * 64 + i] * h2[i];
    q[o] = (int32_t)clampi(requant(acc, m->r3), -(1 << 24), 1 << 24);
  }
}

/* clamp(round-half-even(v * 2^12), -32768, 32767); NaN -> 0 */
static int32_t quantise(double v) {
  double t = v * 4096.0;
  if (t != t) return 0;
  if (t >= 32767.0) return 32767;
  if (t <= -32768.0) return -32768;
  return (int32_t)nearbyint(t);
}

typedef struct { uint64_t key; int64_t j; } cellkey_t;
static int cmp_cellkey(const void *a, const void *b) {
  const cellkey_t *x = a, *y = b;
  return x->key < y->key ? -1 : (x->key > y->key ? 1 : (x->j < y->j ? -1 : x->j > y->j));
}

/* Number of reference agents sharing the grid cell floor(x/cell) of each slot
 * (records of at least 5 words; the cell coordinates must lie within
 * +-2^20), clamped to 127; 0 for slots without a valid cell. */
static void neighbour_counts(const msg_t *R, double cell, int32_t *nbr) {
  cellkey_t *keys = malloc(sizeof(cellkey_t) * (size_t)(R->n ? R->n : 1));
  int64_t nk = 0;
  for (int64_t j = 0; j < R->n; ++j) {
    nbr[j] = 0;
    const uint8_t *rec = record(R, j);
    if (rec_words_of(rec) < 5) continue;
    int64_t c[3];
    int ok = 1;
    for (int a = 0; a < 3; ++a) {
      double f = floor(as_f64(get64(rec + 16 + 8 * a)) / cell);
      if (!(f > -1048576.0 && f < 1048576.0)) ok = 0;
      else c[a] = (int64_t)f;
    }
    if (!ok) continue;
    uint64_t key = ((uint64_t)(c[0] + 1048576) << 42) | ((uint64_t)(c[1] + 1048576) << 21) |
                   (uint64_t)(c[2] + 1048576);
    keys[nk].key = key;
    keys[nk].j = j;
    ++nk;
  }
  qsort(keys, (size_t)nk, sizeof(cellkey_t), cmp_cellkey);
  for (int64_t s = 0; s < nk;) {
    int64_t e = s;
    while (e < nk && keys[e].key == keys[s].key) ++e;
    int32_t cnt = (int32_t)((e - s) > 127 ? 127 : (e - s));
    for (int64_t t = s; t < e; ++t) nbr[keys[t].j] = cnt;
    s = e;
  }
  free(keys);
}

/* Inputs of slot j: q(R-h1) (4), q(h1-h2) (4), neighbour count, behaviour
 * count, class, history length.  Returns 1 when the slot is predicted at all
 * (history present and a record of at least 6 words). */
static int slot_inputs(const msg_t *R, int64_t j, const orc_hist *h, const int32_t *nbr, int32_t in[12]) {
  const uint8_t *rec = record(R, j);
  int hl = h->hlen[j];
  if (hl < 1 || rec_words_of(rec) < 6) return 0;
  uint64_t hdr = get64(rec + 8);
  for (int k = 0; k < 4; ++k) {
    double r = as_f64(get64(rec + 16 + 8 * k));
    double a1 = as_f64(h->h1[4 * j + k]);
    double a2 = as_f64(h->h2[4 * j + k]);
    in[k] = quantise(r - a1);
    in[4 + k] = hl >= 2 ? quantise(a1 - a2) : 0;
  }
  in[8] = nbr[j];
  in[9] = (int32_t)((hdr >> 16) & 0xFFFF);
  in[10] = (int32_t)(hdr & 0xFFFF);
  in[11] = hl;
  return 1;
}

int orc_predictor_inputs(const uint8_t *ref, int64_t ref_len, const orc_hist *h, double cell, int32_t *in,
                         uint8_t *pred) {
  msg_t R;
  int st = open_msg(ref, ref_len, &R);
  if (st) return st;
  int32_t *nbr = malloc(sizeof(int32_t) * (size_t)(R.n ? R.n : 1));
  neighbour_counts(&R, cell, nbr);
  for (int64_t j = 0; j < R.n; ++j) {
    memset(in + 12 * j, 0, 12 * sizeof(int32_t));
    pred[j] = (uint8_t)slot_inputs(&R, j, h, nbr, in + 12 * j);
  }
  free(nbr);
  return ORC_OK;
}

/* X[j]: the words the residual of slot j is taken against.  Plain: the
 * reference record.  Learned: the reference record with words 2..5 (fields
 * x, y, z, diameter) replaced by R + q * 2^-12 for predicted slots. */
static void predicted_record(const msg_t *R, int64_t j, const orc_mlp *m, const orc_hist *h, const int32_t *nbr,
                             uint64_t *X) {
  const uint8_t *rec = record(R, j);
  int64_t words = rec_words_of(rec);
  for (int64_t k = 0; k < words; ++k) X[k] = get64(rec + 8 * k);
  if (!m) return;
  int32_t in[12], q[4];
  if (!slot_inputs(R, j, h, nbr, in)) return;
  orc_mlp_forward(m, in, q);
  for (int k = 0; k < 4; ++k) {
    double r = as_f64(X[2 + k]);
    if (q[k] != 0 && isfinite(r)) X[2 + k] = f64_bits(r + ldexp((double)q[k], -12));
  }
}

/* ======================================================================== */
/* Zero-block packer                                                         */
/* ======================================================================== */
/*
 * The residual D (W words) is cut into groups of 64 words.  Group g has a
 * bitmap word (bit k set when D[64g+k] != 0) and a data block: one length
 * nibble per nonzero word (number of low-order bytes up to the highest
 * nonzero byte, 1..8; two per byte, low nibble first), then those bytes of
 * every nonzero word in order, zero-padded to a multiple of 8 bytes.  A group
 * without nonzero words has an empty block.  The block size / 8 is kept in a
 * byte table.
 */
static int sig_len(uint64_t w) {
  int len = 8;
  while (len > 0 && ((w >> (8 * (len - 1))) & 0xFF) == 0) --len;
  return len;
}

static int64_t group_block_bytes(const uint64_t *D, int64_t W, int64_t g) {
  int64_t popc = 0, sig = 0;
  for (int64_t q = 64 * g; q < W && q < 64 * g + 64; ++q)
    if (D[q]) { ++popc; sig += sig_len(D[q]); }
  return round8((popc + 1) / 2 + sig);
}

static int64_t packed_var_bytes(const uint64_t *D, int64_t W) {
  int64_t total = 0;
  for (int64_t g = 0; g < (W + 63) / 64; ++g) total += group_block_bytes(D, W, g);
  return total;
}

/* ======================================================================== */
/* Delta encoding                                                            */
/* ======================================================================== */
/*
 * TAD1 encoding of C against R:
 *   64-byte header {u32 magic "TAD1", u16 version 1, u8 mode (0 plain,
 *   1 learned, 2 mixed: per group, bit 7 of its size byte set = learned),
 *   u8 packer 1, u32 n_ref, u32 n_match, u32 n_new, u32 0,
 *   u64 ref_words, u64 XOR of all reference uids, u64 W, u64 new_words,
 *   u64 var_bytes};
 *   presence bitmap: ceil(n_ref/64) u64, bit j = reference slot j matched;
 *   word bitmap: ceil(W/64) u64;
 *   group block sizes: ceil(W/64) u8 (bytes / 8), zero-padded to 8 bytes;
 *   new record sizes: n_new u32 (words), zero-padded to 8 bytes;
 *   new records verbatim (new_words words);
 *   group blocks (var_bytes).
 * Matched: same uid and same header word (class, behaviour count, size).
 * C' = matched current records in reference order, then new ones in current
 * order; it is the next reference of both sides.
 */
typedef struct { uint64_t uid; int64_t i; } uidpos_t;
static int cmp_uidpos(const void *a, const void *b) {
  const uidpos_t *x = a, *y = b;
  return x->uid < y->uid ? -1 : (x->uid > y->uid);
}

static int sorted_uids(const msg_t *M, uidpos_t **out) {
  uidpos_t *u = malloc(sizeof(uidpos_t) * (size_t)(M->n ? M->n : 1));
  for (int64_t i = 0; i < M->n; ++i) {
    u[i].uid = get64(record(M, i));
    u[i].i = i;
    if (u[i].uid == 0) { free(u); return ORC_INVALID; }
  }
  qsort(u, (size_t)M->n, sizeof(uidpos_t), cmp_uidpos);
  for (int64_t i = 1; i < M->n; ++i)
    if (u[i].uid == u[i - 1].uid) { free(u); return ORC_INVALID; }
  *out = u;
  return ORC_OK;
}

static void write_history(const msg_t *R, int64_t n_out, const int64_t *slot_of, const orc_hist *hin,
                          orc_hist *hout) {
  /* slot_of[k] = reference slot of C' record k, or -1 for a new record */
  for (int64_t k = 0; k < n_out; ++k) {
    int64_t j = slot_of[k];
    if (j < 0) {
      for (int t = 0; t < 4; ++t) hout->h1[4 * k + t] = hout->h2[4 * k + t] = 0;
      hout->hlen[k] = 0;
      continue;
    }
    const uint8_t *rec = record(R, j);
    int has = rec_words_of(rec) >= 6;
    for (int t = 0; t < 4; ++t) {
      hout->h2[4 * k + t] = hin ? hin->h1[4 * j + t] : 0;
      hout->h1[4 * k + t] = has ? get64(rec + 16 + 8 * t) : 0;
    }
    int hl = hin ? hin->hlen[j] : 0;
    hout->hlen[k] = (uint8_t)(hl + 1 > 2 ? 2 : hl + 1);
  }
}

/* The difference operator of Sec. 2.3, which the paper leaves open.
 * op 0: XOR of the two 8-byte words.  op 1: each of the eight bytes
 * subtracted on its own, modulo 256 (no borrow between bytes); inverting it
 * adds the bytes back modulo 256. */
static uint64_t diff_word(uint64_t c, uint64_t x, int op) {
  if (op == 0) return c ^ x;
  uint64_t d = 0;
  for (int b = 0; b < 8; ++b) {
    uint8_t cb = (uint8_t)(c >> (8 * b)), xb = (uint8_t)(x >> (8 * b));
    d |= (uint64_t)(uint8_t)(cb - xb) << (8 * b);
  }
  return d;
}

static uint64_t undiff_word(uint64_t d, uint64_t x, int op) {
  if (op == 0) return d ^ x;
  uint64_t c = 0;
  for (int b = 0; b < 8; ++b) {
    uint8_t db = (uint8_t)(d >> (8 * b)), xb = (uint8_t)(x >> (8 * b));
    c |= (uint64_t)(uint8_t)(db + xb) << (8 * b);
  }
  return c;
}

int orc_delta_encode(const uint8_t *cur, int64_t cur_len, const uint8_t *ref, int64_t ref_len, const orc_mlp *mlp,
                     const orc_hist *hin, orc_hist *hout, uint8_t *out, int64_t cap, int64_t *out_len,
                     uint8_t *newref, int64_t newref_cap, int64_t *newref_len, int *mode_used, int op) {
  msg_t C, R;
  if (op < 0 || op > 1) return ORC_INVALID;
  if (open_msg(cur, cur_len, &C) || open_msg(ref, ref_len, &R)) return ORC_INVALID;
  if (mlp && !hin) return ORC_INVALID;
  uidpos_t *cu = NULL, *ru = NULL;
  if (sorted_uids(&C, &cu)) return ORC_INVALID;
  if (sorted_uids(&R, &ru)) { free(cu); return ORC_INVALID; }
  free(ru);

  /* match: m[j] = current index of reference slot j, or -1 */
  int64_t *m = malloc(sizeof(int64_t) * (size_t)(R.n + 1));
  uint8_t *used = calloc((size_t)C.n + 1, 1);
  int64_t n_match = 0, W = 0;
  uint64_t fold = 0;
  for (int64_t j = 0; j < R.n; ++j) {
    const uint8_t *rj = record(&R, j);
    uidpos_t key = {get64(rj), 0};
    fold ^= key.uid;
    uidpos_t *hit = C.n ? bsearch(&key, cu, (size_t)C.n, sizeof(uidpos_t), cmp_uidpos) : NULL;
    m[j] = -1;
    if (hit && get64(record(&C, hit->i) + 8) == get64(rj + 8)) {
      m[j] = hit->i;
      used[hit->i] = 1;
      ++n_match;
      W += rec_words_of(rj);
    }
  }
  free(cu);
  int64_t n_new = 0, new_words = 0;
  for (int64_t i = 0; i < C.n; ++i)
    if (!used[i]) { ++n_new; new_words += rec_words_of(record(&C, i)); }

  /* residual of the matched records against X (plain, and learned if asked) */
  uint64_t *Dp = malloc(sizeof(uint64_t) * (size_t)(W + 1));
  uint64_t *Dl = mlp ? malloc(sizeof(uint64_t) * (size_t)(W + 1)) : NULL;
  uint64_t *X = malloc(sizeof(uint64_t) * (size_t)(R.rec_words + 1));
  int32_t *nbr = NULL;
  if (mlp) {
    nbr = malloc(sizeof(int32_t) * (size_t)(R.n + 1));
    neighbour_counts(&R, mlp->cell, nbr);
  }
  int64_t q = 0;
  for (int64_t j = 0; j < R.n; ++j) {
    if (m[j] < 0) continue;
    const uint8_t *rj = record(&R, j), *ci = record(&C, m[j]);
    int64_t words = rec_words_of(rj);
    if (mlp) predicted_record(&R, j, mlp, hin, nbr, X);
    for (int64_t k = 0; k < words; ++k) {
      Dp[q + k] = diff_word(get64(ci + 8 * k), get64(rj + 8 * k), op);
      if (mlp) Dl[q + k] = diff_word(get64(ci + 8 * k), X[k], op);
    }
    q += words;
  }
  free(nbr);
  free(X);
  int64_t var_plain = packed_var_bytes(Dp, W);
  int mode = 0;
  const uint64_t *D = Dp;
  int64_t var_bytes = var_plain;
  int64_t G = (W + 63) / 64;
  /* learned calls: per group the smaller of the two residuals (the learned
   * one only when strictly smaller); the segment is plain when that is no
   * smaller than the plain residual, learned when no smaller than the learned
   * one, and mixed (mode 2, a flag per group) otherwise */
  uint64_t *Dm = NULL;
  uint8_t *gl = NULL;
  if (mlp) {
    int64_t var_learned = packed_var_bytes(Dl, W), var_mixed = 0;
    Dm = malloc(sizeof(uint64_t) * (size_t)(W + 1));
    gl = calloc((size_t)G + 1, 1);
    for (int64_t g = 0; g < G; ++g) {
      int64_t bp = group_block_bytes(Dp, W, g), bl = group_block_bytes(Dl, W, g);
      gl[g] = bl < bp;
      var_mixed += gl[g] ? bl : bp;
      for (int64_t w = 64 * g; w < W && w < 64 * g + 64; ++w) Dm[w] = gl[g] ? Dl[w] : Dp[w];
    }
    if (var_mixed == var_plain) {
      mode = 0;
    } else if (var_mixed == var_learned) {
      mode = 1; D = Dl; var_bytes = var_learned;
    } else {
      mode = 2; D = Dm; var_bytes = var_mixed;
    }
  }

  int64_t sz_pres = 8 * ((R.n + 63) / 64), sz_bits = 8 * G, sz_gs = round8(G), sz_ns = round8(4 * n_new);
  int64_t total = 64 + sz_pres + sz_bits + sz_gs + sz_ns + 8 * new_words + var_bytes;
  int64_t n_out = n_match + n_new;
  int64_t newref_size = 32 + 8 * ((n_out + 1) / 2) + 8 * (W + new_words);
  *out_len = total;
  *newref_len = newref_size;
  *mode_used = mode;
  int st = ORC_OK;
  if (total > cap || newref_size > newref_cap) st = ORC_CAPACITY;

  if (st == ORC_OK) {
    memset(out, 0, (size_t)total);
    put32(out, TAD1_MAGIC);
    put16(out + 4, 1);
    out[6] = (uint8_t)mode;
    out[7] = 1;
    put32(out + 8, (uint32_t)R.n);
    put32(out + 12, (uint32_t)n_match);
    put32(out + 16, (uint32_t)n_new);
    put32(out + 20, (uint32_t)op);
    put64(out + 24, (uint64_t)R.rec_words);
    put64(out + 32, fold);
    put64(out + 40, (uint64_t)W);
    put64(out + 48, (uint64_t)new_words);
    put64(out + 56, (uint64_t)var_bytes);
    uint8_t *pres = out + 64, *bits = pres + sz_pres, *gs = bits + sz_bits, *ns = gs + sz_gs;
    uint8_t *nrec = ns + sz_ns, *var = nrec + 8 * new_words;
    for (int64_t j = 0; j < R.n; ++j)
      if (m[j] >= 0) pres[j / 8] |= (uint8_t)(1u << (j % 8));
    for (int64_t w = 0; w < W; ++w)
      if (D[w]) bits[w / 8] |= (uint8_t)(1u << (w % 8));
    int64_t at = 0;
    for (int64_t g = 0; g < G; ++g) {
      int64_t blk = group_block_bytes(D, W, g);
      gs[g] = (uint8_t)(blk / 8 | (mode == 2 && gl[g] ? 0x80 : 0));
      int64_t popc = 0;
      for (int64_t w = 64 * g; w < W && w < 64 * g + 64; ++w) popc += D[w] != 0;
      uint8_t *nib = var + at, *sig = var + at + (popc + 1) / 2;
      int64_t t = 0;
      for (int64_t w = 64 * g; w < W && w < 64 * g + 64; ++w) {
        if (!D[w]) continue;
        int len = sig_len(D[w]);
        nib[t / 2] |= (uint8_t)(t % 2 ? len << 4 : len);
        for (int b = 0; b < len; ++b) *sig++ = (uint8_t)(D[w] >> (8 * b));
        ++t;
      }
      at += blk;
    }
    int64_t r = 0, wpos = 0;
    for (int64_t i = 0; i < C.n; ++i) {
      if (used[i]) continue;
      const uint8_t *ci = record(&C, i);
      int64_t words = rec_words_of(ci);
      put32(ns + 4 * r, (uint32_t)words);
      memcpy(nrec + 8 * wpos, ci, (size_t)(8 * words));
      ++r;
      wpos += words;
    }

    /* C': matched in reference order, then new in current order */
    memset(newref, 0, (size_t)newref_size);
    put32(newref, TAM1_MAGIC);
    put16(newref + 4, 1);
    put32(newref + 8, (uint32_t)n_out);
    put64(newref + 16, (uint64_t)(W + new_words));
    uint8_t *offs = newref + 32, *recs = newref + 32 + 8 * ((n_out + 1) / 2);
    int64_t k = 0, wat = 0;
    int64_t *slot_of = malloc(sizeof(int64_t) * (size_t)(n_out + 1));
    for (int64_t j = 0; j < R.n; ++j) {
      if (m[j] < 0) continue;
      const uint8_t *ci = record(&C, m[j]);
      int64_t words = rec_words_of(ci);
      put32(offs + 4 * k, (uint32_t)wat);
      memcpy(recs + 8 * wat, ci, (size_t)(8 * words));
      slot_of[k++] = j;
      wat += words;
    }
    for (int64_t i = 0; i < C.n; ++i) {
      if (used[i]) continue;
      const uint8_t *ci = record(&C, i);
      int64_t words = rec_words_of(ci);
      put32(offs + 4 * k, (uint32_t)wat);
      memcpy(recs + 8 * wat, ci, (size_t)(8 * words));
      slot_of[k++] = -1;
      wat += words;
    }
    if (hout) write_history(&R, n_out, slot_of, hin, hout);
    free(slot_of);
  }
  free(m);
  free(used);
  free(Dp);
  free(Dl);
  free(Dm);
  free(gl);
  return st;
}

/* ======================================================================== */
/* Delta decoding                                                            */
/* ======================================================================== */
int orc_delta_decode(const uint8_t *enc, int64_t enc_len, const uint8_t *ref, int64_t ref_len, const orc_mlp *mlp,
                     const orc_hist *hin, orc_hist *hout, uint8_t *out, int64_t cap, int64_t *out_len, int op) {
  msg_t R;
  if (enc_len < 64) return ORC_CORRUPT;
  if (get32(enc) != TAD1_MAGIC || get16(enc + 4) != 1 || enc[7] != 1 || enc[6] > 2 || get32(enc + 20) > 1)
    return ORC_CORRUPT;
  int mode = enc[6];
  /* both ends of a pair agree on the operator, as on the predictor */
  if ((mode >= 1 && (!mlp || !hin)) || (int)get32(enc + 20) != op) return ORC_INVALID;
  if (open_msg(ref, ref_len, &R)) return ORC_INVALID;
  int64_t n_ref = get32(enc + 8), n_match = get32(enc + 12), n_new = get32(enc + 16);
  uint64_t ref_words = get64(enc + 24), fold = get64(enc + 32);
  uint64_t W = get64(enc + 40), new_words = get64(enc + 48), var_bytes = get64(enc + 56);
  uint64_t rfold = 0;
  for (int64_t j = 0; j < R.n; ++j) rfold ^= get64(record(&R, j));
  if (n_ref != R.n || ref_words != (uint64_t)R.rec_words || fold != rfold) return ORC_REF_MISMATCH;
  if (n_match > n_ref || W > ref_words || n_new > enc_len / 4 || new_words > (uint64_t)enc_len / 8 ||
      var_bytes > (uint64_t)enc_len)
    return ORC_CORRUPT;
  int64_t G = ((int64_t)W + 63) / 64;
  int64_t sz_pres = 8 * ((n_ref + 63) / 64), sz_bits = 8 * G, sz_gs = round8(G), sz_ns = round8(4 * n_new);
  int64_t total = 64 + sz_pres + sz_bits + sz_gs + sz_ns + 8 * (int64_t)new_words + (int64_t)var_bytes;
  if (total != enc_len) return ORC_CORRUPT;
  const uint8_t *pres = enc + 64, *bits = pres + sz_pres, *gs = bits + sz_bits, *ns = gs + sz_gs;
  const uint8_t *nrec = ns + sz_ns, *var = nrec + 8 * new_words;

  /* presence bitmap: no bits past n_ref; counts agree with the header */
  int64_t cnt = 0;
  uint64_t wsum = 0;
  for (int64_t j = 0; j < 8 * sz_pres; ++j) {
    int bit = (pres[j / 8] >> (j % 8)) & 1;
    if (!bit) continue;
    if (j >= n_ref) return ORC_CORRUPT;
    ++cnt;
    wsum += (uint64_t)rec_words_of(record(&R, j));
  }
  if (cnt != n_match || wsum != W) return ORC_CORRUPT;
  for (int64_t w = (int64_t)W; w < 8 * sz_bits; ++w)
    if ((bits[w / 8] >> (w % 8)) & 1) return ORC_CORRUPT;
  /* mode 2: bit 7 of a group's size byte says its residual is against the
   * prediction; the size is the other 7 bits */
  const uint8_t size_mask = mode == 2 ? 0x7F : 0xFF;
  uint64_t gsum = 0;
  for (int64_t g = 0; g < G; ++g) gsum += 8u * (gs[g] & size_mask);
  for (int64_t g = G; g < sz_gs; ++g)
    if (gs[g]) return ORC_CORRUPT;
  if (gsum != var_bytes) return ORC_CORRUPT;
  uint64_t nsum = 0;
  for (int64_t r = 0; r < n_new; ++r) {
    uint32_t sz = get32(ns + 4 * r);
    if (sz < 2) return ORC_CORRUPT;
    nsum += sz;
  }
  for (int64_t b = 4 * n_new; b < sz_ns; ++b)
    if (ns[b]) return ORC_CORRUPT;
  if (nsum != new_words) return ORC_CORRUPT;

  /* unpack the residual */
  uint64_t *D = calloc((size_t)W + 1, sizeof(uint64_t));
  int64_t at = 0;
  for (int64_t g = 0; g < G; ++g) {
    int64_t blk = 8 * (int64_t)(gs[g] & size_mask);
    int64_t popc = 0;
    for (int64_t w = 64 * g; w < (int64_t)W && w < 64 * g + 64; ++w) popc += (bits[w / 8] >> (w % 8)) & 1;
    int64_t need = (popc + 1) / 2;
    if (need > blk) { free(D); return ORC_CORRUPT; }
    const uint8_t *nib = var + at;
    int64_t sp = need, t = 0;
    for (int64_t w = 64 * g; w < (int64_t)W && w < 64 * g + 64; ++w) {
      if (!((bits[w / 8] >> (w % 8)) & 1)) continue;
      int len = (nib[t / 2] >> (4 * (t % 2))) & 0xF;
      if (len < 1 || len > 8 || sp + len > blk) { free(D); return ORC_CORRUPT; }
      uint64_t v = 0;
      for (int b = 0; b < len; ++b) v |= (uint64_t)nib[sp + b] << (8 * b);
      if ((v >> (8 * (len - 1))) == 0) { free(D); return ORC_CORRUPT; }
      D[w] = v;
      sp += len;
      ++t;
    }
    if (popc % 2 && (nib[popc / 2] >> 4) != 0) { free(D); return ORC_CORRUPT; }
    if (round8(sp) != blk) { free(D); return ORC_CORRUPT; }
    for (int64_t b = sp; b < blk; ++b)
      if (nib[b]) { free(D); return ORC_CORRUPT; }
    at += blk;
  }

  /* C' = matched slots restored in reference order, then the new records */
  int64_t n_out = n_match + n_new;
  int64_t size = 32 + 8 * ((n_out + 1) / 2) + 8 * (int64_t)(W + new_words);
  *out_len = size;
  if (size > cap) { free(D); return ORC_CAPACITY; }
  int32_t *nbr = NULL;
  if (mode >= 1) {
    nbr = malloc(sizeof(int32_t) * (size_t)(R.n + 1));
    neighbour_counts(&R, mlp->cell, nbr);
  }
  uint64_t *X = malloc(sizeof(uint64_t) * (size_t)(R.rec_words + 1));
  memset(out, 0, (size_t)size);
  put32(out, TAM1_MAGIC);
  put16(out + 4, 1);
  put32(out + 8, (uint32_t)n_out);
  put64(out + 16, W + new_words);
  uint8_t *offs = out + 32, *recs = out + 32 + 8 * ((n_out + 1) / 2);
  int64_t *slot_of = malloc(sizeof(int64_t) * (size_t)(n_out + 1));
  int64_t k = 0, wat = 0, q = 0;
  int st = ORC_OK;
  for (int64_t j = 0; j < n_ref && st == ORC_OK; ++j) {
    if (!((pres[j / 8] >> (j % 8)) & 1)) continue;
    const uint8_t *rj = record(&R, j);
    int64_t words = rec_words_of(rj);
    if (mode >= 1) predicted_record(&R, j, mlp, hin, nbr, X);
    else for (int64_t t = 0; t < words; ++t) X[t] = get64(rj + 8 * t);
    put32(offs + 4 * k, (uint32_t)wat);
    for (int64_t t = 0; t < words; ++t) {
      /* mode 2: the prediction only in groups flagged learned */
      int use_x = mode != 2 || (gs[(q + t) / 64] & 0x80);
      put64(recs + 8 * (wat + t), undiff_word(D[q + t], use_x ? X[t] : get64(rj + 8 * t), op));
    }
    /* identity and shape of a matched record are those of the reference */
    if (get64(recs + 8 * wat) != get64(rj) || get64(recs + 8 * wat + 8) != get64(rj + 8)) st = ORC_CORRUPT;
    slot_of[k++] = j;
    wat += words;
    q += words;
  }
  for (int64_t r = 0; r < n_new && st == ORC_OK; ++r) {
    int64_t words = get32(ns + 4 * r);
    const uint8_t *src = nrec + 8 * (wat - (int64_t)W);
    if (get64(src) == 0 || (int64_t)(get64(src + 8) >> 32) != words) { st = ORC_CORRUPT; break; }
    put32(offs + 4 * k, (uint32_t)wat);
    memcpy(recs + 8 * wat, src, (size_t)(8 * words));
    slot_of[k++] = -1;
    wat += words;
  }
  if (st == ORC_OK && hout) write_history(&R, n_out, slot_of, hin, hout);
  free(slot_of);
  free(X);
  free(nbr);
  free(D);
  return st;
}

/* ======================================================================== */
/* Store after a migration exchange (Sec. 2.1 "Agent Migration", records as  */
/* serialized in Sec. 2.2.1)                                                 */
/* ======================================================================== */
/*
 * Partition q of the result: the agents of input partition q that lie inside
 * box q (offset 0 on every axis, i.e. not selected as migrants), in store
 * order; then the records of every message s with dest[s] == q, messages in
 * ascending s, records in message order.  A kept agent keeps all nf_cols fp64
 * and ni_cols int32 columns and its behaviour bytes.  An unpacked record gives
 * uid (word 0), class and behaviour count (word 1), the class's fp64 fields
 * (the next n_f64 words), its int32 attributes (the next ceil(n_i32/2) words,
 * two per word, low half first), zeros in the remaining columns, and the rest
 * of the record as behaviour bytes.
 */
static int msg_span(const uint8_t *msgs, int64_t msgs_len, const int64_t *msg_off, int64_t s, msg_t *m) {
  int64_t a = msg_off[s], b = msg_off[s + 1];
  if (a < 0 || b < a || b > msgs_len || a % 8 != 0) return ORC_INVALID;
  return open_msg(msgs + a, b - a, m);
}

int orc_migrate_apply(const orc_agents *in, int64_t P, const int64_t *part_off, const double *boxes,
                      int n_classes, const uint16_t *n_f64, const uint16_t *n_i32, int nf_cols, int ni_cols,
                      const uint8_t *msgs, int64_t msgs_len, const int64_t *msg_off, int64_t nseg,
                      const int32_t *dest, orc_store *out, int64_t *part_off_out, int64_t *sizes) {
  if (part_off[0] != 0 || part_off[P] > in->n) return ORC_INVALID;
  for (int64_t p = 0; p < P; ++p)
    if (part_off[p + 1] < part_off[p]) return ORC_INVALID;
  /* every message and record is checked, also those of skipped messages */
  for (int64_t s = 0; s < nseg; ++s) {
    msg_t m;
    if (msg_span(msgs, msgs_len, msg_off, s, &m) || dest[s] >= P) return ORC_INVALID;
    for (int64_t r = 0; r < m.n; ++r) {
      const uint8_t *rec = record(&m, r);
      uint64_t h = get64(rec + 8);
      int c = (int)(h & 0xFFFF);
      if (get64(rec) == 0 || c >= n_classes) return ORC_INVALID;
      if (rec_words_of(rec) < 2 + n_f64[c] + (n_i32[c] + 1) / 2) return ORC_INVALID;
    }
  }
  unsigned char *keep = malloc((size_t)in->n + 1);
  int64_t n_out = 0, beh_out = 0;
  for (int64_t q = 0; q < P; ++q) {
    const double *lo = boxes + 6 * q, *hi = boxes + 6 * q + 3;
    for (int64_t i = part_off[q]; i < part_off[q + 1]; ++i) {
      int inside = 1;
      for (int a = 0; a < 3; ++a)
        if (axis_offset(in->f64[a * in->f64_stride + i], lo[a], hi[a]) != 0) inside = 0;
      keep[i] = (unsigned char)inside;
      if (!inside) continue;
      int64_t bytes = in->beh_off[i + 1] - in->beh_off[i];
      if (in->beh_off[i] % 8 != 0 || bytes < 0 || bytes % 8 != 0) { free(keep); return ORC_INVALID; }
      ++n_out;
      beh_out += bytes;
    }
  }
  for (int64_t s = 0; s < nseg; ++s) {
    if (dest[s] < 0) continue;
    msg_t m;
    msg_span(msgs, msgs_len, msg_off, s, &m);
    for (int64_t r = 0; r < m.n; ++r) {
      const uint8_t *rec = record(&m, r);
      int c = (int)(get64(rec + 8) & 0xFFFF);
      ++n_out;
      beh_out += 8 * (rec_words_of(rec) - 2 - n_f64[c] - (n_i32[c] + 1) / 2);
    }
  }
  sizes[0] = n_out;
  sizes[1] = beh_out;
  /* partition starts of the result */
  int64_t pos = 0;
  for (int64_t q = 0; q < P; ++q) {
    part_off_out[q] = pos;
    for (int64_t i = part_off[q]; i < part_off[q + 1]; ++i) pos += keep[i];
    for (int64_t s = 0; s < nseg; ++s)
      if (dest[s] == q) {
        msg_t m;
        msg_span(msgs, msgs_len, msg_off, s, &m);
        pos += m.n;
      }
  }
  part_off_out[P] = pos;
  if (n_out > out->cap || beh_out > out->beh_cap) { free(keep); return ORC_CAPACITY; }
  int64_t j = 0, boff = 0;
  for (int64_t q = 0; q < P; ++q) {
    for (int64_t i = part_off[q]; i < part_off[q + 1]; ++i) {
      if (!keep[i]) continue;
      out->uid[j] = in->uid[i];
      out->cls[j] = in->cls[i];
      out->nb[j] = in->nb[i];
      for (int k = 0; k < nf_cols; ++k) out->f64[k * out->f64_stride + j] = in->f64[k * in->f64_stride + i];
      for (int k = 0; k < ni_cols; ++k) out->i32[k * out->i32_stride + j] = in->i32[k * in->i32_stride + i];
      int64_t bytes = in->beh_off[i + 1] - in->beh_off[i];
      out->beh_off[j] = boff;
      memcpy(out->beh + boff, in->beh + in->beh_off[i], (size_t)bytes);
      boff += bytes;
      ++j;
    }
    for (int64_t s = 0; s < nseg; ++s) {
      if (dest[s] != q) continue;
      msg_t m;
      msg_span(msgs, msgs_len, msg_off, s, &m);
      for (int64_t r = 0; r < m.n; ++r) {
        const uint8_t *rec = record(&m, r);
        uint64_t h = get64(rec + 8);
        int c = (int)(h & 0xFFFF);
        out->uid[j] = get64(rec);
        out->cls[j] = (uint16_t)c;
        out->nb[j] = (uint16_t)((h >> 16) & 0xFFFF);
        const uint8_t *f = rec + 16;
        for (int k = 0; k < nf_cols; ++k) {
          double v = 0.0;
          if (k < n_f64[c]) memcpy(&v, f + 8 * k, 8);
          out->f64[k * out->f64_stride + j] = v;
        }
        const uint8_t *at = f + 8 * n_f64[c];
        for (int k = 0; k < ni_cols; ++k) {
          int32_t v = 0;
          if (k < n_i32[c]) memcpy(&v, at + 4 * k, 4);
          out->i32[k * out->i32_stride + j] = v;
        }
        int64_t fixed = 2 + n_f64[c] + (n_i32[c] + 1) / 2;
        int64_t bytes = 8 * (rec_words_of(rec) - fixed);
        out->beh_off[j] = boff;
        memcpy(out->beh + boff, rec + 8 * fixed, (size_t)bytes);
        boff += bytes;
        ++j;
      }
    }
  }
  out->beh_off[j] = boff;
  free(keep);
  return ORC_OK;
}

/* ======================================================================== */
/* Growth of viewed records (Sec. 2.2.1 "Mutability")                       */
/* ======================================================================== */
/*
 * A record used in place may need more room than it has in its message (a
 * behaviour is added).  The paper's answer is a new block outside the buffer
 * and the old block given up.  Here the new block comes from an arena that
 * follows the last message in the same buffer: bytes [msg_off[nseg], cap),
 * of which *arena_used are taken; a record's block in use must lie below
 * the arena's free part.  A grown record keeps its words, gets zero
 * words up to its new size and that size in its header, and its offset is
 * redirected to the new block (offsets count 8-byte words from the message's
 * record area, so they may now point past it).  Compaction writes messages
 * whose offsets are redirected back in canonical form.
 */
/* Header of a message whose offsets may be redirected: the checks of the
 * view without the ones on offsets and records. */
static int tam1_head(const uint8_t *msg, int64_t len, int64_t *n_out, int64_t *rw_out) {
  if (len < 32) return ORC_INVALID;
  if (get32(msg) != TAM1_MAGIC || get16(msg + 4) != 1 || get16(msg + 6) != 0) return ORC_INVALID;
  if (get32(msg + 12) != 0 || get64(msg + 24) != 0) return ORC_INVALID;
  int64_t n = get32(msg + 8);
  uint64_t rw = get64(msg + 16);
  if (n > len / 4 || rw > (uint64_t)len / 8) return ORC_INVALID;
  if (rw < 2 * (uint64_t)n || (n == 0 && rw != 0)) return ORC_INVALID;
  if (32 + 8 * ((n + 1) / 2) + 8 * (int64_t)rw != len) return ORC_INVALID;
  if (n % 2 && get32(msg + 32 + 4 * n) != 0) return ORC_INVALID;
  *n_out = n;
  *rw_out = (int64_t)rw;
  return ORC_OK;
}

/* Byte position of record r of the message at a (header already checked)
 * and its size in words; the record must lie below byte `limit`. */
static int locate_any(const uint8_t *msgs, int64_t limit, int64_t a, int64_t n, int64_t r, int64_t *pos,
                      int64_t *words) {
  int64_t recs = a + 32 + 8 * ((n + 1) / 2);
  int64_t p = recs + 8 * (int64_t)get32(msgs + a + 32 + 4 * r);
  if (p + 16 > limit) return ORC_INVALID;
  int64_t w = (int64_t)(get64(msgs + p + 8) >> 32);
  if (w < 2 || p + 8 * w > limit) return ORC_INVALID;
  *pos = p;
  *words = w;
  return ORC_OK;
}

int orc_view_grow(uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg, const int32_t *seg,
                  const uint32_t *rec, const uint32_t *words, int64_t n, int64_t *arena_used) {
  if (nseg < 0 || n < 0 || cap > ((int64_t)1 << 35)) return ORC_INVALID;
  int64_t a0 = msg_off[nseg];
  if (a0 < 0 || a0 > cap || a0 % 8 != 0 || *arena_used < 0 || *arena_used % 8 != 0) return ORC_INVALID;
  int64_t need = 0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t s = seg[k];
    if (s < 0 || s >= nseg) return ORC_INVALID;
    if (k > 0 && (seg[k] < seg[k - 1] || (seg[k] == seg[k - 1] && rec[k] <= rec[k - 1]))) return ORC_INVALID;
    int64_t a = msg_off[s], nn, rw, pos, w;
    if (a < 0 || msg_off[s + 1] < a || msg_off[s + 1] > a0 || a % 8 != 0) return ORC_INVALID;
    if (tam1_head(msgs + a, msg_off[s + 1] - a, &nn, &rw) || rec[k] >= nn) return ORC_INVALID;
    /* the block in use lies below the arena's free part (the part this call fills) */
    if (locate_any(msgs, a0 + *arena_used, a, nn, rec[k], &pos, &w) || (int64_t)words[k] < w) return ORC_INVALID;
    need += 8 * (int64_t)words[k];
  }
  if (a0 + *arena_used + need > cap) return ORC_CAPACITY;
  int64_t at = a0 + *arena_used;
  for (int64_t k = 0; k < n; ++k) {
    int64_t s = seg[k], a = msg_off[s], nn, rw, pos, w;
    tam1_head(msgs + a, msg_off[s + 1] - a, &nn, &rw);
    locate_any(msgs, cap, a, nn, rec[k], &pos, &w);
    memcpy(msgs + at, msgs + pos, (size_t)(8 * w));
    memset(msgs + at + 8 * w, 0, (size_t)(8 * ((int64_t)words[k] - w)));
    uint64_t h = get64(msgs + at + 8);
    put64(msgs + at + 8, (h & 0xFFFFFFFFull) | ((uint64_t)words[k] << 32));
    int64_t recs = a + 32 + 8 * ((nn + 1) / 2);
    put32(msgs + a + 32 + 4 * (int64_t)rec[k], (uint32_t)((at - recs) / 8));
    at += 8 * (int64_t)words[k];
  }
  *arena_used += need;
  return ORC_OK;
}

int orc_view_compact(const uint8_t *msgs, int64_t cap, const int64_t *msg_off, int64_t nseg, uint8_t *out,
                     int64_t out_cap, int64_t *out_off) {
  if (nseg < 0) return ORC_INVALID;
  int64_t total = 0;
  for (int64_t s = 0; s < nseg; ++s) {
    int64_t a = msg_off[s], nn, rw, pos, w, sum = 0;
    if (a < 0 || msg_off[s + 1] < a || msg_off[s + 1] > cap || a % 8 != 0) return ORC_INVALID;
    if (tam1_head(msgs + a, msg_off[s + 1] - a, &nn, &rw)) return ORC_INVALID;
    for (int64_t r = 0; r < nn; ++r) {
      if (locate_any(msgs, cap, a, nn, r, &pos, &w)) return ORC_INVALID;
      sum += w;
    }
    out_off[s] = total;
    total += 32 + 8 * ((nn + 1) / 2) + 8 * sum;
  }
  out_off[nseg] = total;
  if (total > out_cap) return ORC_CAPACITY;
  for (int64_t s = 0; s < nseg; ++s) {
    int64_t a = msg_off[s], nn, rw, pos, w, sum = 0;
    tam1_head(msgs + a, msg_off[s + 1] - a, &nn, &rw);
    uint8_t *m = out + out_off[s];
    uint8_t *recs = m + 32 + 8 * ((nn + 1) / 2);
    for (int64_t r = 0; r < nn; ++r) {
      locate_any(msgs, cap, a, nn, r, &pos, &w);
      put32(m + 32 + 4 * r, (uint32_t)sum);
      memcpy(recs + 8 * sum, msgs + pos, (size_t)(8 * w));
      sum += w;
    }
    if (nn % 2) put32(m + 32 + 4 * nn, 0);
    put32(m, TAM1_MAGIC);
    put32(m + 4, 1);  /* version 1, flags 0 */
    put32(m + 8, (uint32_t)nn);
    put32(m + 12, 0);
    put64(m + 16, (uint64_t)sum);
    put64(m + 24, 0);
  }
  return ORC_OK;
}
