// ta_predict.hpp -- the learned predictor on the device: weights, input
// quantisation, and the integer MLP 12 -> 64 -> 64 -> 4 evaluated by one wave
// for 16 records at a time.  The 64x64 int8 layer runs on the matrix cores
// (v_mfma_i32_16x16x32_i8, int32 accumulation); the small first and last
// layers run on the vector ALUs.  All arithmetic is integer and exact, so
// every evaluation (encoder, decoder, any launch shape) gives the same bits.
#pragma once
#include <stdint.h>

#include "ta_device.hpp"

namespace ta {

struct PredW {
  int8_t w1[64 * 12];  // [out][in]
  int8_t w2[64 * 64];  // [out][in]
  int8_t w3[4 * 64];   // [out][in]
  int32_t b1[64];
  int32_t b2[64];
  int32_t b3[4];
  uint32_t r1, r2, r3, pad;
  double cell;
};

typedef int v4i __attribute__((ext_vector_type(4)));

// floor((v + 2^(r-1)) / 2^r): the shift of a signed int32 is arithmetic
__device__ inline int32_t requant(int32_t v, uint32_t r) { return r ? (v + (1 << (r - 1))) >> r : v; }
__device__ inline int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// clamp(round-half-even(v * 2^12), -32768, 32767); NaN -> 0
__device__ inline int32_t quantise(double v) {
  const double t = v * 4096.0;
  if (t != t) return 0;
  if (t >= 32767.0) return 32767;
  if (t <= -32768.0) return -32768;
  return (int32_t)rint(t);
}

// The matrix-core layout of v_mfma_i32_16x16x32_i8 (A 16x32, B 32x16, D
// 16x16, int8 operands, int32 accumulation): lane l holds row l%16 of A and
// column l%16 of B for k = 8*(l/16) .. +7 (eight bytes, lowest k in the low
// byte); D holds rows 4*(l/16) .. +3 of column l%16.
__device__ inline v4i mfma_i8(int64_t a, int64_t b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, c, 0, 0, 0);
}

// The B operands of the three layers for this lane, read once from the
// weights: layer 1 (W1 transposed, k = input, padded from 12 to 32 with
// zeros), four blocks of 16 hidden units; layer 2 (W2 transposed), four
// blocks of 16 outputs times two halves of k; layer 3 (W3 transposed, four
// output columns of 16, the others zero), two halves of k.
struct MlpOps {
  int64_t b1[4];
  int64_t b2[4][2];
  int64_t b3[2];
};
__device__ inline MlpOps mlp_ops(const PredW& W) {
  const int l = lane_id();
  const int rc = l & 15, qd = l >> 4;
  MlpOps o;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    uint64_t v = 0;
    const int j = 16 * ob + rc;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = 8 * qd + t;
      if (k < 12) v |= (uint64_t)(uint8_t)W.w1[j * 12 + k] << (8 * t);
    }
    o.b1[ob] = (int64_t)v;
#pragma unroll
    for (int half = 0; half < 2; ++half)
      o.b2[ob][half] = *reinterpret_cast<const int64_t*>(&W.w2[j * 64 + 32 * half + 8 * qd]);
  }
#pragma unroll
  for (int half = 0; half < 2; ++half)
    o.b3[half] = rc < 4 ? *reinterpret_cast<const int64_t*>(&W.w3[rc * 64 + 32 * half + 8 * qd]) : 0;
  return o;
}

// Inputs of up to 64 rows as three int8 planes: a value v in [-32768,
// 65535] (int16 moves and counts, u16 behaviour count and class) is split
// exactly as v = a*2^14 + b*2^7 + c with c, b in [0,127] and a in [-2,3].
// Row j of plane p holds the 12 inputs' bytes in bytes 0..11 of p[p][j];
// bytes 12..15 meet zero weights and are never significant.
struct MlpIn {
  uint64_t p[3][64][2];
};

// Row `row` of `dst` from 12 int32 inputs (one lane per row).
__device__ inline void mlp_in_store(MlpIn& dst, int row, const int32_t (&v)[12]) {
  uint64_t pl[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int h = i >> 3, sh = 8 * (i & 7);
    pl[0][h] |= (uint64_t)(uint8_t)(int8_t)(v[i] >> 14) << sh;
    pl[1][h] |= (uint64_t)(uint32_t)((v[i] >> 7) & 127) << sh;
    pl[2][h] |= (uint64_t)(uint32_t)(v[i] & 127) << sh;
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) *reinterpret_cast<ulonglong2*>(dst.p[p][row]) = ulonglong2{pl[p][0], pl[p][1]};
}

// One wave: rows row0 .. row0+15 of `in` -> s_q (4 outputs each), all
// three layers on the matrix cores.  Layer 1 takes one MFMA per input plane:
// W1 v = 2^14 W1 a + 2^7 W1 b + W1 c, every sum exact in int32.  Between
// layers the activations go through s_h (16 rows x 64 bytes of LDS, this
// wave's) from the output layout into the input layout.
__device__ inline void mlp16(const PredW& W, const MlpOps& ops, const MlpIn& in, int row0, uint8_t (*s_h)[64],
                             int32_t (*s_q)[4]) {
  const int l = lane_id();
  const int rc = l & 15, qd = l >> 4;
  // layer 1 A operands: row rc, inputs 8qd .. 8qd+7 (lanes with qd >= 2 and
  // inputs past 11 meet zero weights)
  const int64_t pa = (int64_t)in.p[0][row0 + rc][qd & 1];
  const int64_t pb = (int64_t)in.p[1][row0 + rc][qd & 1];
  const int64_t pc = (int64_t)in.p[2][row0 + rc][qd & 1];
  // layer 1: 64 hidden units in four blocks; rows 4qd .. 4qd+3, unit 16ob + rc
  // (the bias and rounding half start plane c's accumulator)
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const v4i z = v4i{0, 0, 0, 0};
    const int32_t c1 = W.b1[16 * ob + rc];
    const v4i da = mfma_i8(pa, ops.b1[ob], z);
    const v4i db = mfma_i8(pb, ops.b1[ob], z);
    const v4i dc = mfma_i8(pc, ops.b1[ob], v4i{c1, c1, c1, c1});
    const int j = 16 * ob + rc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t acc = da[r] * 16384 + db[r] * 128 + dc[r];
      s_h[4 * qd + r][j] = (uint8_t)clampi(acc >> W.r1, 0, 127);
    }
  }
  wave_sync();
  int64_t a[2];
#pragma unroll
  for (int half = 0; half < 2; ++half) a[half] = *reinterpret_cast<const int64_t*>(&s_h[rc][32 * half + 8 * qd]);
  wave_sync();  // every lane has its layer 1 operands before s_h is rewritten
  // layer 2: 4 blocks of 16 outputs, K = 64 in two steps
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const int n = 16 * ob + rc;
    const int32_t b = W.b2[n];
    v4i acc = v4i{b, b, b, b};
    acc = mfma_i8(a[0], ops.b2[ob][0], acc);
    acc = mfma_i8(a[1], ops.b2[ob][1], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) s_h[4 * qd + r][n] = (uint8_t)clampi(acc[r] >> W.r2, 0, 127);
  }
  wave_sync();
#pragma unroll
  for (int half = 0; half < 2; ++half) a[half] = *reinterpret_cast<const int64_t*>(&s_h[rc][32 * half + 8 * qd]);
  wave_sync();
  // layer 3: output o = column rc < 4
  const int32_t c3 = rc < 4 ? W.b3[rc & 3] : 0;
  v4i o = v4i{c3, c3, c3, c3};
  o = mfma_i8(a[0], ops.b3[0], o);
  o = mfma_i8(a[1], ops.b3[1], o);
  if (rc < 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s_q[4 * qd + r][rc] = clampi(o[r] >> W.r3, -(1 << 24), 1 << 24);
  }
}

// Copy the weights into LDS (all threads of the block) and add to every
// bias the rounding half 2^(r-1) of the requantisation that follows its
// layer: floor((a + b + h) / 2^r) is then one arithmetic shift (h = 0 when
// r = 0).  The LDS copy is only for mlp16.
__device__ inline int32_t round_half(uint32_t r) { return r ? 1 << (r - 1) : 0; }
__device__ inline void load_weights(PredW* dst, const PredW* src) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < sizeof(PredW) / 4; i += blockDim.x) d[i] = s[i];
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < 64 + 64 + 4; i += blockDim.x) {
    if (i < 64) dst->b1[i] += round_half(dst->r1);
    else if (i < 128) dst->b2[i - 64] += round_half(dst->r2);
    else dst->b3[i - 128] += round_half(dst->r3);
  }
  __syncthreads();
}

}  // namespace ta
