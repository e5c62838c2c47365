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

// One wave: rows 0..15 of s_in (12 inputs each) -> s_q (4 outputs each).
// MFMA operand layout (16x16x32, int8): lane l holds row l%16 of A and
// column l%16 of B for k = 8*(l/16) .. +7; the result holds rows
// 4*(l/16) .. +3 of column l%16.
__device__ inline void mlp16(const PredW& W, const int32_t (*s_in)[12], int32_t (*s_q)[4]) {
  const int l = lane_id();
  const int rc = l & 15, qd = l >> 4;
  // layer 1 for row rc: hidden units 8qd..8qd+7 and 32+8qd..32+8qd+7
  int64_t a[2];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    uint64_t packed = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int j = 32 * half + 8 * qd + t;
      int32_t acc = W.b1[j];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc += (int32_t)W.w1[j * 12 + c] * s_in[rc][c];
      const int32_t h = clampi(requant(acc, W.r1), 0, 127);
      packed |= (uint64_t)(uint8_t)h << (8 * t);
    }
    a[half] = (int64_t)packed;
  }
  // layer 2 on the matrix cores: 4 blocks of 16 outputs, K = 64 in two steps
  v4i acc[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const int n = 16 * ob + rc;  // output neuron of this lane's column
    const int32_t b = W.b2[n];
    acc[ob] = v4i{b, b, b, b};
    const int64_t b0 = *reinterpret_cast<const int64_t*>(&W.w2[n * 64 + 8 * qd]);
    const int64_t b1 = *reinterpret_cast<const int64_t*>(&W.w2[n * 64 + 32 + 8 * qd]);
    acc[ob] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a[0], b0, acc[ob], 0, 0, 0);
    acc[ob] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a[1], b1, acc[ob], 0, 0, 0);
  }
  // layer 3: partial sums over this lane's 4 columns for its 4 rows
  int32_t part[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 0; o < 4; ++o) part[r][o] = 0;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const int j = 16 * ob + rc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t h2 = clampi(requant(acc[ob][r], W.r2), 0, 127);
#pragma unroll
      for (int o = 0; o < 4; ++o) part[r][o] += (int32_t)W.w3[o * 64 + j] * h2;
    }
  }
  // sum over the 16 lanes holding the same rows
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) part[r][o] += __shfl_xor(part[r][o], d, WAVE);
  if (rc == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int o = 0; o < 4; ++o)
        s_q[4 * qd + r][o] = clampi(requant(part[r][o] + W.b3[o], W.r3), -(1 << 24), 1 << 24);
  }
}

// Copy the weights into LDS (all threads of the block).
__device__ inline void load_weights(PredW* dst, const PredW* src) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (uint32_t i = threadIdx.x; i < sizeof(PredW) / 4; i += blockDim.x) d[i] = s[i];
  __syncthreads();
}

}  // namespace ta
