// ta_predict.hpp -- the learned predictor's weights on the device and the
// predicted words of matched reference records.
#pragma once
#include <stdint.h>

namespace ta {

struct PredW {
  int8_t w1[64 * 12];
  int8_t w2[64 * 64];
  int8_t w3[4 * 64];
  int32_t b1[64];
  int32_t b2[64];
  int32_t b3[4];
  uint32_t r1, r2, r3, pad;
  double cell;
};

}  // namespace ta
