// ta_predict.hip -- loading the learned predictor and evaluating it on given
// inputs (the exchange evaluates it inside ta_delta_encode/decode).
#include <math.h>
#include <string.h>

#include "ta_internal.hpp"
#include "ta_predict.hpp"

using namespace ta;

namespace {

constexpr uint32_t TAP1_MAGIC = 0x31504154u;  // "TAP1"
constexpr size_t BLOB_LEN = 5672;

// Rows are handled 64 per wave (one per lane, four groups of 16 through
// the network); weights live in LDS.
__global__ __launch_bounds__(BLOCK) void k_pred_eval(const PredW* w, const int32_t* in, int32_t* q, int64_t n) {
  __shared__ PredW s_w;
  __shared__ MlpIn s_in[WAVES];
  __shared__ int32_t s_q[WAVES][WAVE][4];
  __shared__ uint8_t s_h[WAVES][16][64];
  load_weights(&s_w, w);
  const MlpOps ops = mlp_ops(s_w);
  const int l = lane_id(), wv = wave_id();
  const int64_t chunks = (n + WAVE - 1) / WAVE;
  for (int64_t ch = (int64_t)blockIdx.x * WAVES + wv; ch < chunks; ch += (int64_t)gridDim.x * WAVES) {
    const int64_t row = ch * WAVE + l;
    int32_t v[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) v[i] = row < n ? in[row * 12 + i] : 0;
    mlp_in_store(s_in[wv], l, v);
    wave_sync();
    const int64_t left = n - ch * WAVE;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (16 * r < left) mlp16(s_w, ops, s_in[wv], 16 * r, s_h[wv], s_q[wv] + 16 * r);
    wave_sync();
    if (row < n) {
#pragma unroll
      for (int c = 0; c < 4; ++c) q[row * 4 + c] = s_q[wv][l][c];
    }
    wave_sync();
  }
}

}  // namespace

extern "C" ta_status ta_predictor_load(ta_ctx* c, const void* blob, size_t len, ta_predictor** out) {
  if (!c || !blob || !out || len != BLOB_LEN) return TA_ERR_INVALID;
  const uint8_t* b = static_cast<const uint8_t*>(blob);
  uint32_t magic, ver;
  memcpy(&magic, b, 4);
  memcpy(&ver, b + 4, 4);
  if (magic != TAP1_MAGIC || ver != 1) return TA_ERR_INVALID;
  PredW w;
  memset(&w, 0, sizeof(w));
  const uint8_t* p = b + 8;
  memcpy(w.w1, p, sizeof(w.w1));
  p += sizeof(w.w1);
  memcpy(w.w2, p, sizeof(w.w2));
  p += sizeof(w.w2);
  memcpy(w.w3, p, sizeof(w.w3));
  p += sizeof(w.w3);
  memcpy(w.b1, p, sizeof(w.b1));
  p += sizeof(w.b1);
  memcpy(w.b2, p, sizeof(w.b2));
  p += sizeof(w.b2);
  memcpy(w.b3, p, sizeof(w.b3));
  p += sizeof(w.b3);
  w.r1 = p[0];
  w.r2 = p[1];
  w.r3 = p[2];
  p += 8;
  memcpy(&w.cell, p, 8);
  for (int i = 0; i < 64; ++i)
    if (w.b1[i] > (1 << 24) || w.b1[i] < -(1 << 24) || w.b2[i] > (1 << 24) || w.b2[i] < -(1 << 24))
      return TA_ERR_INVALID;
  for (int i = 0; i < 4; ++i)
    if (w.b3[i] > (1 << 24) || w.b3[i] < -(1 << 24)) return TA_ERR_INVALID;
  if (w.r1 > 24 || w.r2 > 24 || w.r3 > 24 || !(w.cell > 0) || !isfinite(w.cell)) return TA_ERR_INVALID;
  ta_predictor* pr = new ta_predictor();
  pr->device = c->device;
  if (hipMalloc(&pr->dev, sizeof(PredW)) != hipSuccess ||
      hipMemcpy(pr->dev, &w, sizeof(PredW), hipMemcpyHostToDevice) != hipSuccess) {
    if (pr->dev) (void)hipFree(pr->dev);
    delete pr;
    return TA_ERR_HIP;
  }
  *out = pr;
  return TA_OK;
}

extern "C" void ta_predictor_free(ta_predictor* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(p->dev);
  delete p;
}

extern "C" ta_status ta_predictor_eval(ta_ctx* c, const ta_predictor* p, const int32_t* in, int32_t* q, int64_t n,
                                       void* stream) {
  if (!c || !p || n < 0 || (n > 0 && (!in || !q))) return TA_ERR_INVALID;
  if (n == 0) return TA_OK;
  c->grid = c->grid_default;
  const int g = grid_for(c, ceil_div(n, WAVE), WAVES);
  k_pred_eval<<<g, BLOCK, 0, (hipStream_t)stream>>>(static_cast<const PredW*>(p->dev), in, q, n);
  TA_LAUNCH_CHECK();
  return TA_OK;
}
