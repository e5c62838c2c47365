// ta_train.hip -- training the learned predictor on the GPU.
//
// Parameters are fp32 (W1 64x12, b1 64, W2 64x64, b2 64, W3 4x64, b3 4).  The
// forward pass rounds them (int8 weights, integer biases) and runs the very
// integer network the exchange evaluates; the loss is the L1 distance, in
// quanta of 2^-12 um, between the unrounded output o / 2^r3 and the true next
// move.  The backward pass lets gradients through every rounding unchanged
// and through the activation clamps where 0 <= pre-clamp value <= 127.
//
// k_train_grad: each block takes tiles of 64 samples; 256 threads compute
//   the forward pass in LDS, then the backward pass, and keep their share of
//   the gradient in registers (each parameter owned by one thread of the
//   block), so a block's partial gradient needs no atomics.
// k_train_reduce: sums the block partials in a fixed order (deterministic).
// k_adam: Adam update, parameters kept inside the representable range.
#include <math.h>
#include <string.h>

#include <vector>

#include "ta_internal.hpp"
#include "ta_predict.hpp"

using namespace ta;

namespace {

constexpr int NP = 768 + 64 + 4096 + 64 + 256 + 4;  // 5252 parameters
constexpr int O_W1 = 0, O_B1 = 768, O_W2 = 832, O_B2 = 4928, O_W3 = 4992, O_B3 = 5248;
constexpr int TS = 64;        // samples per tile
constexpr int TRAIN_BLOCKS = 256;

struct QW {
  int8_t w1[768];
  int8_t w2[4096];
  int8_t w3[256];
  int32_t b1[64];
  int32_t b2[64];
  int32_t b3[4];
};

__global__ void k_quantize(const float* theta, QW* q) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
    const float v = rintf(theta[p]);
    if (p < O_B1) q->w1[p] = (int8_t)fminf(fmaxf(v, -128.f), 127.f);
    else if (p < O_W2) q->b1[p - O_B1] = (int32_t)fminf(fmaxf(v, -16777216.f), 16777216.f);
    else if (p < O_B2) q->w2[p - O_W2] = (int8_t)fminf(fmaxf(v, -128.f), 127.f);
    else if (p < O_W3) q->b2[p - O_B2] = (int32_t)fminf(fmaxf(v, -16777216.f), 16777216.f);
    else if (p < O_B3) q->w3[p - O_W3] = (int8_t)fminf(fmaxf(v, -128.f), 127.f);
    else q->b3[p - O_B3] = (int32_t)fminf(fmaxf(v, -16777216.f), 16777216.f);
  }
}

__global__ __launch_bounds__(BLOCK) void k_train_grad(const QW* qw, const int32_t* in, const float* tgt, int64_t n,
                                                      uint32_t r1, uint32_t r2, uint32_t r3, float* partial) {
  __shared__ QW sq;
  __shared__ float sX[TS][12];
  __shared__ float sH1[TS][64], sH2[TS][64], sGA2[TS][64], sGA1[TS][64];
  __shared__ uint8_t sM1[TS][64], sM2[TS][64];
  __shared__ float sGO[TS][4];
  __shared__ float sLoss[BLOCK];
  {
    const uint32_t* s = reinterpret_cast<const uint32_t*>(qw);
    uint32_t* d = reinterpret_cast<uint32_t*>(&sq);
    for (uint32_t i = threadIdx.x; i < sizeof(QW) / 4; i += BLOCK) d[i] = s[i];
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int s_ = t & (TS - 1), q = t >> 6;  // sample, quarter of the hidden units
  const float inv1 = ldexpf(1.f, -(int)r1), inv2 = ldexpf(1.f, -(int)r2);
  const double inv3 = ldexp(1.0, -(int)r3);
  const float gscale = (float)(inv3 / (double)n);
  float accW2[16], accW1[3];
  float accW3 = 0.f, accb3 = 0.f, accb2 = 0.f, accb1 = 0.f, loss = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) accW2[k] = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) accW1[k] = 0.f;
  const int64_t ntiles = (n + TS - 1) / TS;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * TS + s_;
    const bool valid = row < n;
    for (int e = t; e < TS * 12; e += BLOCK) {
      const int64_t r = tile * TS + e / 12;
      sX[e / 12][e % 12] = r < n ? (float)in[r * 12 + e % 12] : 0.f;
    }
    __syncthreads();
    // layer 1: 16 hidden units of sample s_
    #pragma unroll 2
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * q + jj;
      int32_t a = sq.b1[j];
      for (int c = 0; c < 12; ++c) a += (int32_t)sq.w1[j * 12 + c] * (int32_t)sX[s_][c];
      const int32_t z = requant(a, r1);
      sM1[s_][j] = (z >= 0 && z <= 127) ? 1 : 0;
      sH1[s_][j] = (float)clampi(z, 0, 127);
    }
    __syncthreads();
    // layer 2
    #pragma unroll 2
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * q + jj;
      int32_t a = sq.b2[j];
      for (int i = 0; i < 64; ++i) a += (int32_t)sq.w2[j * 64 + i] * (int32_t)sH1[s_][i];
      const int32_t z = requant(a, r2);
      sM2[s_][j] = (z >= 0 && z <= 127) ? 1 : 0;
      sH2[s_][j] = (float)clampi(z, 0, 127);
    }
    __syncthreads();
    // layer 3 (output q of sample s_) and the L1 loss gradient
    {
      int32_t o = sq.b3[q];
      for (int j = 0; j < 64; ++j) o += (int32_t)sq.w3[q * 64 + j] * (int32_t)sH2[s_][j];
      float go = 0.f;
      if (valid) {
        const double diff = (double)o * inv3 - (double)tgt[row * 4 + q];
        loss += (float)fabs(diff);
        go = diff > 0 ? gscale : (diff < 0 ? -gscale : 0.f);
      }
      sGO[s_][q] = go;
    }
    __syncthreads();
    // backward through layer 3
    #pragma unroll 2
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * q + jj;
      float gh = 0.f;
      for (int k = 0; k < 4; ++k) gh += (float)sq.w3[k * 64 + j] * sGO[s_][k];
      sGA2[s_][j] = sM2[s_][j] ? gh * inv2 : 0.f;
    }
    {
      const int k = t >> 6, j = t & 63;  // dW3[k][j]
      #pragma unroll 2
      for (int s = 0; s < TS; ++s) accW3 += sGO[s][k] * sH2[s][j];
      if (t < 4)
        #pragma unroll 2
        for (int s = 0; s < TS; ++s) accb3 += sGO[s][t];
    }
    __syncthreads();
    // backward through layer 2
    #pragma unroll 2
    for (int ii = 0; ii < 16; ++ii) {
      const int i = 16 * q + ii;
      float gh = 0.f;
      for (int j = 0; j < 64; ++j) gh += (float)sq.w2[j * 64 + i] * sGA2[s_][j];
      sGA1[s_][i] = sM1[s_][i] ? gh * inv1 : 0.f;
    }
    {
      const int j = t >> 2, i0 = 16 * (t & 3);  // dW2[j][i0..i0+15]
      #pragma unroll 2
      for (int s = 0; s < TS; ++s) {
        const float g = sGA2[s][j];
#pragma unroll
        for (int k = 0; k < 16; ++k) accW2[k] += g * sH1[s][i0 + k];
      }
      if (t < 64)
        #pragma unroll 2
        for (int s = 0; s < TS; ++s) accb2 += sGA2[s][t];
    }
    __syncthreads();
    // gradients of layer 1
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int p = 3 * t + e;  // dW1[p / 12][p % 12]
      #pragma unroll 2
      for (int s = 0; s < TS; ++s) accW1[e] += sGA1[s][p / 12] * sX[s][p % 12];
    }
    if (t < 64)
      #pragma unroll 2
      for (int s = 0; s < TS; ++s) accb1 += sGA1[s][t];
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * (NP + 1);
  out[O_W3 + t] = accW3;
  if (t < 4) out[O_B3 + t] = accb3;
  {
    const int j = t >> 2, i0 = 16 * (t & 3);
#pragma unroll
    for (int k = 0; k < 16; ++k) out[O_W2 + j * 64 + i0 + k] = accW2[k];
  }
  if (t < 64) {
    out[O_B2 + t] = accb2;
    out[O_B1 + t] = accb1;
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) out[O_W1 + 3 * t + e] = accW1[e];
  sLoss[t] = loss;
  __syncthreads();
  if (t == 0) {
    float l = 0.f;
    for (int i = 0; i < BLOCK; ++i) l += sLoss[i];
    out[NP] = l / (float)n;
  }
}

__global__ void k_train_reduce(const float* partial, int nb, float* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NP) return;
  float acc = 0.f;
  for (int b = 0; b < nb; ++b) acc += partial[(int64_t)b * (NP + 1) + p];
  grad[p] = acc;  // grad[NP] is the loss
}

__global__ void k_adam(float* theta, float* m, float* v, const float* grad, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  float th = theta[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  const bool is_w = p < O_B1 || (p >= O_W2 && p < O_B2) || (p >= O_W3 && p < O_B3);
  th = is_w ? fminf(fmaxf(th, -128.f), 127.f) : fminf(fmaxf(th, -16777216.f), 16777216.f);
  theta[p] = th;
}

}  // namespace

struct ta_trainer {
  int device;
  float* theta = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;     // [NP + 1]: gradient, loss
  float* partial = nullptr;  // [TRAIN_BLOCKS][NP + 1]
  QW* qw = nullptr;
  uint32_t r1, r2, r3;
  double cell;
  int64_t step = 0;
};

extern "C" ta_status ta_trainer_create(ta_ctx* c, const float* init, uint32_t r1, uint32_t r2, uint32_t r3, double cell,
                                       ta_trainer** out) {
  if (!c || !init || !out || r1 > 24 || r2 > 24 || r3 > 24 || !(cell > 0) || !isfinite(cell)) return TA_ERR_INVALID;
  ta_trainer* t = new ta_trainer();
  t->device = c->device;
  t->r1 = r1;
  t->r2 = r2;
  t->r3 = r3;
  t->cell = cell;
  bool ok = hipMalloc(&t->theta, 4 * NP) == hipSuccess && hipMalloc(&t->m, 4 * NP) == hipSuccess &&
            hipMalloc(&t->v, 4 * NP) == hipSuccess && hipMalloc(&t->grad, 4 * (NP + 1)) == hipSuccess &&
            hipMalloc(&t->partial, sizeof(float) * (size_t)TRAIN_BLOCKS * (NP + 1)) == hipSuccess &&
            hipMalloc(&t->qw, sizeof(QW)) == hipSuccess;
  ok = ok && hipMemcpy(t->theta, init, 4 * NP, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(t->m, 0, 4 * NP) == hipSuccess && hipMemset(t->v, 0, 4 * NP) == hipSuccess;
  if (!ok) {
    ta_trainer_free(t);
    return TA_ERR_HIP;
  }
  *out = t;
  return TA_OK;
}

extern "C" void ta_trainer_free(ta_trainer* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(t->theta);
  (void)hipFree(t->m);
  (void)hipFree(t->v);
  (void)hipFree(t->grad);
  (void)hipFree(t->partial);
  (void)hipFree(t->qw);
  delete t;
}

extern "C" ta_status ta_trainer_grad(ta_ctx* c, ta_trainer* t, const int32_t* in, const float* tgt, int64_t n,
                                     float* grad_out, void* stream) {
  if (!c || !t || n <= 0 || !in || !tgt) return TA_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  k_quantize<<<ceil_div(NP, BLOCK), BLOCK, 0, s>>>(t->theta, t->qw);
  const int nb = (int)std::min<int64_t>(TRAIN_BLOCKS, ceil_div(n, TS));
  k_train_grad<<<nb, BLOCK, 0, s>>>(t->qw, in, tgt, n, t->r1, t->r2, t->r3, t->partial);
  k_train_reduce<<<ceil_div(NP + 1, BLOCK), BLOCK, 0, s>>>(t->partial, nb, t->grad);
  if (grad_out) TA_HIP(hipMemcpyAsync(grad_out, t->grad, 4 * (NP + 1), hipMemcpyDeviceToDevice, s));
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_trainer_step(ta_ctx* c, ta_trainer* t, const int32_t* in, const float* tgt, int64_t n,
                                     float lr, float beta1, float beta2, float eps, void* stream) {
  ta_status st = ta_trainer_grad(c, t, in, tgt, n, nullptr, stream);
  if (st) return st;
  t->step += 1;
  const float c1 = 1.f - powf(beta1, (float)t->step), c2 = 1.f - powf(beta2, (float)t->step);
  k_adam<<<ceil_div(NP, BLOCK), BLOCK, 0, (hipStream_t)stream>>>(t->theta, t->m, t->v, t->grad, lr, beta1, beta2, eps,
                                                                 c1, c2);
  TA_LAUNCH_CHECK();
  return TA_OK;
}

extern "C" ta_status ta_trainer_params(ta_trainer* t, float* host_out) {
  if (!t || !host_out) return TA_ERR_INVALID;
  TA_HIP(hipDeviceSynchronize());
  TA_HIP(hipMemcpy(host_out, t->theta, 4 * NP, hipMemcpyDeviceToHost));
  return TA_OK;
}

extern "C" ta_status ta_trainer_export(ta_trainer* t, void* blob, size_t len) {
  if (!t || !blob || len != 5672) return TA_ERR_INVALID;
  std::vector<float> th(NP);
  TA_HIP(hipDeviceSynchronize());
  TA_HIP(hipMemcpy(th.data(), t->theta, 4 * NP, hipMemcpyDeviceToHost));
  uint8_t* b = static_cast<uint8_t*>(blob);
  memset(b, 0, len);
  const uint32_t magic = 0x31504154u, ver = 1;
  memcpy(b, &magic, 4);
  memcpy(b + 4, &ver, 4);
  auto w8 = [&](int off, int cnt, uint8_t* dst) {
    for (int i = 0; i < cnt; ++i) {
      const float v = fminf(fmaxf(rintf(th[off + i]), -128.f), 127.f);
      dst[i] = (uint8_t)(int8_t)v;
    }
  };
  auto w32 = [&](int off, int cnt, uint8_t* dst) {
    for (int i = 0; i < cnt; ++i) {
      const int32_t v = (int32_t)fminf(fmaxf(rintf(th[off + i]), -16777216.f), 16777216.f);
      memcpy(dst + 4 * i, &v, 4);
    }
  };
  uint8_t* p = b + 8;
  w8(O_W1, 768, p);
  p += 768;
  w8(O_W2, 4096, p);
  p += 4096;
  w8(O_W3, 256, p);
  p += 256;
  w32(O_B1, 64, p);
  p += 256;
  w32(O_B2, 64, p);
  p += 256;
  w32(O_B3, 4, p);
  p += 16;
  p[0] = (uint8_t)t->r1;
  p[1] = (uint8_t)t->r2;
  p[2] = (uint8_t)t->r3;
  p += 8;
  memcpy(p, &t->cell, 8);
  return TA_OK;
}

extern "C" ta_status ta_set_window_tap(ta_ctx* c, int32_t* in_out, float* tgt_out, int64_t cap, uint64_t* count) {
  if (!c) return TA_ERR_INVALID;
  if (!in_out) {
    c->tap_in = nullptr;
    c->tap_tgt = nullptr;
    c->tap_cap = 0;
    c->tap_count = nullptr;
    return TA_OK;
  }
  if (!tgt_out || !count || cap < 0) return TA_ERR_INVALID;
  c->tap_in = in_out;
  c->tap_tgt = tgt_out;
  c->tap_cap = cap;
  c->tap_count = reinterpret_cast<unsigned long long*>(count);
  return TA_OK;
}
