// Internal interface of the learned proposer's network (gdg_mlp.hip) and its
// BF16 matrix-core scoring routine, shared with the decode kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GDG_MLP_IN 17
#define GDG_MLP_H 64
#ifndef GDG_MLP_PARAMS
#define GDG_MLP_PARAMS 5377
#endif
// W1 [IN][H], b1 [H], W2 [H][H], b2 [H], w3 [H], b3
static_assert(GDG_MLP_PARAMS ==
                  GDG_MLP_IN * GDG_MLP_H + GDG_MLP_H + GDG_MLP_H * GDG_MLP_H + 2 * GDG_MLP_H + 1,
              "parameter count of the 17-64-64-1 network");

// Inference copy of the network: the weight matrices transposed and rounded
// to BF16 (round to nearest even), laid out as the A operands of
// v_mfma_f32_16x16x16_bf16 -- for output tile mt and K step s, lane l holds
// 4 values of W^T[16 mt + l % 16][16 s + 4 (l / 16) + j], j = 0..3 -- and the
// biases and output weights in FP32.
struct gdg_model_dev {
  const uint2* a1;    // [4 mt][2 s][64 lanes]  layer 1 (inputs padded 17 -> 32)
  const uint2* a2;    // [4 mt][4 s][64 lanes]  layer 2
  const float* b1;    // [64]
  const float* b2;    // [64]
  const float* w3;    // [64]
  float b3;
};

typedef short gdg_bf16x4 __attribute__((ext_vector_type(4)));
typedef float gdg_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t gdg_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return u >> 16;
}

__device__ __forceinline__ gdg_bf16x4 gdg_bf16x4_of(float a, float b, float c, float d) {
  gdg_bf16x4 r;
  r.x = (short)gdg_bf16_bits(a);
  r.y = (short)gdg_bf16_bits(b);
  r.z = (short)gdg_bf16_bits(c);
  r.w = (short)gdg_bf16_bits(d);
  return r;
}

__device__ __forceinline__ gdg_bf16x4 gdg_bf16x4_load(const uint2* p) {
  const uint2 u = *p;
  gdg_bf16x4 r;
  r.x = (short)(u.x & 0xffffu);
  r.y = (short)(u.x >> 16);
  r.z = (short)(u.y & 0xffffu);
  r.w = (short)(u.y >> 16);
  return r;
}

// Scores 16 samples (candidates) with one wavefront; all 64 lanes must be
// active. Lane l supplies features 4 (l / 16) .. 4 (l / 16) + 3 of sample
// l % 16 in f[], and lanes l < 16 also feature 16 (deg). The layers are
// computed transposed (H^T = W^T X^T), so each layer's accumulator layout is
// the next layer's B operand layout. Returns the logit of sample l % 16.
__device__ __forceinline__ float mlp_score_tile(const gdg_model_dev& md, const float f[4],
                                                float deg) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const gdg_bf16x4 x0 = gdg_bf16x4_of(f[0], f[1], f[2], f[3]);
  const gdg_bf16x4 x1 = gdg_bf16x4_of(q == 0 ? deg : 0.0f, 0.0f, 0.0f, 0.0f);
  gdg_bf16x4 h1[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    gdg_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(gdg_bf16x4_load(md.a1 + (mt * 2 + 0) * 64 + lane),
                                                    x0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(gdg_bf16x4_load(md.a1 + (mt * 2 + 1) * 64 + lane),
                                                    x1, acc, 0, 0, 0);
    const int u = 16 * mt + 4 * q;
    h1[mt] = gdg_bf16x4_of(fmaxf(acc.x + md.b1[u + 0], 0.0f), fmaxf(acc.y + md.b1[u + 1], 0.0f),
                           fmaxf(acc.z + md.b1[u + 2], 0.0f), fmaxf(acc.w + md.b1[u + 3], 0.0f));
  }
  float part = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    gdg_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(gdg_bf16x4_load(md.a2 + (mt * 4 + s) * 64 + lane),
                                                      h1[s], acc, 0, 0, 0);
    const int u = 16 * mt + 4 * q;
    part += fmaxf(acc.x + md.b2[u + 0], 0.0f) * md.w3[u + 0];
    part += fmaxf(acc.y + md.b2[u + 1], 0.0f) * md.w3[u + 1];
    part += fmaxf(acc.z + md.b2[u + 2], 0.0f) * md.w3[u + 2];
    part += fmaxf(acc.w + md.b2[u + 3], 0.0f) * md.w3[u + 3];
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  (void)c;
  return part + md.b3;
}

size_t gdg_mlp_grad_work_floats(int n);
hipError_t gdg_launch_mlp_grad(int n, const float* prm, const float* x, const float* y, float* grad,
                               float* loss, float* work, hipStream_t st);
hipError_t gdg_launch_mlp_forward(int n, const float* prm, const float* x, float* z,
                                  hipStream_t st);
hipError_t gdg_launch_mlp_adam(int t, float lr, float b1, float b2, float eps, float* prm,
                               const float* g, float* m, float* v, hipStream_t st);
hipError_t gdg_launch_mlp_infer(const gdg_model_dev& md, int n, const float* x, float* z,
                                hipStream_t st);
