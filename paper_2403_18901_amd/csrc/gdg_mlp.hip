// The learned decimation proposer's network: a 17-64-64-1 perceptron with
// ReLU hidden layers and a logit output (the score that a candidate VN's
// favoured value is its true error bit). FP32 training kernels (forward, loss
// and backward of the mean binary cross-entropy, a deterministic gradient
// reduction, Adam) and a BF16 matrix-core inference path shared with the
// decode kernel.
//
// Parameter vector (FP32, 5377 entries): W1 [17][64] (input-major), b1 [64],
// W2 [64][64], b2 [64], w3 [64], b3.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gdg_kernels.h"
#include "gdg_mlp.h"

namespace {

constexpr int kIn = GDG_MLP_IN, kH = GDG_MLP_H, kP = GDG_MLP_PARAMS;
constexpr int kW1 = 0, kB1 = kW1 + kIn * kH, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH,
              kB3 = kW3 + kH;
constexpr int kChunk = 64;   // samples per workgroup in the gradient kernel

// Numerically stable log(1 + e^z) - y z and its derivative sigma(z) - y.
__device__ __forceinline__ float bce(float z, float y, float& dz) {
  const float e = expf(-fabsf(z));
  const float s = z >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
  dz = s - y;
  return fmaxf(z, 0.0f) - y * z + log1pf(e);
}

// Per-workgroup partial gradient of the mean loss over samples
// [chunk * kChunk, ...) (divided by n_total) and partial loss.
__global__ __launch_bounds__(256) void mlp_grad_partial(int n, const float* __restrict__ prm,
                                                        const float* __restrict__ x,
                                                        const float* __restrict__ y,
                                                        float* __restrict__ part) {
  __shared__ float P[kP];
  __shared__ float X[kChunk][kIn];
  __shared__ float H1[kChunk][kH], H2[kChunk][kH], D1[kChunk][kH], D2[kChunk][kH];
  __shared__ float DZ[kChunk], LS[kChunk];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kChunk;
  const int ns = min(kChunk, n - s0);
  for (int i = tid; i < kP; i += blockDim.x) P[i] = prm[i];
  for (int i = tid; i < kChunk * kIn; i += blockDim.x) {
    const int s = i / kIn, f = i % kIn;
    X[s][f] = s < ns ? x[(long long)(s0 + s) * kIn + f] : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < kChunk * kH; i += blockDim.x) {
    const int s = i / kH, j = i % kH;
    float a = P[kB1 + j];
    for (int f = 0; f < kIn; ++f) a += X[s][f] * P[kW1 + f * kH + j];
    H1[s][j] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  for (int i = tid; i < kChunk * kH; i += blockDim.x) {
    const int s = i / kH, j = i % kH;
    float a = P[kB2 + j];
    for (int f = 0; f < kH; ++f) a += H1[s][f] * P[kW2 + f * kH + j];
    H2[s][j] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  for (int s = tid; s < kChunk; s += blockDim.x) {
    float z = P[kB3];
    for (int j = 0; j < kH; ++j) z += H2[s][j] * P[kW3 + j];
    float dz = 0.0f, l = 0.0f;
    if (s < ns) {
      l = bce(z, y[s0 + s], dz);
      dz /= (float)n;
      l /= (float)n;
    }
    DZ[s] = dz;
    LS[s] = l;
  }
  __syncthreads();
  for (int i = tid; i < kChunk * kH; i += blockDim.x) {
    const int s = i / kH, j = i % kH;
    D2[s][j] = H2[s][j] > 0.0f ? DZ[s] * P[kW3 + j] : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < kChunk * kH; i += blockDim.x) {
    const int s = i / kH, f = i % kH;
    float a = 0.0f;
    for (int j = 0; j < kH; ++j) a += D2[s][j] * P[kW2 + f * kH + j];
    D1[s][f] = H1[s][f] > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  float* out = part + (long long)blockIdx.x * (kP + 1);
  for (int p = tid; p < kP + 1; p += blockDim.x) {
    float g = 0.0f;
    if (p < kB1) {
      const int f = p / kH, j = p % kH;
      for (int s = 0; s < kChunk; ++s) g += X[s][f] * D1[s][j];
    } else if (p < kW2) {
      for (int s = 0; s < kChunk; ++s) g += D1[s][p - kB1];
    } else if (p < kB2) {
      const int f = (p - kW2) / kH, j = (p - kW2) % kH;
      for (int s = 0; s < kChunk; ++s) g += H1[s][f] * D2[s][j];
    } else if (p < kW3) {
      for (int s = 0; s < kChunk; ++s) g += D2[s][p - kB2];
    } else if (p < kB3) {
      for (int s = 0; s < kChunk; ++s) g += H2[s][p - kW3] * DZ[s];
    } else if (p == kB3) {
      for (int s = 0; s < kChunk; ++s) g += DZ[s];
    } else {
      for (int s = 0; s < kChunk; ++s) g += LS[s];
    }
    out[p] = g;
  }
}

// grad[p] = sum over workgroups b of part[b][p], in order b = 0, 1, ...
__global__ void mlp_grad_reduce(int n_parts, const float* __restrict__ part,
                                float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kP) return;
  float g = 0.0f;
  for (int b = 0; b < n_parts; ++b) g += part[(long long)b * (kP + 1) + p];
  if (p < kP)
    grad[p] = g;
  else if (loss)
    *loss = g;
}

__global__ void mlp_forward_kernel(int n, const float* __restrict__ prm,
                                   const float* __restrict__ x, float* __restrict__ z) {
  __shared__ float P[kP];
  for (int i = threadIdx.x; i < kP; i += blockDim.x) P[i] = prm[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float in[kIn], h1[kH];
  for (int f = 0; f < kIn; ++f) in[f] = x[(long long)s * kIn + f];
  for (int j = 0; j < kH; ++j) {
    float a = P[kB1 + j];
    for (int f = 0; f < kIn; ++f) a += in[f] * P[kW1 + f * kH + j];
    h1[j] = fmaxf(a, 0.0f);
  }
  float out = P[kB3];
  for (int j = 0; j < kH; ++j) {
    float a = P[kB2 + j];
    for (int f = 0; f < kH; ++f) a += h1[f] * P[kW2 + f * kH + j];
    out += fmaxf(a, 0.0f) * P[kW3 + j];
  }
  z[s] = out;
}

// Adam (Kingma and Ba) with bias correction; step t >= 1.
__global__ void mlp_adam_kernel(int t, float lr, float b1, float b2, float eps,
                                float* __restrict__ prm, const float* __restrict__ g,
                                float* __restrict__ m, float* __restrict__ v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kP) return;
  const float mi = b1 * m[p] + (1.0f - b1) * g[p];
  const float vi = b2 * v[p] + (1.0f - b2) * g[p] * g[p];
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Standalone BF16 inference of 16-sample tiles through mlp_score_tile; each
// wavefront walks tiles with a grid stride, so the weights it loads (loop
// invariant) stay in registers rather than being read again per tile.
__global__ __launch_bounds__(64) void mlp_infer_kernel(gdg_model_dev md, int n,
                                                       const float* __restrict__ x,
                                                       float* __restrict__ z) {
  const int lane = threadIdx.x;
  const int c = lane & 15, q = lane >> 4;
  for (int t = blockIdx.x; t * 16 < n; t += gridDim.x) {
    const int s = t * 16 + c;
    float f[4], deg = 0.0f;
    for (int j = 0; j < 4; ++j) f[j] = s < n ? x[(long long)s * kIn + 4 * q + j] : 0.0f;
    if (s < n) deg = x[(long long)s * kIn + 16];
    const float out = mlp_score_tile(md, f, deg);
    if (q == 0 && s < n) z[s] = out;
  }
}

}  // namespace

size_t gdg_mlp_grad_work_floats(int n) {
  return (size_t)((n + kChunk - 1) / kChunk) * (kP + 1);
}

hipError_t gdg_launch_mlp_grad(int n, const float* prm, const float* x, const float* y, float* grad,
                               float* loss, float* work, hipStream_t st) {
  const int nb = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(mlp_grad_partial, dim3(nb), dim3(256), 0, st, n, prm, x, y, work);
  hipLaunchKernelGGL(mlp_grad_reduce, dim3((kP + 1 + 255) / 256), dim3(256), 0, st, nb, work, grad,
                     loss);
  return hipGetLastError();
}

hipError_t gdg_launch_mlp_forward(int n, const float* prm, const float* x, float* z,
                                  hipStream_t st) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 127) / 128), dim3(128), 0, st, n, prm, x, z);
  return hipGetLastError();
}

hipError_t gdg_launch_mlp_adam(int t, float lr, float b1, float b2, float eps, float* prm,
                               const float* g, float* m, float* v, hipStream_t st) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kP + 255) / 256), dim3(256), 0, st, t, lr, b1, b2, eps,
                     prm, g, m, v);
  return hipGetLastError();
}

hipError_t gdg_launch_mlp_infer(const gdg_model_dev& md, int n, const float* x, float* z,
                                hipStream_t st) {
  // 24 wavefronts per CU on 256 CUs (as many as its registers allow), or one
  // per tile if fewer
  const int tiles = (n + 15) / 16;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(tiles < 6144 ? tiles : 6144), dim3(64), 0, st, md, n,
                     x, z);
  return hipGetLastError();
}
