// LDS bandwidth probe: the measured LDS rates that the decode kernel's LDS
// roofline is set against. Every workgroup (256 threads) fills 32 KiB (or
// 16 KiB, for more resident workgroups per CU) of LDS, then each thread
// streams `reps` rounds of up to 16 accesses of one width (4, 8 or 16 bytes
// per lane) to distinct addresses, lanes on consecutive addresses so that no
// two lanes of a wavefront share a bank in one access. Reads are summed into
// a value written once per thread, so none can be dropped.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kProbeBytes = 32 * 1024;
constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ float as_sum(const T& v);
template <>
__device__ __forceinline__ float as_sum<float>(const float& v) { return v; }
template <>
__device__ __forceinline__ float as_sum<float2>(const float2& v) { return v.x + v.y; }
template <>
__device__ __forceinline__ float as_sum<float4>(const float4& v) { return v.x + v.y + v.z + v.w; }

template <typename T, int kBytes>
__global__ __launch_bounds__(kThreads) void lds_read_kernel(int reps, float* __restrict__ sink) {
  __shared__ __align__(16) unsigned char buf[kBytes];
  const int tid = threadIdx.x;
  for (int i = tid * 4; i < kBytes; i += kThreads * 4)
    *(float*)(buf + i) = (float)(i & 1023) * 1e-3f;
  __syncthreads();
  constexpr int kW = (int)sizeof(T);
  constexpr int kSlots = kBytes / (kThreads * kW);   // per-thread slots in the buffer
  constexpr int kPer = kSlots < 16 ? kSlots : 16;         // distinct accesses per round
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int slot = (r + j) % kSlots;
      const T v = *(const T*)(buf + (slot * kThreads + tid) * kW);
      acc[j & 3] += as_sum<T>(v);
    }
  }
  sink[blockIdx.x * kThreads + tid] = acc[0] + acc[1] + acc[2] + acc[3];
}

__global__ __launch_bounds__(kThreads) void lds_write_kernel(int reps, float* __restrict__ sink) {
  __shared__ __align__(16) float buf[kProbeBytes / 4];
  const int tid = threadIdx.x;
  constexpr int kSlots = kProbeBytes / (kThreads * 4);
  float v = (float)tid;
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int slot = (r + j) % kSlots;
      buf[slot * kThreads + tid] = v;
      v += 1.0f;
    }
  }
  __syncthreads();
  sink[blockIdx.x * kThreads + tid] = buf[(tid * 7) % (kProbeBytes / 4)];
}

}  // namespace

// mode 0: 4-byte reads, 1: 8-byte reads, 2: 16-byte reads, 3: 4-byte writes,
// all on 32 KiB per workgroup; 4, 5, 6: the reads of 0, 1, 2 on 16 KiB.
// Launches n_blocks workgroups of 256 threads on `stream`; sink holds
// n_blocks * 256 floats. lds_probe_bytes gives the LDS bytes one launch moves.
// Returns 0, or -1 for a bad argument or a failed launch.
extern "C" int lds_probe_launch(int mode, int n_blocks, int reps, float* sink, void* stream) {
  if (n_blocks < 1 || reps < 1 || !sink || mode < 0 || mode > 6) return -1;
  hipStream_t st = (hipStream_t)stream;
  constexpr int B = kProbeBytes, H = kProbeBytes / 2;
  const dim3 g(n_blocks), b(kThreads);
  switch (mode) {
    case 0: hipLaunchKernelGGL((lds_read_kernel<float, B>), g, b, 0, st, reps, sink); break;
    case 1: hipLaunchKernelGGL((lds_read_kernel<float2, B>), g, b, 0, st, reps, sink); break;
    case 2: hipLaunchKernelGGL((lds_read_kernel<float4, B>), g, b, 0, st, reps, sink); break;
    case 3: hipLaunchKernelGGL(lds_write_kernel, g, b, 0, st, reps, sink); break;
    case 4: hipLaunchKernelGGL((lds_read_kernel<float, H>), g, b, 0, st, reps, sink); break;
    case 5: hipLaunchKernelGGL((lds_read_kernel<float2, H>), g, b, 0, st, reps, sink); break;
    default: hipLaunchKernelGGL((lds_read_kernel<float4, H>), g, b, 0, st, reps, sink); break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" double lds_probe_bytes(int mode, int n_blocks, int reps) {
  const int width = (mode == 1 || mode == 5) ? 8 : (mode == 2 || mode == 6) ? 16 : 4;
  const int slots = (mode >= 4 ? kProbeBytes / 2 : kProbeBytes) / (kThreads * width);
  const int per = mode == 3 ? 16 : (slots < 16 ? slots : 16);
  return (double)n_blocks * kThreads * per * reps * width;
}
