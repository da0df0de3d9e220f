// Microbenchmarks that measure the roofline denominators on the GPU the
// library runs on (used by the benchmark, not by the rendering path):
//
//  - LDS read delivery: every lane of 256-thread workgroups reads 16-byte
//    vectors (ds_read_b128) from a 64 KiB LDS array, sixteen independent reads
//    per step, either at per-lane distinct, bank-conflict-free addresses or
//    at one wave-uniform (broadcast) address -- the pattern the compositing
//    kernels use for staged Gaussian records.  Lane-delivered bytes = lanes x
//    reads x 16.
//  - HBM streaming read: a grid-stride read of a large buffer with 16-byte
//    loads, summed so the loads stay live.
//
// Each call enqueues one kernel on `stream`; the caller times it.  The sink
// buffer only receives a value when an impossible sum occurs (it keeps the
// reads alive) and must hold 256 x blocks floats.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kLdsVec = 4096;  // float4 entries: 64 KiB

template <int BROADCAST>
__global__ __launch_bounds__(256) void k_probe_lds(float* __restrict__ sink, int steps) {
  __shared__ float4 buf[kLdsVec];
  for (int i = threadIdx.x; i < kLdsVec; i += 256)
    buf[i] = make_float4((float)i, (float)(i + 1), (float)(i + 2), (float)(i + 3));
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = BROADCAST ? 16 * wave : lane + 64 * wave;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int it = 0; it < steps; ++it) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = BROADCAST ? ((base + u + 16 * it) & (kLdsVec - 1))
                                : ((base + 256 * u + 64 * it) & (kLdsVec - 1));
      const float4 v = buf[idx];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
  }
  if (acc.x == -1.f) sink[blockIdx.x * 256 + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

__global__ __launch_bounds__(256) void k_probe_hbm(const float4* __restrict__ src, int64_t n,
                                                   float* __restrict__ sink) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const float4 v = src[i];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  if (acc.x == -1.f) sink[blockIdx.x * 256 + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" {

// LDS: `blocks` workgroups of 256 lanes, `steps` x 16 reads of 16 bytes each;
// broadcast = 0 per-lane addresses, 1 one address per wave.  Returns 0, or -1
// for a bad argument.
int gsff_probe_lds(int broadcast, int blocks, int steps, float* sink, void* stream) {
  if (blocks < 1 || steps < 1 || !sink) return -1;
  if (broadcast)
    hipLaunchKernelGGL(k_probe_lds<1>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, sink,
                       steps);
  else
    hipLaunchKernelGGL(k_probe_lds<0>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, sink,
                       steps);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// HBM: read n16 16-byte vectors of src with `blocks` workgroups of 256.
int gsff_probe_hbm_read(const void* src, int64_t n16, int blocks, float* sink, void* stream) {
  if (!src || n16 < 1 || blocks < 1 || !sink) return -1;
  hipLaunchKernelGGL(k_probe_hbm, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (const float4*)src, n16, sink);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
