// Mapping support (Sec. 3.2, mapping loss Eqs. 7-8): the scale regulariser
// and a fused Adam step over the Gaussians' parameter groups.
//
// Regulariser.  L_reg = (1/N) sum_i |s_i - sbar|_1 with s_i = exp(log-scale
// i) (three components), sbar their mean over the N Gaussians, |.|_1 summed
// over the components.  Its gradient with respect to component k of s_i is
// (1/N) (sign(s_ik - sbar_k) - (1/N) sum_j sign(s_jk - sbar_k)) (the mean
// moves with every s_i; sign(0) = 0), times s_ik for the log-scale.  Three
// launches: per-block sums of s; per-block sign and absolute-value sums
// around sbar; the gradient.  Block partials are FP64 and every later block
// adds them in the same order, so the result does not depend on timing.
//
// Adam.  Up to kAdamGroups (parameter, gradient, first moment, second
// moment, length, rate) groups in one launch; FP32 throughout, bias
// corrections from the host.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsff_internal.h"

namespace gsff {
namespace {

constexpr int kRegBlock = 256;
constexpr int kAdamGroups = 8;

__device__ __forceinline__ double block_sum_f64(double v, double* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wv = threadIdx.x >> 6;
  __syncthreads();  // s_red may hold the previous sum
  if ((threadIdx.x & 63) == 0) s_red[wv] = v;
  __syncthreads();
  return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// sum over the blocks' partials [nb][stride] of column k, in block order
__device__ __forceinline__ double partial_total(const double* part, int nb, int stride, int k,
                                                double* s_red) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRegBlock) v += part[(int64_t)b * stride + k];
  return block_sum_f64(v, s_red);
}

__global__ __launch_bounds__(kRegBlock) void k_reg_sum(const float* __restrict__ log_scales,
                                                       int64_t P, double* __restrict__ part) {
  __shared__ double s_red[4];
  const int64_t i = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
  for (int k = 0; k < 3; ++k) {
    const double s = i < P ? (double)expf(log_scales[k * P + i]) : 0.0;
    const double t = block_sum_f64(s, s_red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 3 + k] = t;
  }
}

__global__ __launch_bounds__(kRegBlock) void k_reg_sign(const float* __restrict__ log_scales,
                                                        int64_t P, const double* __restrict__ part1,
                                                        double* __restrict__ part2) {
  __shared__ double s_red[4];
  const int nb = gridDim.x;
  const int64_t i = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
  for (int k = 0; k < 3; ++k) {
    const double mean = partial_total(part1, nb, 3, k, s_red) / (double)P;
    double sg = 0.0, ab = 0.0;
    if (i < P) {
      const double d = (double)expf(log_scales[k * P + i]) - mean;
      sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
      ab = fabs(d);
    }
    const double ts = block_sum_f64(sg, s_red);
    const double ta = block_sum_f64(ab, s_red);
    if (threadIdx.x == 0) {
      part2[(int64_t)blockIdx.x * 6 + k] = ts;
      part2[(int64_t)blockIdx.x * 6 + 3 + k] = ta;
    }
  }
}

__global__ __launch_bounds__(kRegBlock) void k_reg_grad(const float* __restrict__ log_scales,
                                                        int64_t P, const double* __restrict__ part1,
                                                        const double* __restrict__ part2,
                                                        float lambda, float* __restrict__ grad,
                                                        float* __restrict__ loss,
                                                        int accumulate) {
  __shared__ double s_red[4];
  const int nb = gridDim.x;
  const int64_t i = (int64_t)blockIdx.x * kRegBlock + threadIdx.x;
  const double invN = 1.0 / (double)P;
  double labs = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double mean = partial_total(part1, nb, 3, k, s_red) * invN;
    const double ssum = partial_total(part2, nb, 6, k, s_red);
    if (blockIdx.x == 0) labs += partial_total(part2, nb, 6, 3 + k, s_red);
    if (i < P && grad) {
      const float ls = log_scales[k * P + i];
      const double s = (double)expf(ls);
      const double d = s - mean;
      const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
      const float gk = (float)((double)lambda * invN * (sg - ssum * invN) * s);
      float* dst = grad + k * P + i;
      *dst = accumulate ? *dst + gk : gk;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    const float l = (float)((double)lambda * invN * labs);
    *loss = accumulate ? *loss + l : l;
  }
}

struct AdamGroup {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
};
struct AdamArgs {
  AdamGroup grp[kAdamGroups];
  int64_t end[kAdamGroups];  // cumulative lengths
  int ngroups;
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t total = a.end[a.ngroups - 1];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    int q = 0;
    while (e >= a.end[q]) ++q;  // a handful of groups
    const AdamGroup& G = a.grp[q];
    const int64_t i = e - (q > 0 ? a.end[q - 1] : 0);
    const float g = G.g[i];
    const float m = b1 * G.m[i] + (1.f - b1) * g;
    const float v = b2 * G.v[i] + (1.f - b2) * g * g;
    G.m[i] = m;
    G.v[i] = v;
    G.p[i] -= G.lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

}  // namespace
}  // namespace gsff

using namespace gsff;

extern "C" {

gsff_status gsff_scale_reg(const float* log_scales, int64_t P, float lambda, float* workspace,
                           size_t ws_bytes, float* grad_log_scales, float* loss,
                           int32_t accumulate, void* stream) {
  if (P <= 0 || !log_scales || !workspace || !std::isfinite(lambda))
    return GSFF_ERR_INVALID_ARGUMENT;
  if (((uintptr_t)workspace & 7u) != 0) return GSFF_ERR_INVALID_ARGUMENT;
  const int64_t nb = (P + kRegBlock - 1) / kRegBlock;
  if (nb > 0x7FFFFFFF || ws_bytes < (size_t)nb * 9 * sizeof(double))
    return GSFF_ERR_INVALID_ARGUMENT;
  double* part1 = (double*)workspace;
  double* part2 = part1 + nb * 3;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_reg_sum, dim3((unsigned)nb), dim3(kRegBlock), 0, s, log_scales, P, part1);
  hipLaunchKernelGGL(k_reg_sign, dim3((unsigned)nb), dim3(kRegBlock), 0, s, log_scales, P,
                     (const double*)part1, part2);
  hipLaunchKernelGGL(k_reg_grad, dim3((unsigned)nb), dim3(kRegBlock), 0, s, log_scales, P,
                     (const double*)part1, (const double*)part2, lambda, grad_log_scales, loss,
                     (int)accumulate);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

gsff_status gsff_scale_reg_workspace_size(int64_t P, size_t* bytes) {
  if (P < 0 || !bytes) return GSFF_ERR_INVALID_ARGUMENT;
  *bytes = (size_t)((P + kRegBlock - 1) / kRegBlock) * 9 * sizeof(double);
  return GSFF_OK;
}

gsff_status gsff_adam_step(const gsff_adam_group* groups, int32_t ngroups, int32_t step,
                           float beta1, float beta2, float eps, void* stream) {
  if (!groups || ngroups < 1 || ngroups > kAdamGroups || step < 1)
    return GSFF_ERR_INVALID_ARGUMENT;
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return GSFF_ERR_INVALID_ARGUMENT;
  AdamArgs a{};
  int64_t total = 0;
  for (int q = 0; q < ngroups; ++q) {
    const gsff_adam_group& G = groups[q];
    if (G.n < 0 || (G.n > 0 && (!G.param || !G.grad || !G.m || !G.v)) || !std::isfinite(G.lr))
      return GSFF_ERR_INVALID_ARGUMENT;
    a.grp[q] = AdamGroup{G.param, G.grad, G.m, G.v, G.n, G.lr};
    total += G.n;
    a.end[q] = total;
  }
  a.ngroups = ngroups;
  if (total == 0) return GSFF_OK;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  const int64_t blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a, beta1,
                     beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

}  // extern "C"
