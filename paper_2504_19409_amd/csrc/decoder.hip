// Learned 1x1 feature decoder on BF16 matrix cores (gfx950 MFMA).
//
// The paper supervises the rendered N-channel feature map against 512-channel
// foundation-model features through a lift o(.) with an L1 loss (Eq. 11).
// Here o(.) is a per-pixel MLP  Y = GELU(X W1 + b1) W2 + b2  with
// X: 16 latent channels, 128 hidden units, 512 outputs, GELU in its tanh form.
// All maps are planar [channels, pixels], the layout of the rasterizer's
// feature output, so the decoder reads the rendered latent map as is.
//
// MFMA v_mfma_f32_32x32x16_bf16 (lane l, g = l / 32, i = l % 32):
//   A[i][8g + t], B[8g + t][i] for t = 0..7 (eight bf16 per lane),
//   D: acc[r] = D[8 (r/4) + 4g + r%4][i].
// Every product is computed transposed -- pixels along N -- so a lane always
// holds one pixel.  The D registers of one product then serve directly as
// the B operand of the next one if the reduction index is visited in the
// order the registers hold it: K-step s of a dimension split in 32-blocks
// covers, for k-slot (g, t), index
//   pi(s, g, t) = 32 (s/2) + 16 (s%2) + 8 (t/4) + 4g + t%4.
// The matching A operands are bf16 weight copies stored in that permuted
// order (k_dec_prepare), one 16-byte load per lane and step.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <mutex>

#include "gsff_internal.h"

namespace gsff {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLat = 16, kHid = 128, kOut = 512;
constexpr int kWgradGroups = 128;     // split-K workgroups of the weight-gradient GEMMs
constexpr int kWgradWaves = 8;
// column blocks per workgroup of the two weight-gradient GEMMs, W2 (16 in
// four workgroups) and W1 (4 in one), divide the wave count
static_assert(kWgradWaves % ((kOut / 32) / 4) == 0 && kWgradWaves % (kHid / 32) == 0, "");

__host__ __device__ inline int dec_pi(int s, int g, int t) {
  return 32 * (s / 2) + 16 * (s % 2) + 8 * (t / 4) + 4 * g + (t % 4);
}

// ---- decoder workspace layout (bytes, 256-aligned) ----
struct DecLayout {
  int64_t npx = 0, npad = 0, nblk = 0;
  uint64_t w1t = 0, w1p = 0, w2tp = 0, w2p = 0, xbuf = 0, hbuf = 0, dzbuf = 0, dys = 0,
           part2 = 0, part1 = 0, total = 0;
};

static DecLayout dec_layout(int64_t npx) {
  DecLayout L;
  L.npx = npx;
  L.nblk = (npx + 31) / 32;
  // the training kernel's buffers cover every pixel its workgroups (128
  // pixels each) are launched for, so none of its stores needs a test
  L.npad = (npx + 127) / 128 * 128;
  uint64_t o = 0;
  auto take = [&](uint64_t b) {
    const uint64_t at = o;
    o = align_up(o + b, 256);
    return at;
  };
  L.w1t = take(2ull * kHid * kLat);
  L.w1p = take(2ull * 32 * 8 * 16);
  L.w2tp = take(2ull * kOut * 8 * 16);
  L.w2p = take(2ull * kHid * 32 * 16);
  L.xbuf = take(2ull * kLat * L.npad);
  L.hbuf = take(2ull * kHid * L.npad);
  L.dzbuf = take(2ull * kHid * L.npad);
  L.dys = take(1ull * kOut * L.npad);
  L.part2 = take(4ull * kWgradGroups * (kHid * kOut + kOut));
  L.part1 = take(4ull * kWgradGroups * (32 * kHid + kHid));
  L.total = o;
  return L;
}

// GELU in its tanh form, 0.5 z (1 + tanh(u)) with u = sqrt(2/pi) (z + 0.044715 z^3),
// evaluated as the equal z / (1 + exp(-2u)): one exp2 and one hardware
// reciprocal (1 ulp each) with the constants folded into the polynomial; at
// the ends 1 / inf = 0 and 1 / 1 = 1, so the limits -0 and z are exact
__device__ __forceinline__ float gelu_f(float z) {
  const float a = z * fmaf(z * z, -2.f * 1.4426950408889634f * 0.7978845608028654f * 0.044715f,
                           -2.f * 1.4426950408889634f * 0.7978845608028654f);  // -2u log2(e)
  return z * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(a));
}

// derivative of the tanh form; tanh(u) = 1 - 2 / (exp(2u) + 1)
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float u = 0.7978845608028654f * (z + 0.044715f * z * z * z);
  const float t = 1.f - 2.f * __builtin_amdgcn_rcpf(__expf(2.f * u) + 1.f);
  const float du = 0.7978845608028654f * (1.f + 3.f * 0.044715f * z * z);
  return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * du;
}

__device__ __forceinline__ bf16x8 load8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// --------------------------------------------------------- weight copies ----

// bf16 copies of the FP32 master weights in the operand orders above:
//   w1t [128 hid][16 k]           A of layer 1 (natural k order)
//   w1p [32 rows][8 s][2 g][8 t]  A of dX^T = W1 dZ^T (rows >= 16 zero)
//   w2tp[512 ch][8 s][2 g][8 t]   A of Y^T = W2^T H^T
//   w2p [128 hid][32 s][2 g][8 t] A of dH^T = W2 dY^T
__global__ __launch_bounds__(256) void k_dec_prepare(const float* __restrict__ W1,
                                                     const float* __restrict__ W2,
                                                     __bf16* w1t, __bf16* w1p, __bf16* w2tp,
                                                     __bf16* w2p) {
  const int n1 = kHid * kLat, n2 = 32 * 8 * 16, n3 = kOut * 8 * 16, n4 = kHid * 32 * 16;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n1 + n2 + n3 + n4; e += gridDim.x * 256) {
    if (e < n1) {
      const int h = e / kLat, k = e % kLat;
      w1t[e] = (__bf16)W1[k * kHid + h];
    } else if (e < n1 + n2) {
      const int q = e - n1;
      const int row = q / 128, s = (q / 16) % 8, g = (q / 8) % 2, t = q % 8;
      w1p[q] = row < kLat ? (__bf16)W1[row * kHid + dec_pi(s, g, t)] : (__bf16)0.f;
    } else if (e < n1 + n2 + n3) {
      const int q = e - n1 - n2;
      const int ch = q / 128, s = (q / 16) % 8, g = (q / 8) % 2, t = q % 8;
      w2tp[q] = (__bf16)W2[dec_pi(s, g, t) * kOut + ch];
    } else {
      const int q = e - n1 - n2 - n3;
      const int h = q / 512, s = (q / 16) % 32, g = (q / 8) % 2, t = q % 8;
      w2p[q] = (__bf16)W2[h * kOut + dec_pi(s, g, t)];
    }
  }
}

// The eight bf16 of K-step s (within a 32-block) from a D register block.
__device__ __forceinline__ bf16x8 regs_to_b(const f32x16& d, int half) {
  bf16x8 b;
#pragma unroll
  for (int t = 0; t < 8; ++t) b[t] = (__bf16)d[8 * half + t];
  return b;
}

// ------------------------------------------------------------- forward -----

// One wave decodes NPB blocks of 32 pixels.  The second layer takes the
// hidden activations as the A operand (pixels along M) and the weights as B,
// so lane (g, i) ends with output channel 32 c + i of pixels
// 8 k + 4 g .. 8 k + 4 g + 3 (k = 0..3) of each block.  The weights of output
// block c (32 channels x 128 hidden, 8 KB) are copied once per workgroup into
// a padded LDS tile, one block ahead (each thread 32 bytes, loaded while the
// current block is multiplied), and all four waves read their fragments from
// it: a quarter of the cache traffic of per-wave loads, and no register
// double buffer, so three waves fit on a SIMD.  ROWS (rows of Y 16-byte
// aligned): the wave's 32 channels x 32 NPB pixels pass through LDS, and every
// store instruction writes 16 bytes per lane as whole row segments (eight
// lanes per row); otherwise one element per store.
template <int NPB, typename OT, bool ROWS>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(3)))
void k_dec_forward(const __bf16* __restrict__ X, const float* __restrict__ b1,
                   const float* __restrict__ b2, const __bf16* __restrict__ w1t,
                   const __bf16* __restrict__ w2tp, OT* __restrict__ Y, int64_t npx) {
  constexpr int PXW = 32 * NPB;                    // pixels per wave
  constexpr int VEC = 16 / (int)sizeof(OT);        // elements per 16-byte store
  constexpr int STRIDE = PXW + VEC;                // LDS row pitch: 16-byte rows, banks staggered
  constexpr int WP = kHid + 8;                     // weight row pitch (272 bytes): 16 lanes, 16 bank groups
  __shared__ __attribute__((aligned(16))) OT s_y[ROWS ? 4 : 1][ROWS ? 32 : 1][ROWS ? STRIDE : 1];
  __shared__ __attribute__((aligned(16))) __bf16 s_w[2][32 * WP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 5, i = lane & 31, wv = tid >> 6;
  const int64_t wave = (int64_t)blockIdx.x * 4 + wv;
  const int64_t wbase = wave * PXW;
  __shared__ __attribute__((aligned(16))) float s_b1[kHid];
  if (tid < kHid) s_b1[tid] = b1[tid];
  __syncthreads();
  // weight tile copy: thread tid moves bytes 32 (tid % 8) .. + 31 of row tid / 8
  const int wr = tid >> 3, wc = (tid & 7) * 16;
  u32x4 wt0, wt1;
  auto wload = [&](int c) {
    const __bf16* src = w2tp + (int64_t)(32 * c + wr) * kHid + wc;
    wt0 = *reinterpret_cast<const u32x4*>(src);
    wt1 = *reinterpret_cast<const u32x4*>(src + 8);
  };
  auto wstore = [&](int buf) {
    __bf16* d = &s_w[buf][wr * WP + wc];
    *reinterpret_cast<u32x4*>(d) = wt0;
    *reinterpret_cast<u32x4*>(d + 8) = wt1;
  };
  bf16x8 hf[NPB][8];
#pragma unroll
  for (int q = 0; q < NPB; ++q) {
    const int64_t px = wbase + 32 * q + i;
    const bool ok = px < npx;
    bf16x8 xb;
#pragma unroll
    for (int t = 0; t < 8; ++t) xb[t] = ok ? X[(int64_t)(8 * g + t) * npx + px] : (__bf16)0.f;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      f32x16 z = {};
      z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(w1t + (32 * h + i) * kLat + 8 * g), xb, z,
                                                  0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) z[r] = gelu_f(z[r] + s_b1[32 * h + 8 * (r / 4) + 4 * g + r % 4]);
      hf[q][2 * h] = regs_to_b(z, 0);
      hf[q][2 * h + 1] = regs_to_b(z, 1);
    }
  }
  wload(0);
  wstore(0);
  __syncthreads();
  const bool full = wbase + PXW <= npx;  // uniform: every pixel of the wave in range
#pragma unroll 1
  for (int c = 0; c < kOut / 32; ++c) {
    if (c + 1 < kOut / 32) wload(c + 1);
    const float bias = b2[32 * c + i];
    const __bf16* wrow = &s_w[c & 1][i * WP + 8 * g];
    f32x16 acc[NPB];
#pragma unroll
    for (int q = 0; q < NPB; ++q) acc[q] = f32x16{};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const bf16x8 w = *reinterpret_cast<const bf16x8*>(wrow + 16 * s);
#pragma unroll
      for (int q = 0; q < NPB; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hf[q][s], w, acc[q], 0, 0, 0);
    }
    if constexpr (ROWS) {
      // the wave's tile: row = channel i, pixels 32 q + 8 k + 4 g .. +3
#pragma unroll
      for (int q = 0; q < NPB; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          OT* d = &s_y[wv][i][32 * q + 8 * k + 4 * g];
#pragma unroll
          for (int t = 0; t < 4; ++t) d[t] = (OT)(acc[q][4 * k + t] + bias);
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      // lanes in groups of PXW / VEC per row, rows in turn
      constexpr int LPR = PXW / VEC;  // lanes per row
      constexpr int RPI = 64 / LPR;   // rows per store instruction
#pragma unroll
      for (int r0 = 0; r0 < 32; r0 += RPI) {
        const int row = r0 + lane / LPR, col = (lane % LPR) * VEC;
        const u32x4 v = *reinterpret_cast<const u32x4*>(&s_y[wv][row][col]);
        const int64_t p0 = wbase + col;
        OT* dst = Y + (int64_t)(32 * c + row) * npx + p0;
        if (full) {
          // one 16-byte store, nontemporal: the map streams past the caches
          __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(dst));
        } else {
          const OT* e = reinterpret_cast<const OT*>(&v);
#pragma unroll
          for (int t = 0; t < VEC; ++t)
            if (p0 + t < npx) dst[t] = e[t];
        }
      }
    } else {
      OT* row = Y + (int64_t)(32 * c + i) * npx;
#pragma unroll
      for (int q = 0; q < NPB; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int64_t p0 = wbase + 32 * q + 8 * k + 4 * g;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (p0 + t < npx) row[p0 + t] = (OT)(acc[q][4 * k + t] + bias);
        }
    }
    // the other weight buffer was last read before the previous barrier; the
    // barrier below also orders this wave's tile reads before the next writes
    if (c + 1 < kOut / 32) wstore((c + 1) & 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------- train step -----

// Fused forward, L1 against the target and the backward to the latent:
// per 32-pixel wave, Z, H and Y by MFMA; dY = sign(Y - T) (its sign is kept
// in int8 for the weight gradients, the scale applied to FP32 results);
// dH^T = W2 dY^T accumulated over the 16 output blocks as they are produced;
// dZ = scale dH GELU'(Z); dX^T = W1 dZ^T.  H and dZ are stored in bf16 for
// the weight-gradient GEMMs.  Pixels beyond npx contribute zeros.
__global__ __launch_bounds__(256) void k_dec_train(
    const __bf16* __restrict__ X, const float* __restrict__ b1, const float* __restrict__ b2,
    const __bf16* __restrict__ T, const __bf16* __restrict__ w1t, const __bf16* __restrict__ w1p,
    const __bf16* __restrict__ w2tp, const __bf16* __restrict__ w2p, __bf16* __restrict__ xbuf,
    __bf16* __restrict__ hbuf, __bf16* __restrict__ dzbuf, int8_t* __restrict__ dys,
    float* __restrict__ dX, float* loss, float scale, int64_t npx, int64_t npad) {
  __shared__ float s_loss[4];
  __shared__ float s_b1[kHid], s_b2[kOut];  // biases: one LDS read per element, no global
  // the targets of one 32-channel output block for the workgroup's 128
  // pixels, double-buffered: block c + 1's are loaded with 16-byte loads
  // while block c is computed
  constexpr int TP = 128 + 8;  // row pitch
  __shared__ __attribute__((aligned(16))) __bf16 s_t[2][32][TP];
  for (int e = threadIdx.x; e < kHid; e += 256) s_b1[e] = b1[e];
  for (int e = threadIdx.x; e < kOut; e += 256) s_b2[e] = b2[e];
  const int64_t pw = (int64_t)blockIdx.x * 128;  // the workgroup's first pixel
  const int trow = threadIdx.x >> 3, tseg = (threadIdx.x & 7) * 16;
  // whole 16-byte runs when every pixel of the workgroup is in range and rows
  // are 16-byte aligned (uniform); otherwise one clamped element at a time
  const bool tvec =
      (npx % 8) == 0 && pw + 128 <= npx && (reinterpret_cast<uintptr_t>(T) & 15u) == 0u;
  u32x4 tl[2];
  auto load_tile = [&](int cc) {
    const int64_t src = (int64_t)(32 * cc + trow) * npx + pw + tseg;
    if (tvec) {
      tl[0] = *reinterpret_cast<const u32x4*>(T + src);
      tl[1] = *reinterpret_cast<const u32x4*>(T + src + 8);
    } else {
      uint16_t e[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t p = min(pw + tseg + j, npx - 1);
        e[j] = reinterpret_cast<const uint16_t*>(T)[(int64_t)(32 * cc + trow) * npx + p];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          tl[q][k] = (uint32_t)e[8 * q + 2 * k] | ((uint32_t)e[8 * q + 2 * k + 1] << 16);
    }
  };
  auto store_tile = [&](int buf) {
    *reinterpret_cast<u32x4*>(&s_t[buf][trow][tseg]) = tl[0];
    *reinterpret_cast<u32x4*>(&s_t[buf][trow][tseg + 8]) = tl[1];
  };
  // the block's weight operands the same way: W2^T rows 32 c .. 32 c + 31 in
  // their K-step order, and the W2 columns of K-steps 2 c, 2 c + 1 (rows
  // padded so the lanes' 16-byte reads fall in distinct banks)
  constexpr int WTP = 128 + 8, WP = 32 + 8;
  __shared__ __attribute__((aligned(16))) __bf16 s_w2t[2][32 * WTP];
  __shared__ __attribute__((aligned(16))) __bf16 s_w2[2][kHid * WP];
  u32x4 wl[4];
  const int wh = threadIdx.x >> 1, we = (threadIdx.x & 1) * 16;
  auto load_w = [&](int cc) {
    const __bf16* a = w2tp + ((int64_t)32 * cc * 128 + threadIdx.x * 16);
    wl[0] = *reinterpret_cast<const u32x4*>(a);
    wl[1] = *reinterpret_cast<const u32x4*>(a + 8);
    const __bf16* bp = w2p + ((int64_t)(wh * 32 + 2 * cc) * 16 + we);
    wl[2] = *reinterpret_cast<const u32x4*>(bp);
    wl[3] = *reinterpret_cast<const u32x4*>(bp + 8);
  };
  auto store_w = [&](int buf) {
    __bf16* a = &s_w2t[buf][trow * WTP + tseg];
    *reinterpret_cast<u32x4*>(a) = wl[0];
    *reinterpret_cast<u32x4*>(a + 8) = wl[1];
    __bf16* bp = &s_w2[buf][wh * WP + we];
    *reinterpret_cast<u32x4*>(bp) = wl[2];
    *reinterpret_cast<u32x4*>(bp + 8) = wl[3];
  };
  load_tile(0);
  load_w(0);
  store_tile(0);
  store_w(0);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 5, i = lane & 31;
  const int64_t px = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + i;
  const bool ok = px < npx;
  // loads read a pixel in range and the value is dropped where !ok, so no
  // load sits in a branch (a branch around a load makes the compiler wait
  // for every load in flight where the paths join); every launched pixel is
  // below npad, so the stores need no test either
  const int64_t pxc = ok ? px : npx - 1;
  bf16x8 xb;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 v = X[(int64_t)(8 * g + t) * npx + pxc];
    xb[t] = ok ? v : (__bf16)0.f;
    xbuf[(int64_t)(8 * g + t) * npad + px] = xb[t];  // zero-padded copy for dW1
  }
  // (the pre-activations are computed again for the GELU derivative at the
  // end instead of being held in 64 registers across the output blocks)
  bf16x8 hf[8];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    f32x16 z = {};
    z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(w1t + (32 * h + i) * kLat + 8 * g), xb, z, 0,
                                                0, 0);
    f32x16 hv;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int hid = 32 * h + 8 * (r / 4) + 4 * g + r % 4;
      z[r] += s_b1[hid];
      hv[r] = ok ? gelu_f(z[r]) : 0.f;
      hbuf[(int64_t)hid * npad + px] = (__bf16)hv[r];
    }
    hf[2 * h] = regs_to_b(hv, 0);
    hf[2 * h + 1] = regs_to_b(hv, 1);
  }
  f32x16 dh[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) dh[h] = f32x16{};
  float lsum = 0.f;
  const int wcol = (threadIdx.x >> 6) * 32 + i;  // this lane's pixel in the tile
  for (int c = 0; c < kOut / 32; ++c) {
    load_tile(min(c + 1, kOut / 32 - 1));  // (the last block reloads itself)
    load_w(min(c + 1, kOut / 32 - 1));
    const __bf16* wt = &s_w2t[c & 1][i * WTP + 8 * g];
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
          *reinterpret_cast<const bf16x8*>(wt + 16 * s), hf[s], acc, 0, 0, 0);
    f32x16 sg;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ch = 32 * c + 8 * (r / 4) + 4 * g + r % 4;
      const float tv = (float)s_t[c & 1][8 * (r / 4) + 4 * g + r % 4][wcol];
      const float d = ok ? acc[r] + s_b2[ch] - tv : 0.f;
      lsum += fabsf(d);
      const float sv = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      sg[r] = sv;
      dys[(int64_t)ch * npad + px] = (int8_t)sv;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const bf16x8 b = regs_to_b(sg, e);
#pragma unroll
      for (int h = 0; h < 4; ++h)
        dh[h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            *reinterpret_cast<const bf16x8*>(&s_w2[c & 1][(32 * h + i) * WP + 16 * e + 8 * g]), b,
            dh[h], 0, 0, 0);
    }
    store_tile((c + 1) & 1);
    store_w((c + 1) & 1);
    __syncthreads();  // the next block's targets are in; this block's are read
  }
  bf16x8 dzf[8];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    f32x16 z = {};
    z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(w1t + (32 * h + i) * kLat + 8 * g), xb, z, 0,
                                                0, 0);
    f32x16 dz;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int hid = 32 * h + 8 * (r / 4) + 4 * g + r % 4;
      dz[r] = ok ? scale * dh[h][r] * gelu_grad_f(z[r] + s_b1[hid]) : 0.f;
      dzbuf[(int64_t)hid * npad + px] = (__bf16)dz[r];
    }
    dzf[2 * h] = regs_to_b(dz, 0);
    dzf[2 * h + 1] = regs_to_b(dz, 1);
  }
  f32x16 dx = {};
#pragma unroll
  for (int s = 0; s < 8; ++s)
    dx = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load8(w1p + (i * 8 + s) * 16 + 8 * g), dzf[s], dx,
                                                 0, 0, 0);
  if (ok) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {  // rows 8(r/4) + 4g + r%4 < 16
      const int k = 8 * (r / 4) + 4 * g + r % 4;
      dX[(int64_t)k * npx + px] = dx[r];
    }
  }
  if (loss) {
    float v = lsum;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) s_loss[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float t = (s_loss[0] + s_loss[1]) + (s_loss[2] + s_loss[3]);
      if (t != 0.f) unsafeAtomicAdd(loss, t * scale);
    }
  }
}

// -------------------------------------------------- weight-gradient GEMM ----

// part[wg][m][n] = sum over this workgroup's pixel range of A[m][k] B[n][k]
// and part[wg][M*N + n] = sum_k B[n][k].  A: bf16 [rows >= 32 MB][ld], rows
// >= m_valid read as zero; B: bf16 or int8 [N][ld].  Output blocks (mb, nb)
// are dealt round-robin to the 8 waves.
__device__ __forceinline__ bf16x8 load_b8(const __bf16* p) { return load8(p); }
__device__ __forceinline__ bf16x8 load_b8(const int8_t* p) {
  const int2 v = *reinterpret_cast<const int2*>(p);
  bf16x8 b;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    b[t] = (__bf16)(float)(int8_t)((v.x >> (8 * t)) & 0xFF);
    b[4 + t] = (__bf16)(float)(int8_t)((v.y >> (8 * t)) & 0xFF);
  }
  return b;
}

template <typename BT, int MAXB>
__global__ __launch_bounds__(64 * kWgradWaves) void k_dec_wgrad(
    const __bf16* __restrict__ A, int m_valid, int MB, const BT* __restrict__ B, int NB,
    int64_t ld, int64_t kchunk, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, g = lane >> 5, i = lane & 31;
  const int wv = threadIdx.x >> 6;
  const int M = 32 * MB, N = 32 * NB;
  const int64_t k0 = (int64_t)blockIdx.x * kchunk;
  const int64_t k1 = min(k0 + kchunk, ld);
  f32x16 acc[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) acc[j] = f32x16{};
  float bsum = 0.f;
  // this workgroup's output blocks: every row block of the columns
  // blockIdx.y nbq .. blockIdx.y nbq + nbq - 1, so each workgroup reads only
  // its share of B and every workgroup of a K range all of A (the smaller).
  // nbq divides the wave count, so all of a wave's blocks lie in one column
  // block: its B operand is loaded and converted once per K step, and the
  // wave holds row block 0 (whose column sums give the bias gradient) when
  // wv < nbq
  const int nbq = NB / (int)gridDim.y;
  const int nloc = MB * nbq;
  const int nb = (int)blockIdx.y * nbq + wv % nbq;
  const BT* brow = B + (int64_t)(32 * nb + i) * ld + 8 * g;
  // (waves beyond the workgroup's blocks, W1 only, skip the loop)
  for (int64_t k = wv < nloc ? k0 : k1; k < k1; k += 16) {
    const bf16x8 bb = load_b8(brow + k);
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
      const int l = wv + kWgradWaves * j;
      if (l >= nloc) break;
      const int row = 32 * (l / nbq) + i;
      // (a row in range is read and dropped beyond m_valid: no load in a branch)
      const bf16x8 av = load8(A + (int64_t)min(row, m_valid - 1) * ld + k + 8 * g);
      const bf16x8 a = row < m_valid ? av : bf16x8{};
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[j], 0, 0, 0);
    }
    if (wv < nbq) {
      float sacc = 0.f;
#pragma unroll
      for (int t = 0; t < 8; ++t) sacc += (float)bb[t];
      bsum += sacc;
    }
  }
  float* out = part + (int64_t)blockIdx.x * (M * N + N);
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    const int l = wv + kWgradWaves * j;
    if (l >= nloc) break;
    const int mb = l / nbq;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      out[(32 * mb + 8 * (r / 4) + 4 * g + r % 4) * N + 32 * nb + i] = acc[j][r];
    if (mb == 0) {
      const float v = bsum + __shfl_xor(bsum, 32, 64);
      if (g == 0) out[M * N + 32 * nb + i] = v;
    }
  }
}

// out[e] = scale * sum_wg part[wg][src(e)]; rows >= m_valid of the M x N
// block are dropped, the N bias sums follow the m_valid x N gradient.
// Sum of the split-K partials in a fixed order: 32 outputs per workgroup,
// the groups of each output split into 8 slices of at most 16 consecutive
// groups, whose loads are all in flight at once (a clamped group index, the
// value dropped), then the slice sums added in slice order.
constexpr int kRedCols = 32, kRedSlices = 8, kRedPerSlice = 16;
static_assert(kWgradGroups <= kRedSlices * kRedPerSlice, "split-K groups exceed the reduction");
__global__ __launch_bounds__(256) void k_dec_reduce(const float* __restrict__ part, int groups,
                                                    int M, int N, int m_valid, float scale_w,
                                                    float scale_b, float* __restrict__ dW,
                                                    float* __restrict__ db) {
  __shared__ float s_sum[kRedSlices][kRedCols];
  const int c = threadIdx.x % kRedCols, sl = threadIdx.x / kRedCols;
  const int e = blockIdx.x * kRedCols + c;
  const int nw = m_valid * N;
  const bool ok = e < nw + N;
  const int src = !ok ? 0 : (e < nw ? e : M * N + (e - nw));
  const int64_t stride = (int64_t)M * N + N;
  const int per = (groups + kRedSlices - 1) / kRedSlices;
  const int w0 = sl * per, w1 = min(groups, w0 + per);
  float v[kRedPerSlice];
#pragma unroll
  for (int k = 0; k < kRedPerSlice; ++k)
    v[k] = part[(int64_t)min(w0 + k, groups - 1) * stride + src];
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kRedPerSlice; ++k) acc += w0 + k < w1 ? v[k] : 0.f;
  s_sum[sl][c] = acc;
  __syncthreads();
  if (sl == 0 && ok) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kRedSlices; ++k) t += s_sum[k][c];
    if (e < nw)
      dW[e] = scale_w * t;
    else
      db[e - nw] = scale_b * t;
  }
}


// ---- decode + query (Eqs. 10 and 12) ----------------------------------------
//
// p(l | x) = softmax over the K labels of o(F)(x) . q(l): the dot product with
// the queries is linear, so it folds into the second layer,
//   logits = GELU(X W1 + b1) (W2 Q^T) + b2 Q^T,
// and the 512-channel map is never formed.  FP32 throughout (the folded
// weights are 128 x K padded to a multiple of 16 labels).  Outputs: probabilities [K, n], the label
// of the largest logit (the first of equal ones) [n], and the cross-entropy
// against given labels (Eq. 9), as per-block partials summed in block order.
constexpr int kQueryMaxK = 64;
constexpr int kQueryBlock = 256;

// one wave per folded weight: lanes take 8 of the 512 channels each
__global__ __launch_bounds__(256) void k_query_fold(const float* __restrict__ W2,
                                                    const float* __restrict__ b2,
                                                    const float* __restrict__ Q, int K, int KP,
                                                    float* __restrict__ w2q,
                                                    float* __restrict__ b2q) {
  // w2q [128][KP] (zero past K), b2q [KP]
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= (kHid + 1) * KP) return;  // uniform in the wave
  const int j = e / KP, k = e % KP;
  float acc = 0.f;
  if (k < K) {
    const float* row = j < kHid ? W2 + (int64_t)j * kOut : b2;
    const float* q = Q + (int64_t)k * kOut;
#pragma unroll
    for (int t = 0; t < kOut / 64; ++t) acc = __builtin_fmaf(row[64 * t + lane], q[64 * t + lane], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  }
  if (lane == 0) {
    if (j < kHid)
      w2q[j * KP + k] = acc;
    else
      b2q[k] = acc;
  }
}

typedef float f32x4q __attribute__((ext_vector_type(4)));

template <int NLT>  // label tiles of 16
__global__ __attribute__((amdgpu_flat_work_group_size(kQueryBlock, kQueryBlock),
                          amdgpu_waves_per_eu(5))) void k_query(
    const __bf16* __restrict__ X, const float* __restrict__ W1, const float* __restrict__ b1,
    const float* __restrict__ w2q, const float* __restrict__ b2q, int K, int64_t n,
    float* __restrict__ prob, int32_t* __restrict__ label, const int32_t* __restrict__ gt,
    float* __restrict__ ce_part) {
  constexpr int KP = 16 * NLT, NHT = kHid / 16;
  __shared__ float s_a1[NHT][4][64];       // W1^T operand of k-step s, lane order
  __shared__ float s_a2[NLT][NHT][4][64];  // W2q^T operand, lane order
  __shared__ float s_b1[kHid], s_b2[KP];
  __shared__ float s_red[kQueryBlock / 64];
  const int lane = threadIdx.x & 63, r = lane & 15, c4 = lane >> 4;
  for (int e = threadIdx.x; e < NHT * 4 * 64; e += kQueryBlock) {
    const int t = e >> 8, k = (e >> 6) & 3, l = e & 63;
    s_a1[t][k][l] = W1[(4 * k + (l >> 4)) * kHid + 16 * t + (l & 15)];
  }
  for (int e = threadIdx.x; e < NLT * NHT * 4 * 64; e += kQueryBlock) {
    const int u = e / (NHT * 256), rem = e % (NHT * 256);
    const int t = rem >> 8, i = (rem >> 6) & 3, l = rem & 63;
    s_a2[u][t][i][l] = w2q[(16 * t + 4 * (l >> 4) + i) * KP + 16 * u + (l & 15)];
  }
  if (threadIdx.x < kHid) s_b1[threadIdx.x] = b1[threadIdx.x];
  if (threadIdx.x < KP) s_b2[threadIdx.x] = b2q[threadIdx.x];
  __syncthreads();
  const int64_t ngroups = (n + 15) / 16;
  const int64_t nwaves = (int64_t)gridDim.x * (kQueryBlock / 64);
  float ce = 0.f;
  // B of layer 1, k-step s: latent 4 s + l / 16 of pixel l % 16; the next
  // group's are loaded while this one is computed
  // (a pixel in range is read and the value dropped outside it: a load in a
  // branch would make the compiler wait for every load in flight where the
  // paths join)
  auto load_x = [&](int64_t g, float* x) {
    const int64_t q = g * 16 + r;
    const bool in = g < ngroups && q < n;
    const int64_t qc = in ? q : n - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v = (float)X[(int64_t)(4 * k + c4) * n + qc];
      x[k] = in ? v : 0.f;
    }
  };
  int64_t grp = (int64_t)blockIdx.x * (kQueryBlock / 64) + (threadIdx.x >> 6);
  float xb[4];
  load_x(grp, xb);
  for (; grp < ngroups; grp += nwaves) {
    const int64_t p = grp * 16 + r;
    const bool ok = p < n;
    float xn[4];
    load_x(grp + nwaves, xn);
    const int gl = gt ? gt[ok ? p : n - 1] : -1;  // (gt is uniform)
    // the operands are read from LDS at every step: an empty asm keeps the
    // compiler from holding all 32 + 32 NLT of them in registers across the
    // loop, which would leave room for two waves per SIMD
    int li = lane;
    asm volatile("" : "+v"(li));
    float h[NHT][4];
#pragma unroll
    for (int t = 0; t < NHT; ++t) {
      f32x4q z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        z = __builtin_amdgcn_mfma_f32_16x16x4f32(s_a1[t][k][li], xb[k], z, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) h[t][i] = gelu_f(z[i] + s_b1[16 * t + 4 * c4 + i]);
    }
    float lg[NLT][4];
#pragma unroll
    for (int u = 0; u < NLT; ++u) {
      f32x4q acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NHT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s_a2[u][t][i][li], h[t][i], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) lg[u][i] = acc[i] + s_b2[16 * u + 4 * c4 + i];
    }
    // the pixel's labels are spread over lanes r, r + 16, r + 32, r + 48
    float m = -INFINITY;
    int arg = 0x7FFFFFFF;
#pragma unroll
    for (int u = 0; u < NLT; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lab = 16 * u + 4 * c4 + i;
        if (lab < K && (lg[u][i] > m || (lg[u][i] == m && lab < arg))) {
          m = lg[u][i];
          arg = lab;
        }
      }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const float mo = __shfl_xor(m, off, 64);
      const int ao = __shfl_xor(arg, off, 64);
      if (mo > m || (mo == m && ao < arg)) {
        m = mo;
        arg = ao;
      }
    }
    float z = 0.f;
#pragma unroll
    for (int u = 0; u < NLT; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (16 * u + 4 * c4 + i < K) z += __expf(lg[u][i] - m);
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) z += __shfl_xor(z, off, 64);
    if (ok) {
      if (prob) {
        const float inv = 1.f / z;
#pragma unroll
        for (int u = 0; u < NLT; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int lab = 16 * u + 4 * c4 + i;
            if (lab < K) prob[(int64_t)lab * n + p] = __expf(lg[u][i] - m) * inv;
          }
      }
      if (label && c4 == 0) label[p] = arg;
      if (gt) {
        const int l = gl;
#pragma unroll
        for (int u = 0; u < NLT; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (16 * u + 4 * c4 + i == l && l < K) ce += (m + __logf(z)) - lg[u][i];  // -log p
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) xb[k] = xn[k];
  }
  if (ce_part) {
    float v = ce;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) ce_part[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  }
}

// the loss: the blocks' partials in block order, over n pixels
__global__ __launch_bounds__(256) void k_query_ce(const float* __restrict__ part, int nb,
                                                  int64_t n, float* __restrict__ loss) {
  __shared__ double s_red[4];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += part[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (float)(((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])) / (double)n);
}

}  // namespace gsff

using namespace gsff;

extern "C" {

gsff_status gsff_decoder_workspace_size(int64_t n_px, size_t* bytes) {
  if (!bytes || n_px < 0) return GSFF_ERR_INVALID_ARGUMENT;
  *bytes = (size_t)dec_layout(n_px).total;
  return GSFF_OK;
}

static hipError_t dec_prepare(const float* W1, const float* W2, char* ws, const DecLayout& L,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_dec_prepare, dim3(256), dim3(256), 0, s, W1, W2, (__bf16*)(ws + L.w1t),
                     (__bf16*)(ws + L.w1p), (__bf16*)(ws + L.w2tp), (__bf16*)(ws + L.w2p));
  return hipGetLastError();
}

gsff_status gsff_decoder_forward(const void* X, const float* W1, const float* b1,
                                 const float* W2, const float* b2, void* Y, int32_t y_dtype,
                                 int64_t n_px, void* ws, size_t ws_bytes, void* stream) {
  if (n_px < 0 || !ws || (n_px > 0 && (!X || !W1 || !b1 || !W2 || !b2 || !Y)))
    return GSFF_ERR_INVALID_ARGUMENT;
  if (y_dtype != GSFF_DTYPE_F32 && y_dtype != GSFF_DTYPE_BF16) return GSFF_ERR_UNSUPPORTED;
  if (((uintptr_t)ws & 255u) != 0) return GSFF_ERR_INVALID_ARGUMENT;
  const DecLayout L = dec_layout(n_px);
  if (ws_bytes < L.total) return GSFF_ERR_INVALID_ARGUMENT;
  if (n_px == 0) return GSFF_OK;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (dec_prepare(W1, W2, w, L, s) != hipSuccess) return GSFF_ERR_HIP;
  constexpr int NPB = 2;  // two blocks per wave: 156 registers, three waves per SIMD
  const int64_t waves = (L.nblk + NPB - 1) / NPB;
  const unsigned grid = (unsigned)((waves + 3) / 4);
  // rows of the output map 16-byte aligned: whole row segments per store
  const bool y16 = ((uintptr_t)Y & 15u) == 0;
#define GSFF_DEC_FWD(OTT, ROWS)                                                              \
  hipLaunchKernelGGL((k_dec_forward<NPB, OTT, ROWS>), dim3(grid), dim3(256), 0, s,          \
                     (const __bf16*)X, b1, b2, (const __bf16*)(w + L.w1t),                  \
                     (const __bf16*)(w + L.w2tp), (OTT*)Y, n_px)
  if (y_dtype == GSFF_DTYPE_BF16) {
    if (y16 && n_px % 8 == 0) GSFF_DEC_FWD(__bf16, true);
    else GSFF_DEC_FWD(__bf16, false);
  } else {
    if (y16 && n_px % 4 == 0) GSFF_DEC_FWD(float, true);
    else GSFF_DEC_FWD(float, false);
  }
#undef GSFF_DEC_FWD
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

gsff_status gsff_decoder_train_step(const void* X, const float* W1, const float* b1,
                                    const float* W2, const float* b2, const void* T,
                                    int64_t n_px, float scale, float* loss, float* dX,
                                    float* dW1, float* db1, float* dW2, float* db2, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (n_px <= 0 || !ws || !X || !W1 || !b1 || !W2 || !b2 || !T || !dX || !dW1 || !db1 || !dW2 ||
      !db2)
    return GSFF_ERR_INVALID_ARGUMENT;
  if (((uintptr_t)ws & 255u) != 0) return GSFF_ERR_INVALID_ARGUMENT;
  const DecLayout L = dec_layout(n_px);
  if (ws_bytes < L.total) return GSFF_ERR_INVALID_ARGUMENT;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if (dec_prepare(W1, W2, w, L, s) != hipSuccess) return GSFF_ERR_HIP;
  const unsigned grid = (unsigned)((L.nblk + 3) / 4);
  hipLaunchKernelGGL(k_dec_train, dim3(grid), dim3(256), 0, s, (const __bf16*)X, b1, b2,
                     (const __bf16*)T, (const __bf16*)(w + L.w1t), (const __bf16*)(w + L.w1p),
                     (const __bf16*)(w + L.w2tp), (const __bf16*)(w + L.w2p),
                     (__bf16*)(w + L.xbuf), (__bf16*)(w + L.hbuf), (__bf16*)(w + L.dzbuf),
                     (int8_t*)(w + L.dys), dX, loss, scale, n_px, L.npad);
  // split-K over the padded pixel range, in steps of 16
  int64_t kchunk = (L.npad + kWgradGroups - 1) / kWgradGroups;
  kchunk = (kchunk + 15) / 16 * 16;
  const int64_t groups = (L.npad + kchunk - 1) / kchunk;
  // dW2[h][c] = scale sum_p H[h][p] sign[c][p];  db2[c] = scale sum_p sign[c][p]
  // (W2: 64 output blocks in four workgroups of 16 per K range, each with
  // all four row blocks of four column blocks, so the GEMM has four waves per
  // SIMD to hide its loads and reads the signs once)
  hipLaunchKernelGGL((k_dec_wgrad<int8_t, 2>), dim3((unsigned)groups, 4u), dim3(64 * kWgradWaves), 0,
                     s, (const __bf16*)(w + L.hbuf), kHid, kHid / 32, (const int8_t*)(w + L.dys),
                     kOut / 32, L.npad, kchunk, (float*)(w + L.part2));
  // dW1[k][h] = sum_p X[k][p] dZ[h][p];  db1[h] = sum_p dZ[h][p]  (dZ carries the scale)
  hipLaunchKernelGGL((k_dec_wgrad<__bf16, 1>), dim3((unsigned)groups, 1u), dim3(64 * kWgradWaves), 0,
                     s, (const __bf16*)(w + L.xbuf), kLat, 1, (const __bf16*)(w + L.dzbuf),
                     kHid / 32, L.npad, kchunk, (float*)(w + L.part1));
  hipLaunchKernelGGL(k_dec_reduce, dim3((kHid * kOut + kOut + kRedCols - 1) / kRedCols), dim3(256),
                     0, s, (const float*)(w + L.part2), (int)groups, kHid, kOut, kHid, scale, scale,
                     dW2, db2);
  hipLaunchKernelGGL(k_dec_reduce, dim3((kLat * kHid + kHid + kRedCols - 1) / kRedCols), dim3(256),
                     0, s, (const float*)(w + L.part1), (int)groups, 32, kHid, kLat, 1.f, 1.f, dW1, db1);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}


static int64_t query_blocks(int64_t n_px) {
  const int64_t groups = (n_px + 15) / 16;  // 16 pixels per wave step
  const int64_t b = (groups + 15) / 16;     // about four steps per wave
  return b < 1024 ? b : 1024;
}

gsff_status gsff_decoder_query_workspace_size(int32_t K, int64_t n_px, size_t* bytes) {
  if (!bytes || K < 1 || K > kQueryMaxK || n_px < 0) return GSFF_ERR_INVALID_ARGUMENT;
  *bytes = (size_t)(4 * ((kHid + 1) * kQueryMaxK + query_blocks(n_px) + 1));
  return GSFF_OK;
}

static gsff_status query_impl(const void* X, const float* W1, const float* b1, const float* W2,
                              const float* b2, const float* Q, int32_t K, int64_t n_px,
                              float* prob, int32_t* label, const int32_t* gt, float* ce_loss,
                              float* ws, hipStream_t s) {
  const int NLT = (K + 15) / 16, KP = 16 * NLT;
  float* w2q = ws;
  float* b2q = w2q + kHid * KP;
  float* part = ws + (kHid + 1) * kQueryMaxK;
  hipLaunchKernelGGL(k_query_fold, dim3((unsigned)(((kHid + 1) * KP + 3) / 4)), dim3(256), 0, s,
                     W2, b2, Q, (int)K, KP, w2q, b2q);
  const int64_t nb = n_px > 0 ? query_blocks(n_px) : 0;
  if (nb > 0) {
    float* cp = gt ? part : nullptr;
#define GSFF_QUERY(NLTV)                                                                        \
  hipLaunchKernelGGL(k_query<NLTV>, dim3((unsigned)nb), dim3(kQueryBlock), 0, s, (const __bf16*)X, \
                     W1, b1, (const float*)w2q, (const float*)b2q, (int)K, n_px, prob, label, gt, \
                     cp)
    if (NLT == 1) GSFF_QUERY(1);
    else if (NLT == 2) GSFF_QUERY(2);
    else if (NLT == 3) GSFF_QUERY(3);
    else GSFF_QUERY(4);
#undef GSFF_QUERY
  }
  if (ce_loss)
    hipLaunchKernelGGL(k_query_ce, dim3(1), dim3(256), 0, s, (const float*)part, (int)nb,
                       n_px > 0 ? n_px : (int64_t)1, ce_loss);
  return hipGetLastError() == hipSuccess ? GSFF_OK : GSFF_ERR_HIP;
}

static bool query_args_ok(const void* X, const float* W1, const float* b1, const float* W2,
                          const float* b2, const float* Q, int32_t K, int64_t n_px,
                          const int32_t* gt, const float* ce_loss) {
  return !(K < 1 || K > kQueryMaxK || n_px < 0 || !W1 || !b1 || !W2 || !b2 || !Q ||
           (n_px > 0 && (!X || (gt == nullptr) != (ce_loss == nullptr))));
}

gsff_status gsff_decoder_query(const void* X, const float* W1, const float* b1, const float* W2,
                               const float* b2, const float* Q, int32_t K, int64_t n_px,
                               float* prob, int32_t* label, const int32_t* gt, float* ce_loss,
                               void* ws, size_t ws_bytes, void* stream) {
  if (!ws || !query_args_ok(X, W1, b1, W2, b2, Q, K, n_px, gt, ce_loss))
    return GSFF_ERR_INVALID_ARGUMENT;
  if (((uintptr_t)ws & 15u) != 0) return GSFF_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  gsff_decoder_query_workspace_size(K, n_px, &need);
  if (ws_bytes < need) return GSFF_ERR_INVALID_ARGUMENT;
  return query_impl(X, W1, b1, W2, b2, Q, K, n_px, prob, label, gt, ce_loss, (float*)ws,
                    (hipStream_t)stream);
}

// ---- the same query without a workspace argument --------------------------
// Its scratch (the folded weights of up to kQueryMaxK labels and the per-block
// cross-entropy partials, at most 1024 blocks whatever n_px) lives in a
// file-scope device array, one copy per GPU for the life of the process.  Host
// code never passes the array's name to a kernel: its device address comes
// from hipGetSymbolAddress, once per device, with that device current.
}  // extern "C"

namespace gsff {
namespace {
constexpr int kQueryScratchFloats = (kHid + 1) * kQueryMaxK + 1024 + 1;
static_assert(kQueryScratchFloats * 4 <= 40 * 1024, "query scratch stays modest");
constexpr int kMaxDevices = 64;
__device__ __align__(256) float scratch[kQueryScratchFloats];
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The calling thread's current device's scratch address (set up on the
// first call on that device).
hipError_t scratch_for_current_device(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace
}  // namespace gsff

extern "C" gsff_status gsff_decoder_query_noalloc(const void* X, const float* W1,
                                                  const float* b1, const float* W2,
                                                  const float* b2, const float* Q, int32_t K,
                                                  int64_t n_px, float* prob, int32_t* label,
                                                  const int32_t* gt, float* ce_loss,
                                                  void* stream) {
  if (K > kQueryMaxK) return GSFF_ERR_INVALID_ARGUMENT;  // beyond the scratch's label count
  if (!query_args_ok(X, W1, b1, W2, b2, Q, K, n_px, gt, ce_loss))
    return GSFF_ERR_INVALID_ARGUMENT;
  float* ws = nullptr;
  if (scratch_for_current_device(&ws) != hipSuccess || !ws) return GSFF_ERR_HIP;
  // every scratch word a call reads it writes first (folded weights, then
  // one partial per block), so nothing is cleared
  return query_impl(X, W1, b1, W2, b2, Q, K, n_px, prob, label, gt, ce_loss, ws,
                    (hipStream_t)stream);
}

