// Front-to-back alpha compositing of colour, depth and a C-channel feature
// payload (Sec. 3.1, Eqs. 2-3) and its adjoint.
//
// One 256-thread workgroup per 16x16 screen tile, one thread per pixel.  The
// tile's depth-ordered Gaussian list is walked in batches staged in LDS
// (records gathered by id, features split into BF16 hi and lo parts on the
// way in).  Alpha, transmittance, the blending weights and every skip / stop
// decision are FP32; the colour, depth and feature sums (and the adjoint's
// contraction over the tile's pixels) are matrix-core products of BF16 hi/lo
// splits of both operands with FP32 accumulation, each product accurate to
// about 2^-16 relative.  A workgroup stops as soon as every pixel in it has
// saturated (T would fall below t_min).
//
// Workgroup -> tile mapping is XCD-aware: the dispatcher hands consecutive
// workgroups to the 8 XCDs in turn, so workgroup b is sent to tile
// (b % 8) * ceil(ntiles/8) + b / 8 -- each XCD then renders a contiguous
// band of tiles and neighbouring tiles (which share most Gaussians) hit the
// same L2.  The adjoint takes list segments longest first.
//
// The adjoint walks back to front from each pixel's last contributor,
// recovering T_i = T_{i+1} / (1 - alpha_i) instead of storing per-pixel
// lists.  Geometry gradients (dalpha and everything behind it) come only
// from the colour, depth and opacity upstream; the feature upstream only
// produces d f_i = sum_p w_ip g_F(p) (Sec. 3.1, last paragraph).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "blend.h"
#include "gsff_internal.h"

namespace gsff {

constexpr int kNumXcd = 8;

__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int per = (ntiles + kNumXcd - 1) / kNumXcd;
  return (b % kNumXcd) * per + b / kNumXcd;
}

__device__ __forceinline__ float load_feat(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_feat(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}
__device__ __forceinline__ float load_feat(const _Float16* p, int64_t i) { return (float)p[i]; }

__device__ __forceinline__ void store_out(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_out(uint16_t* p, int64_t i, float v) {
  // round to nearest even
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) {
    p[i] = 0x7FC0u;
    return;
  }
  u += 0x7FFFu + ((u >> 16) & 1u);
  p[i] = (uint16_t)(u >> 16);
}

// A tile's [start, end) limited to the pair buffer.
__device__ __forceinline__ uint2 clamp_range(uint2 r, uint32_t max_pairs) {
  const uint32_t e = min(r.y, max_pairs);
  return make_uint2(min(r.x, e), e);
}

// Gather the three record vectors of `gid`; an out-of-range id gets zero
// opacity, so every pixel skips it.
// Branch-free (an id past the end reads Gaussian 0 and keeps zeros): a
// conditional assignment through the references made the compiler stage the
// records in private memory.
__device__ __forceinline__ float4 keep4(bool ok, float4 a) {
  return make_float4(ok ? a.x : 0.f, ok ? a.y : 0.f, ok ? a.z : 0.f, ok ? a.w : 0.f);
}
// Issue the gather only; returns whether the id is valid.
__device__ __forceinline__ bool fetch_record(const WsView& w, uint32_t gid, int64_t P, float4& r0,
                                             float4& r1, float4& r2) {
  const bool ok = gid < (uint32_t)P;
  const int64_t g = ok ? (int64_t)gid : 0;
  r0 = w.rec[g];
  r1 = w.rec[P + g];
  r2 = w.rec[2 * P + g];
  return ok;
}
__device__ __forceinline__ void load_record(const WsView& w, uint32_t gid, int64_t P, float4& r0,
                                            float4& r1, float4& r2) {
  const bool ok = fetch_record(w, gid, P, r0, r1, r2);
  r0 = keep4(ok, r0);
  r1 = keep4(ok, r1);
  r2 = keep4(ok, r2);
}
// A prefetched record, settled where it is staged.  The empty asm makes the
// values opaque up to this point: otherwise the compiler moves their first
// use (the zeroing, the scaling) up to the loads and waits for the loads
// there, a memory round trip per batch instead of one hidden by the batch.
__device__ __forceinline__ void opaque4(float4& r) {
  float __attribute__((ext_vector_type(4))) v = {r.x, r.y, r.z, r.w};
  __asm__ volatile("" : "+v"(v));
  r = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void settle_record(bool ok, float4& r0, float4& r1, float4& r2) {
  opaque4(r0);
  opaque4(r1);
  opaque4(r2);
  r0 = keep4(ok, r0);
  r1 = keep4(ok, r1);
  r2 = keep4(ok, r2);
}

// The Gaussian's exponent (Eq. 2's G) in base 2:
//   log2(e) * (-1/2) (A dx^2 + 2 B dx dy + C dy^2) = dx (a dx + b dy) + c dy^2
// with a = kConA A, b = kConB B, c = kConA C.  Both compositing kernels keep
// the conic of a staged batch in this scaled form (the adjoint unscales it
// for the mean and conic gradients).
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kConA = -0.5f * kLog2e, kConB = -kLog2e;
constexpr float kConAInv = -2.f * kLn2, kConBInv = -kLn2;

// A record as staged for eval_alpha: (u, v, a, b) (c, o, z, log2 o) -- the
// stored record's last lane (its valid flag) is not needed once a Gaussian is
// in a tile list.  Applied where a prefetched record is written to LDS, not
// where it is loaded, so the load stays in flight while the current batch
// runs.  A zeroed record (an id past the end) stages log2 0 = -inf: alpha 0.
__device__ __forceinline__ float4 scaled_r0(float4 r0) {
  return make_float4(r0.x, r0.y, r0.z * kConA, r0.w * kConB);
}
__device__ __forceinline__ float4 scaled_r1(float4 r1) {
  return make_float4(r1.x * kConA, r1.y, r1.z, __builtin_amdgcn_logf(r1.y));  // v_log_f32
}

// alpha of one (pixel, Gaussian) pair from a scaled record; forward and
// adjoint call this same code so every skip decision and weight is
// reproduced bit for bit.  The opacity enters the exponent as log2 o, so
// o G = 2^(log2 o + exponent) is one exp2 with no product after it.
struct AlphaEval {
  float dx, dy, oG, alpha;
};

__device__ __forceinline__ AlphaEval eval_alpha(const float4 r0, const float4 r1, float pxc,
                                                float pyc, float alpha_max) {
#pragma clang fp contract(off)
  AlphaEval e;
  e.dx = r0.x - pxc;
  e.dy = r0.y - pyc;
  const float q2 = __builtin_fmaf(e.dx, __builtin_fmaf(r0.z, e.dx, r0.w * e.dy),
                                  __builtin_fmaf(r1.x * e.dy, e.dy, r1.w));
  e.oG = __builtin_amdgcn_exp2f(q2);  // v_exp_f32
  // min(oG, alpha_max) for oG >= 0, as one v_med3_f32 (a plain fminf of the
  // exp2 result makes the compiler quiet a NaN first, one more instruction)
  e.alpha = __builtin_amdgcn_fmed3f(e.oG, 0.f, alpha_max);
  return e;
}

// ------------------------------------------------------ matrix helpers -----

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi), |r| <= 2^-16 |x|.
__device__ __forceinline__ void split8(const float4 a, const float4 b, bf16x8& hi, bf16x8& lo) {
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    hi[t] = (__bf16)v[t];
    lo[t] = (__bf16)(v[t] - (float)hi[t]);
  }
}

__device__ __forceinline__ bf16x8 to_bf16x8(const float4 a, const float4 b) {
  bf16x8 h;
  h[0] = (__bf16)a.x; h[1] = (__bf16)a.y; h[2] = (__bf16)a.z; h[3] = (__bf16)a.w;
  h[4] = (__bf16)b.x; h[5] = (__bf16)b.y; h[6] = (__bf16)b.z; h[7] = (__bf16)b.w;
  return h;
}

// Sixteen 4x4x4 BF16 products at once (FP32 accumulate): block b = lanes
// 4b .. 4b+3; lane 4b + i holds row i of A (k = 0..3 in element order), lane
// 4b + j column j of B, and D[i][j] for i = 0..3 lands in lane 4b + j.
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 mfma4(const bf16x4 a, const bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s16x4, a),
                                                 __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}

// D += A B for one 16x16x32 BF16 tile (FP32 accumulate).  Lane l holds
// A[l % 16][8 (l / 16) .. +7], B[8 (l / 16) .. +7][l % 16] and
// D[4 (l / 16) + r][l % 16] in acc[r].
__device__ __forceinline__ f32x4 mfma16(const bf16x8 a, const bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Workgroup barrier that orders LDS only: global loads and atomics issued
// before it stay in flight (a full __syncthreads() would wait for every
// outstanding global access of the wave).  All communication between the
// waves of the compositing kernels goes through LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------ forward -----

// set bits of m below this lane
__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

constexpr int kFwdNB = 16;
constexpr int kFwdQueue = 256;  // accepted-id ring of the forward's list scan       // Gaussians per batch
constexpr int kFwdWStride = 40;  // LDS row (BF16): a pixel's batch weights, hi at 0, lo at 16
constexpr int kFwdFStride = 24;  // LDS row stride (bf16) of a channel's batch features

template <typename FT>
__device__ __forceinline__ void feat_split(const FT* p, int64_t i, __bf16& hi, __bf16& lo) {
  const float v = load_feat(p, i);
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}
__device__ __forceinline__ void feat_split(const uint16_t* p, int64_t i, __bf16& hi, __bf16& lo) {
  hi = __builtin_bit_cast(__bf16, p[i]);  // BF16 payload: exact
  lo = (__bf16)0.f;
}
// the same split of an element already loaded
__device__ __forceinline__ void split_value(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}
__device__ __forceinline__ void split_value(_Float16 v, __bf16& hi, __bf16& lo) {
  split_value((float)v, hi, lo);
}
__device__ __forceinline__ void split_value(uint16_t v, __bf16& hi, __bf16& lo) {
  hi = __builtin_bit_cast(__bf16, v);
  lo = (__bf16)0.f;
}

// Front-to-back compositing of one tile per workgroup, one thread per pixel.
//
// The tile's list is walked in batches of 16 Gaussians:
//  phase A  each thread walks the batch front to back, branch-free: alpha,
//           the skip / stop decisions, the blending weight w and
//           transmittance (FP32, in list order); the 16 weights go to the
//           wave's own LDS rows as BF16 hi and lo parts.
//  phase B  the colour and depth sums are 4x4x4 BF16 products (the weights'
//           hi and lo parts against the batch's colour and depth, split the
//           same way); the feature sums of the wave's 64 pixels are one
//           16x16x32 BF16 matrix product per 16 pixels x 16 channels: K
//           holds the 16 weights twice, as hi and as lo BF16 parts, against
//           the BF16 features (exact for a BF16 payload; FP32 / FP16
//           payloads add a second product with the features' lo parts), so
//           every product keeps about 2^-16 relative accuracy and the
//           accumulation is FP32.
// Records, ids and features of the next batches are loaded while a batch is
// processed (ids two batches ahead); one LDS-only barrier per batch.  The
// workgroup stops after the batch in which its last pixel saturated.
// Register budget: every tile of a 640x480 frame resident at once needs five
// workgroups (waves) per CU (SIMD); wider channel blocks hold more accumulators.
template <int CP, typename FT, typename OT>
__global__ __attribute__((amdgpu_flat_work_group_size(kBlock, kBlock),
                          amdgpu_waves_per_eu(CP <= 16 ? 5 : (CP <= 32 ? 4 : 3))))
void k_composite_fwd(
    DevSettings st, int64_t P, int C, int c0, int W, int H, int tiles_x, int ntiles,
    int rank_bits, uint32_t max_pairs, WsView w, const FT* __restrict__ feat,
    float* __restrict__ out_rgb, float* __restrict__ out_depth, float* __restrict__ out_alpha,
    OT* __restrict__ out_feat, int write_geo) {
  constexpr int NB = kFwdNB;
  constexpr int NCB = (CP + 15) / 16;                   // 16-channel output blocks
  constexpr bool EXACT = sizeof(FT) == 2 && !__is_same(FT, _Float16);  // BF16 payload
  constexpr int CPs = CP > 0 ? CP : 1;
  constexpr int FPT = CP > 0 ? (NB * CP + kBlock - 1) / kBlock : 0;  // features per thread
  __shared__ __attribute__((aligned(16))) __bf16 s_w[kBlock][kFwdWStride];
  __shared__ __attribute__((aligned(16))) __bf16 s_fh[2][CPs][kFwdFStride];
  __shared__ __attribute__((aligned(16))) __bf16 s_fl[EXACT ? 1 : 2][EXACT ? 1 : CPs][kFwdFStride];
  __shared__ float4 s_r0[2][NB], s_r1[2][NB];
  // colour and depth of the batch as the B operand of the 4x4x4 products:
  // [buffer][hi, lo][group of 4 Gaussians][channel r, g, b, depth][Gaussian]
  __shared__ __attribute__((aligned(8))) __bf16 s_cc[2][2][NB / 4][4][4];
  __shared__ uint32_t s_ids[2][NB];
  __shared__ uint32_t s_nb[4], s_pos[4];  // size and list position of batch k, slot k % 4
  __shared__ uint32_t s_q[kFwdQueue];     // ids accepted for this tile, not yet batched
  __shared__ int s_act[2][kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  {
    // Issue priority from the walk this tile had in the previous forward on
    // this workspace (a hint: any value, even of a fresh workspace, is safe).
    // All tiles of a frame are resident at once, so the launch ends with its
    // longest walks; their waves go first and the short tiles fill the gaps.
    const uint2 prev = w.crange[tile];
    const uint32_t prev_len = __builtin_amdgcn_readfirstlane(prev.y - prev.x);
    if (prev_len >= 12u * kFwdNB) __builtin_amdgcn_s_setprio(3);
    else if (prev_len >= 9u * kFwdNB) __builtin_amdgcn_s_setprio(2);
    else if (prev_len >= 6u * kFwdNB) __builtin_amdgcn_s_setprio(1);
  }
  const int tid = threadIdx.x;
  // the wave index as a scalar: the scan wave's branches and counters stay uniform
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lq = lane >> 4,
            lj = lane & 15;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid & (kTile - 1));
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  // the super-tile's list; this tile's Gaussians are its entries with the tile's bit
  const int sx = (tiles_x + kSuper - 1) / kSuper;
  const int lsub = (ty % kSuper) * kSuper + tx % kSuper;
  const uint32_t bit = 1u << lsub;
  const uint2 sraw = w.tile_ranges[(ty / kSuper) * sx + tx / kSuper];
  if (GSFF_CHECKED && tid == 0) {  // start <= end <= the frame's pairs
    GSFF_CHECK(w.status, GSFF_CHECK_TILE_RANGE, sraw.x, (uint64_t)sraw.y + 1u);
    GSFF_CHECK(w.status, GSFF_CHECK_TILE_RANGE, sraw.y, (uint64_t)w.status[2] + 1u);
  }
  const uint2 sr = clamp_range(sraw, max_pairs);
  // the tile's walked list: kSuper^2 slots of the super-tile's length per super-tile entry
  const uint32_t cbase = (uint32_t)(kSuper * kSuper) * sr.x + (uint32_t)lsub * (sr.y - sr.x);
  const int cn = CP > 0 ? min(CP, C - c0) : 0;
  // Wave 2 scans the list, batches the accepted ids and gathers each batch's
  // records as soon as it has taken the ids, two batches before the batch
  // runs (record lane l < 48 loads vector l / 16 of the batch's Gaussian
  // l % 16), staging them at the end of the batch before it; the other waves
  // issue no record loads, and none waits for one at the top of a batch.
  const bool scan_wave = wave == kBlock / 64 - 2;
  const bool rec_lane = scan_wave && lane < 3 * NB;
  const int rg = lane & (NB - 1), rv = lane / NB;  // a record lane's Gaussian and vector
  uint32_t sc = sr.x, qh = 0, qt = 0;  // scan position, queue head / tail (scan wave)
  // Scan 128 list entries: lanes hold entries sc + lane and sc + 64 + lane.
  auto scan_issue = [&](uint32_t& gA, uint32_t& mA, uint32_t& gB, uint32_t& mB) {
    const uint32_t i0 = sc + (uint32_t)lane, i1 = i0 + 64u;
    gA = i0 < sr.y ? w.pkeys_a[i0] : 0u;
    mA = i0 < sr.y ? (uint32_t)w.pmask[i0] : 0u;
    gB = i1 < sr.y ? w.pkeys_a[i1] : 0u;
    mB = i1 < sr.y ? (uint32_t)w.pmask[i1] : 0u;
  };
  // append the accepted ones to the queue, in list order
  auto scan_commit = [&](uint32_t gA, uint32_t mA, uint32_t gB, uint32_t mB) {
    const bool a = (mA & bit) != 0u && GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, gA, (uint64_t)P);
    const bool b = (mB & bit) != 0u && GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, gB, (uint64_t)P);
    const uint64_t ba = __ballot(a), bb = __ballot(b);
    if (a) s_q[(qt + bits_below_lane(ba)) & (kFwdQueue - 1)] = gA;
    qt += (uint32_t)__popcll(ba);
    if (b) s_q[(qt + bits_below_lane(bb)) & (kFwdQueue - 1)] = gB;
    qt += (uint32_t)__popcll(bb);
    sc = min(sc + 128u, sr.y);
  };
  // the next batch's ids (full unless the list is exhausted), recorded in the
  // tile's walked list; returns the batch size
  auto take_batch = [&](uint32_t& g, uint32_t& pos) {
    while (qt - qh < (uint32_t)NB && sc < sr.y) {  // uniform in the scan wave
      uint32_t gA, mA, gB, mB;
      scan_issue(gA, mA, gB, mB);
      scan_commit(gA, mA, gB, mB);
    }
    const uint32_t n = min((uint32_t)NB, qt - qh);
    g = (uint32_t)P;
    if ((uint32_t)lane < n) {
      g = s_q[(qh + (uint32_t)lane) & (kFwdQueue - 1)];
      if (write_geo && GSFF_CHECK(w.status, GSFF_CHECK_WALK, qh + (uint32_t)lane, sr.y - sr.x))
        w.clist[cbase + qh + (uint32_t)lane] = g;
    }
    pos = qh;
    qh += n;
    return n;
  };

  // colour and depth sums of pixels 4 (lane / 4) + r of the wave, channel
  // lane % 4 (r, g, b, depth): the 4x4x4 products' accumulator
  f32x4 acc_c = {0.f, 0.f, 0.f, 0.f};
  // Record gather of a batch (called by the whole scan wave: ids holds the
  // batch's ids in lanes 0..NB-1, P past the batch); returns whether this
  // lane's Gaussian is valid.
  auto fetch_vec = [&](uint32_t ids, float4& v) {
    const uint32_t gid = __shfl(ids, rg, 64);
    const bool ok = gid < (uint32_t)P;
    if (rec_lane) v = w.rec[(int64_t)rv * P + (ok ? (int64_t)gid : 0)];
    return ok;
  };
  // A record lane stages its vector into buffer sb: (u, v, a, b) and (c, o,
  // z, log2 o) scaled for eval_alpha, colour and depth split hi + lo as the B
  // operand of the colour products.  The empty asm (opaque4) keeps the
  // compiler from using the values, and waiting for the gather, any earlier.
  auto stage_vec = [&](int sb, bool ok, float4 v) {
    opaque4(v);
    v = keep4(ok, v);
    auto colour = [&](int c, float x) {
      const __bf16 h = (__bf16)x;
      s_cc[sb][0][rg >> 2][c][rg & 3] = h;
      s_cc[sb][1][rg >> 2][c][rg & 3] = (__bf16)(x - (float)h);
    };
    if (rv == 0) {
      s_r0[sb][rg] = scaled_r0(v);
    } else if (rv == 1) {
      s_r1[sb][rg] = scaled_r1(v);
      colour(3, v.z);
    } else {
      colour(0, v.x);
      colour(1, v.y);
      colour(2, v.z);
    }
  };
  // T > 0 while the pixel is live.  A pixel stops by keeping -T (the same
  // magnitude), so every later T (1 - alpha) >= t_min test fails (t_min > 0)
  // and no separate done mask is carried; pixels outside the image start
  // stopped.  Every decision and every value is that of the plain loop.
  float T = inside ? 1.f : -1.f;
  uint32_t end = cbase;
  f32x4 acc[4][NCB > 0 ? NCB : 1];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int k = 0; k < (NCB > 0 ? NCB : 1); ++k) acc[rb][k] = f32x4{0.f, 0.f, 0.f, 0.f};

  // ---- prologue: ids of batches 0 and 1 and their record gathers (batch
  // 0's staged here, batch 1's in flight), then batch 0's features
  float4 rv_next = make_float4(0.f, 0.f, 0.f, 0.f);  // records of batch k + 1 (record lanes)
  bool rok_next = false;
  if (scan_wave) {
    uint32_t g0, g1, pos;
    const uint32_t n0 = take_batch(g0, pos);
    if (lane < NB) s_ids[0][lane] = g0;
    if (lane == 0) {
      s_nb[0] = n0;
      s_pos[0] = pos;
    }
    const uint32_t n1 = take_batch(g1, pos);
    if (lane < NB) s_ids[1][lane] = g1;
    if (lane == 0) {
      s_nb[1] = n1;
      s_pos[1] = pos;
    }
    float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool ok0 = fetch_vec(g0, v0);
    rok_next = fetch_vec(g1, rv_next);
    if (rec_lane) stage_vec(0, ok0, v0);
  }
  lds_barrier();
  if (s_nb[0] > 0u) {
    if constexpr (CP > 0) {
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        const int e = tid + kBlock * k;
        const int g = e / CP, c = e % CP;
        if (g < NB) {
          const uint32_t gid = s_ids[0][g];
          __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
          if (c < cn && gid < (uint32_t)P) feat_split(feat, (int64_t)gid * C + c0 + c, h, l);
          s_fh[0][c][g] = h;
          if constexpr (!EXACT) s_fl[0][c][g] = l;
        }
      }
    }
  }
  lds_barrier();

  int buf = 0;
  int nseg_end = 0;  // segment-end states recorded
  // a scan ahead of the queue, issued in one batch and committed at the start
  // of the next one, so its loads have a whole batch to arrive
  uint32_t gA = 0u, mA = 0u, gB = 0u, mB = 0u;
  bool ahead = false;
  for (uint32_t k = 0; s_nb[k & 3] > 0u; ++k) {
    const bool more = s_nb[(k + 1) & 3] > 0u;  // batch k + 1 has ids
    // walked-list position of this batch (uniform: a scalar register)
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(cbase + s_pos[k & 3]);
    // ---- the scan wave: ids of batch k + 2 from the queue (a scan first if the
    // queue runs short), then the next scan ahead
    uint32_t g_after = (uint32_t)P, n_after = 0u, pos_after = 0u;
    if (scan_wave) {
      if (ahead) scan_commit(gA, mA, gB, mB);
      n_after = more ? take_batch(g_after, pos_after) : 0u;
      ahead = qt - qh < 3u * NB && sc < sr.y;
      if (ahead) scan_issue(gA, mA, gB, mB);
    }
    // features of the next batch, raw: split where they are staged, so the
    // loads stay in flight while this batch runs
    FT fraw[FPT > 0 ? FPT : 1];
    if constexpr (CP > 0) {
#pragma unroll
      for (int kk = 0; kk < FPT; ++kk) {
        fraw[kk] = FT(0);
        const int e = tid + kBlock * kk;
        const int g = e / CP, c = e % CP;
        if (more && g < NB) {
          const uint32_t gid = s_ids[buf ^ 1][g];
          // the channel offset is re-formed every batch (an empty asm keeps the
          // compiler from holding a 64-bit base across the loop in a register
          // it does not have)
          int coff = c0 + c;
          asm volatile("" : "+v"(coff));
          if (c < cn && gid < (uint32_t)P) fraw[kk] = feat[(int64_t)gid * C + coff];
        }
      }
    }

    // ---- record gathers of batch k + 2 (k + 1's are in flight since batch
    // k - 1), issued after this batch's other loads: waits count loads in
    // issue order, so the waits for those (at this batch's staging) leave
    // these in flight
    float4 rv_after = make_float4(0.f, 0.f, 0.f, 0.f);
    bool rok_after = false;
    if (scan_wave) rok_after = fetch_vec(g_after, rv_after);

    // ---- every kSegBatches batches, each pixel's transmittance and the
    // colour and depth blended in front of this batch: the adjoint's segments
    // that end here start from them.  Stored after this batch's loads are
    // issued: waits for those loads do not include the stores.
    if (write_geo && k > 0 && k % kSegBatches == 0 && nseg_end < kMaxSeg - 1) {
      float* q = w.seg_state + ((int64_t)tile * (kMaxSeg - 1) + nseg_end) * 5 * kBlock;
      q[tid] = __builtin_fabsf(T);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        q[(1 + (lane & 3)) * kBlock + 64 * wave + 4 * (lane >> 2) + r] = acc_c[r];
      ++nseg_end;
    }
    const bool wave_active = __ballot(T > 0.f) != 0ull;
    if (wave_active) {
      // ---- phase A: weights, transmittance, colour and depth, front to back
      float wv[4];
      uint32_t last = 0u;  // 1 + batch position of the last Gaussian used here
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const float4 r0 = s_r0[buf][jj], r1 = s_r1[buf][jj];
        const AlphaEval e = eval_alpha(r0, r1, pxc, pyc, st.alpha_max);
        const bool ok = e.alpha >= st.alpha_min;          // not skipped
        const float Tn = __builtin_fmaf(-e.alpha, T, T);  // T (1 - alpha), one rounding
        const bool use = ok && Tn >= st.t_min;            // live and not stopping here
        const float wgt = use ? e.alpha * T : 0.f;
        T = use ? Tn : (ok ? -__builtin_fabsf(T) : T);    // a stop keeps -T
        last = use ? (uint32_t)jj + 1u : last;
        // formed here: deferred, the 16 use masks would stay live in SGPRs
        __asm__ volatile("" : "+v"(last));
        wv[jj & 3] = wgt;
        if ((jj & 3) == 3) {  // weight = hi + lo, both BF16: the products' A operands
          const f32x4 q = {wv[0], wv[1], wv[2], wv[3]};
          const bf16x4 h = __builtin_convertvector(q, bf16x4);
          const bf16x4 l = __builtin_convertvector(q - __builtin_convertvector(h, f32x4), bf16x4);
          *reinterpret_cast<bf16x4*>(&s_w[tid][jj - 3]) = h;
          *reinterpret_cast<bf16x4*>(&s_w[tid][16 + jj - 3]) = l;
        }
      }
      end = last ? b0 + last : end;
      // ---- phase B: colour and depth, and the feature sums, on the matrix cores
      // (the wave reads back only its own rows)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
      for (int g4 = 0; g4 < NB / 4; ++g4) {
        // A: this lane's pixel, Gaussians 4 g4 .. +3; B: channel lane % 4
        const bf16x4 h = *reinterpret_cast<const bf16x4*>(&s_w[tid][4 * g4]);
        const bf16x4 l = *reinterpret_cast<const bf16x4*>(&s_w[tid][16 + 4 * g4]);
        const bf16x4 ch = *reinterpret_cast<const bf16x4*>(&s_cc[buf][0][g4][lane & 3][0]);
        const bf16x4 cl = *reinterpret_cast<const bf16x4*>(&s_cc[buf][1][g4][lane & 3][0]);
        acc_c = mfma4(h, ch, acc_c);
        acc_c = mfma4(l, ch, acc_c);
        acc_c = mfma4(h, cl, acc_c);
      }
      if constexpr (CP > 0) {
        const int gk = 8 * (lq & 1);  // Gaussians gk .. gk+7 of the batch
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          // hi weights in lanes 0-31, lo in 32-63 (the K-concatenation of A)
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(
              &s_w[64 * wave + 16 * rb + lj][(lq < 2 ? 0 : 16) + gk]);
#pragma unroll
          for (int kc = 0; kc < NCB; ++kc) {
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&s_fh[buf][16 * kc + lj][gk]);
            acc[rb][kc] = mfma16(a, bh, acc[rb][kc]);
            if constexpr (!EXACT) {
              bf16x8 bl = *reinterpret_cast<const bf16x8*>(&s_fl[buf][16 * kc + lj][gk]);
              if (lq >= 2) bl = bf16x8{};
              acc[rb][kc] = mfma16(a, bl, acc[rb][kc]);
            }
          }
        }
      }
    }
    // ---- stage the next batch, report activity
    if (more) {
      if (rec_lane) stage_vec(buf ^ 1, rok_next, rv_next);
      if constexpr (CP > 0) {
#pragma unroll
        for (int kk = 0; kk < FPT; ++kk) {
          const int e = tid + kBlock * kk;
          const int g = e / CP, c = e % CP;
          if (g < NB) {
            __bf16 h, l;
            split_value(fraw[kk], h, l);
            s_fh[buf ^ 1][c][g] = h;
            if constexpr (!EXACT) s_fl[buf ^ 1][c][g] = l;
          }
        }
      }
    }
    rv_next = rv_after;
    rok_next = rok_after;
    if (scan_wave) {
      if (lane < NB) s_ids[buf][lane] = g_after;  // the slot of batch k + 2
      if (lane == 0) {
        s_nb[(k + 2) & 3] = n_after;
        s_pos[(k + 2) & 3] = pos_after;
      }
    }
    const bool still = __ballot(T > 0.f) != 0ull;
    if (lane == 0) s_act[buf][wave] = still ? 1 : 0;
    lds_barrier();
    if (!more) break;
    if ((s_act[buf][0] | s_act[buf][1] | s_act[buf][2] | s_act[buf][3]) == 0) break;
    buf ^= 1;
  }

  if (write_geo) {  // uniform: end of the walk of this tile's list, for the adjoint
    __shared__ uint32_t s_wend;
    if (tid == 0) s_wend = cbase;
    lds_barrier();
    if (inside) atomicMax(&s_wend, end);
    lds_barrier();
    if (tid == 0) {
      w.tile_walk[tile] = s_wend;
      w.crange[tile] = make_uint2(cbase, s_wend);
    }
  }

  // a split tile also keeps its final colour and depth: the adjoint takes
  // what is blended behind a segment's end as final minus recorded
  if (nseg_end > 0) {
    float* q = w.seg_final + (int64_t)tile * 4 * kBlock;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      q[(lane & 3) * kBlock + 64 * wave + 4 * (lane >> 2) + r] = acc_c[r];
  }
  const int64_t HW = (int64_t)W * H;
  if (write_geo) {
    // colour and depth from the accumulator lanes: channel lane % 4 of pixels
    // 64 wave + 4 (lane / 4) + r of the tile
    const int ch = lane & 3;
    float* dst = ch < 3 ? out_rgb + (int64_t)ch * HW : out_depth;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int tp = 64 * wave + 4 * (lane >> 2) + r;
      const int qx = tx * kTile + (tp & (kTile - 1)), qy = ty * kTile + tp / kTile;
      if (qx < W && qy < H) dst[(int64_t)qy * W + qx] = acc_c[r];
    }
  }
  if (inside && write_geo) {
    const int64_t p = (int64_t)py * W + px;
    out_alpha[p] = 1.f - __builtin_fabsf(T);
    w.pix_T[p] = __builtin_fabsf(T);
    w.pix_end[p] = end;
  }
  if constexpr (CP > 0) {
    if (out_feat) {
      // acc[rb][k][r]: pixel 64 wave + 16 rb + 4 lq + r of the tile, channel 16 k + lj
#pragma unroll
      for (int k = 0; k < NCB; ++k) {
        const int c = 16 * k + lj;
        if (c >= cn) continue;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int tp = 64 * wave + 16 * rb + 4 * lq + r;
            const int qx = tx * kTile + (tp & (kTile - 1)), qy = ty * kTile + tp / kTile;
            if (qx < W && qy < H)
              store_out(out_feat, (int64_t)(c0 + c) * HW + (int64_t)qy * W + qx, acc[rb][k][r]);
          }
      }
    }
  }
}

template <typename OT>
__global__ void k_fill_zero(OT* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = OT(0);
}

// Deterministic mode: every slot of the Gaussians' rectangles empty
// (0xFFFFFFFF) before the adjoint files its rows; the slots in use end where
// the scan of the per-block slot counts ends.
__global__ __launch_bounds__(256) void k_fill_slots(WsView w, int nslot_blk) {
  const uint64_t used = nslot_blk > 0 ? (uint64_t)w.slot_blk[nslot_blk - 1] +
                                             w.slot_cnt[nslot_blk - 1]
                                       : 0ull;
  const uint64_t n = used < w.slot_cap ? used : w.slot_cap;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    w.slots[i] = 0xFFFFFFFFu;
}

// The adjoint's work items and the first adjoint row of every tile, built by
// one workgroup of NT threads (the standalone kernel below, or the first
// workgroup of the L1 upstream pass).
//
// walk_off: an exclusive scan of the walk lengths (the list prefix the
// forward visited) over the tiles.  Items: each tile's walked list in
// segments of kSegLen entries (at most kMaxSeg, the last takes the rest; a
// tile with an empty walk has none), ordered by decreasing length (counting
// sort on buckets of 4 entries), so the items that start after the first
// round of resident workgroups are the short ones.  An item is
// tile | segment << 24 | (a later segment follows) << 30 | (the tile's rows
// fit) << 31, its list range [q1, q2) and the row of list position 0 (rows
// are indexed by list position).
//
// Thread t holds tiles kItemRegs t .. kItemRegs t + kItemRegs - 1 of each
// chunk of NT kItemRegs tiles in registers; with one chunk (up to 2048 tiles
// at 256 threads, 8192 at 1024) the ranges are read once.
constexpr int kItemBuckets = 1024;
constexpr int kItemRegs = 8;
struct ItemScratch {
  uint32_t cnt[kItemBuckets];
  uint32_t part[16];
  uint32_t total;
};

__device__ __forceinline__ uint32_t wave_excl_u32(uint32_t v, uint32_t& total) {
  const int lane = threadIdx.x & 63;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  total = __shfl(inc, 63, 64);
  return inc - v;
}

// exclusive scan over the NT threads of the workgroup (all of them call it)
template <int NT>
__device__ __forceinline__ uint32_t block_excl_u32(uint32_t v, uint32_t& total, uint32_t* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t wt;
  const uint32_t ex = wave_excl_u32(v, wt);
  if (lane == 0) part[wv] = wt;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const uint32_t p = part[k];
    if (k < wv) pre += p;
    tot += p;
  }
  __syncthreads();
  total = tot;
  return pre + ex;
}

template <int NT>
__device__ void build_adjoint_items(const WsView& w, int ntiles, uint32_t max_pairs,
                                    ItemScratch& sm) {
  constexpr int R = kItemRegs, CH = NT * R;
  const int tid = threadIdx.x, lane = tid & 63;
  auto nseg_of = [](uint32_t v) { return min((uint32_t)kMaxSeg, (v + kSegLen - 1) / kSegLen); };
  auto key_of = [](uint32_t v, uint32_t j, uint32_t ns) {
    const uint32_t len = j + 1 < ns ? (uint32_t)kSegLen : v - j * kSegLen;
    return (uint32_t)(kItemBuckets - 1) - min(len >> 2, (uint32_t)(kItemBuckets - 1));
  };
  auto walk_of = [](uint2 r) { return r.y > r.x ? r.y - r.x : 0u; };
  // every segment but a tile's last has kSegLen entries, so one key: those
  // are counted and placed one wave at a time (a wave scan and one atomic),
  // the last segments one at a time
  const uint32_t key_inner = key_of(kSegLen, 0u, 2u);
  for (int k = tid; k < kItemBuckets; k += NT) sm.cnt[k] = 0u;
  __syncthreads();
  uint2 rg[R];
  uint32_t tw[R], off[R];
  auto load = [&](int cb, bool with_off) {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int i = cb + R * tid + m;
      rg[m] = make_uint2(0u, 0u);
      tw[m] = 0u;
      if (i < ntiles) {
        rg[m] = w.crange[i];
        tw[m] = w.tile_walk[i];
        if (with_off) off[m] = w.walk_off[i];
      }
    }
  };
  // the first rows and the bucket counts
  uint32_t carry = 0;
  for (int cb = 0; cb < ntiles; cb += CH) {
    load(cb, false);
    uint32_t s = 0, ninner = 0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      off[m] = s;
      s += walk_of(rg[m]);
    }
    uint32_t tot;
    const uint32_t pre = carry + block_excl_u32<NT>(s, tot, sm.part);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int i = cb + R * tid + m;
      off[m] += pre;
      if (i < ntiles) w.walk_off[i] = off[m];
      const uint32_t v = walk_of(rg[m]), ns = nseg_of(v);
      if (ns > 0u) {
        atomicAdd(&sm.cnt[key_of(v, ns - 1u, ns)], 1u);
        ninner += ns - 1u;
      }
    }
    uint32_t wt;
    wave_excl_u32(ninner, wt);
    if (lane == 0 && wt > 0u) atomicAdd(&sm.cnt[key_inner], wt);
    carry += tot;
  }
  __syncthreads();
  // the buckets' first places
  {
    constexpr int BPT = kItemBuckets / NT;
    uint32_t c[BPT], s = 0;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      c[b] = sm.cnt[BPT * tid + b];
      s += c[b];
    }
    uint32_t tot;
    uint32_t run = block_excl_u32<NT>(s, tot, sm.part);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      sm.cnt[BPT * tid + b] = run;
      run += c[b];
    }
    if (tid == 0) sm.total = tot;
  }
  __syncthreads();
  const uint32_t cap = (uint32_t)ntiles * (uint32_t)kMaxSeg;
  const uint32_t ccap =
      (uint32_t)min((uint64_t)(kSuper * kSuper) * max_pairs, (uint64_t)0xFFFFFFFFu);
  const bool resident = ntiles <= CH;
  for (int cb = 0; cb < ntiles; cb += CH) {
    if (!resident) load(cb, true);
    // places of the thread's inner segments: the wave's block plus the offset
    uint32_t ninner = 0;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const uint32_t ns = nseg_of(walk_of(rg[m]));
      ninner += ns > 0u ? ns - 1u : 0u;
    }
    uint32_t wt;
    const uint32_t woff = wave_excl_u32(ninner, wt);
    uint32_t wbase = 0u;
    if (lane == 0 && wt > 0u) wbase = atomicAdd(&sm.cnt[key_inner], wt);
    uint32_t ipos = __shfl(wbase, 0, 64) + woff;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int i = cb + R * tid + m;
      if (i >= ntiles) break;
      const uint2 cr = rg[m];
      const uint2 r = clamp_range(cr, ccap);
      const uint32_t v = walk_of(cr), ns = nseg_of(v);
      const bool rows_ok = tw[m] == cr.y && cr.y == r.y &&
                           (uint64_t)off[m] + (r.y - r.x) <= (uint64_t)w.row_cap;
      for (uint32_t j = 0; j < ns; ++j) {
        const bool inner = j + 1 < ns;
        const uint32_t pos = inner ? ipos++ : atomicAdd(&sm.cnt[key_of(v, j, ns)], 1u);
        const uint32_t q1 = min(r.x + j * kSegLen, r.y);
        const uint32_t q2 = inner ? min(q1 + kSegLen, r.y) : r.y;
        if (pos < cap)
          w.seg_order[pos] = make_uint4((uint32_t)i | (j << 24) | ((inner ? 1u : 0u) << 30) |
                                            ((rows_ok ? 1u : 0u) << 31),
                                        q1, q2, off[m] - r.x);
      }
    }
  }
  if (tid == 0) w.seg_n[0] = min(sm.total, cap);
}

// The adjoint's slot bases: slot_blk = the exclusive scan of the preprocess's
// per-block slot counts (one workgroup of NT threads; rerun by every adjoint,
// so a second adjoint of the same forward finds the same bases).
template <int NT>
__device__ void scan_slot_blocks(const WsView& w, int nblk, uint32_t* part) {
  uint32_t carry = 0;
  for (int b = 0; b < nblk; b += NT) {
    const int k = b + (int)threadIdx.x;
    const uint32_t v = k < nblk ? w.slot_cnt[k] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_u32<NT>(v, tot, part);
    if (k < nblk) w.slot_blk[k] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(1024) void k_walk_scan(WsView w, int ntiles, uint32_t max_pairs,
                                                    int nslot_blk) {
  __shared__ ItemScratch sm;
  build_adjoint_items<1024>(w, ntiles, max_pairs, sm);
  __syncthreads();
  scan_slot_blocks<1024>(w, nslot_blk, sm.part);
}

hipError_t launch_adjoint_items(const Layout& L, const WsView& w, hipStream_t s) {
  hipLaunchKernelGGL(k_walk_scan, dim3(1), dim3(1024), 0, s, w, L.ntiles, (uint32_t)L.max_pairs,
                     (int)(L.P > 0 ? L.pose_blocks : 0));
  return hipGetLastError();
}

// Visibility record (Sec. 3.2 keyframe selection, Eq. 5): v_i = 1 when
// Gaussian i is blended at some pixel while the transmittance in front of it
// exceeds t_vis.  One workgroup per tile replays the forward's walk of the
// tile's list (the ids it recorded, up to its walk end) in batches of 64 with
// the forward's alpha and transmittance arithmetic, so every decision is the
// forward's; it stops once no pixel of the tile can still mark a Gaussian
// (transmittance only falls along the list).  visible must be zero before.
__global__ __launch_bounds__(kBlock) void k_visibility(DevSettings st, int64_t P, int W, int H,
                                                       int tiles_x, int ntiles, WsView w,
                                                       float t_vis, uint32_t ccap,
                                                       uint8_t* __restrict__ visible) {
  __shared__ float4 s_r0[64], s_r1[64];
  __shared__ uint32_t s_id[64];
  __shared__ uint32_t s_vis[2];  // the batch's marked Gaussians: bits 0-31, 32-63
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;  // uniform
  const int tid = threadIdx.x, lane = tid & 63;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid & (kTile - 1)), py = ty * kTile + tid / kTile;
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  // the walked range, inside the walked lists whatever the workspace holds
  const uint2 craw = w.crange[tile];
  if (GSFF_CHECKED && tid == 0) GSFF_CHECK(w.status, GSFF_CHECK_WALK, craw.y, (uint64_t)ccap + 1u);
  const uint2 cr = clamp_range(craw, ccap);
  float T = 1.f;
  bool done = !inside;
  for (uint32_t b = cr.x; b < cr.y; b += 64u) {
    const uint32_t n = min(64u, cr.y - b);
    if (tid < 64) {
      const uint32_t gid = (uint32_t)tid < n ? w.clist[b + (uint32_t)tid] : (uint32_t)P;
      if (GSFF_CHECKED && (uint32_t)tid < n) GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, gid, (uint64_t)P);
      float4 q0, q1, q2;
      load_record(w, gid, P, q0, q1, q2);
      s_r0[tid] = scaled_r0(q0);
      s_r1[tid] = scaled_r1(q1);
      s_id[tid] = gid;
    }
    if (tid < 2) s_vis[tid] = 0u;
    __syncthreads();
    uint32_t lo = 0u, hi = 0u;
    for (uint32_t j = 0; j < n; ++j) {
      const AlphaEval e = eval_alpha(s_r0[j], s_r1[j], pxc, pyc, st.alpha_max);
      const bool valid = !done && e.alpha >= st.alpha_min;
      const float Tn = __builtin_fmaf(-e.alpha, T, T);  // as the forward
      const bool stop = valid && Tn < st.t_min;
      const bool use = valid && !stop;
      if (use && T > t_vis) {
        if (j < 32u) lo |= 1u << j;
        else hi |= 1u << (j - 32u);
      }
      done = done || stop;
      T = use ? Tn : T;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo |= (uint32_t)__shfl_xor((int)lo, off, 64);
      hi |= (uint32_t)__shfl_xor((int)hi, off, 64);
    }
    if (lane == 0) {
      if (lo) atomicOr(&s_vis[0], lo);
      if (hi) atomicOr(&s_vis[1], hi);
    }
    // a pixel can still mark a later Gaussian only while T > t_vis
    const int live = __syncthreads_or(!done && T > t_vis);
    if (tid < 64 && (uint32_t)tid < n && ((s_vis[tid >> 5] >> (tid & 31)) & 1u) &&
        s_id[tid] < (uint32_t)P)
      visible[s_id[tid]] = 1;
    if (!live) break;  // uniform
    __syncthreads();   // the next batch overwrites the staged records
  }
}

hipError_t launch_visibility(const DevSettings& st, const DevGaussians& g, const Layout& L,
                             const WsView& w, float t_vis, uint8_t* visible, hipStream_t s) {
  if (L.P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero<uint8_t>, dim3((unsigned)((L.P + 255) / 256)), dim3(256), 0, s,
                     visible, (int64_t)L.P);
  if (L.ntiles > 0)
    hipLaunchKernelGGL(k_visibility, dim3((unsigned)L.ntiles), dim3(kBlock), 0, s, st, g.P, L.W,
                       L.H, L.tiles_x, L.ntiles, w, t_vis,
                       (uint32_t)min((uint64_t)(kSuper * kSuper) * (uint64_t)L.max_pairs,
                                     (uint64_t)0xFFFFFFFFu),
                       visible);
  return hipGetLastError();
}

// |a and b| and |a or b| of two visibility records (non-zero = visible), for
// the co-visibility test; counts[2] must be zero before.
__global__ __launch_bounds__(256) void k_covisibility(const uint8_t* __restrict__ a,
                                                      const uint8_t* __restrict__ b, int64_t n,
                                                      uint32_t* __restrict__ counts) {
  uint32_t both = 0u, any = 0u;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const bool x = a[i] != 0, y = b[i] != 0;
    both += (x && y) ? 1u : 0u;
    any += (x || y) ? 1u : 0u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    both += (uint32_t)__shfl_xor((int)both, off, 64);
    any += (uint32_t)__shfl_xor((int)any, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (both) atomicAdd(&counts[0], both);
    if (any) atomicAdd(&counts[1], any);
  }
}

// Keyframe decision (Sec. 3.2): IoU = |a and b| / |a or b| of the two
// records (1 when both are empty) below tau_thresh, compared in FP64.
__global__ void k_keyframe_decide(const uint32_t* __restrict__ counts, float tau,
                                  uint32_t* __restrict__ keyframe) {
  if (threadIdx.x != 0) return;
  const uint32_t both = counts[0], either = counts[1];
  const double iou = either ? (double)both / (double)either : 1.0;
  keyframe[0] = iou < (double)tau ? 1u : 0u;
}

hipError_t launch_covisibility(const uint8_t* a, const uint8_t* b, int64_t n, uint32_t* counts,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero<uint32_t>, dim3(1), dim3(64), 0, s, counts, (int64_t)2);
  if (n > 0) {
    const int64_t blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_covisibility, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n, counts);
  }
  return hipGetLastError();
}

hipError_t launch_keyframe_decide(const uint32_t* counts, float tau, uint32_t* keyframe,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_keyframe_decide, dim3(1), dim3(64), 0, s, counts, tau, keyframe);
  return hipGetLastError();
}

template <int CP, typename FT, typename OT>
static void launch_fwd_t(const DevSettings& st, const DevGaussians& g, const Layout& L,
                         const WsView& w, int c0, float* out_rgb, float* out_depth,
                         float* out_alpha, void* out_feat, int write_geo, hipStream_t s) {
  const int grid = ((L.ntiles + kNumXcd - 1) / kNumXcd) * kNumXcd;
  hipLaunchKernelGGL((k_composite_fwd<CP, FT, OT>), dim3(grid), dim3(kBlock), 0, s, st, g.P, g.C,
                     c0, L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, (uint32_t)L.max_pairs, w,
                     (const FT*)g.feat, out_rgb, out_depth, out_alpha, (OT*)out_feat, write_geo);
}

template <typename FT, typename OT>
static void launch_fwd_dispatch(int cn, const DevSettings& st, const DevGaussians& g,
                                const Layout& L, const WsView& w, int c0, float* out_rgb,
                                float* out_depth, float* out_alpha, void* out_feat,
                                int write_geo, hipStream_t s) {
  if (cn <= 0)
    launch_fwd_t<0, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, nullptr, write_geo, s);
  else if (cn <= 8)
    launch_fwd_t<8, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else if (cn <= 16)
    launch_fwd_t<16, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else if (cn <= 32)
    launch_fwd_t<32, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
  else
    launch_fwd_t<64, FT, OT>(st, g, L, w, c0, out_rgb, out_depth, out_alpha, out_feat, write_geo, s);
}

hipError_t launch_composite_fwd(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                const WsView& w, float* out_rgb, float* out_depth,
                                float* out_alpha, void* out_feat, int32_t out_feat_dtype,
                                hipStream_t s) {
  const bool feat_on = st.render_features && g.C > 0 && out_feat != nullptr;
  const int64_t HW = (int64_t)L.W * L.H;
  if (!feat_on && out_feat && g.C > 0) {
    const int64_t n = HW * g.C;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (out_feat_dtype == GSFF_DTYPE_BF16)
      hipLaunchKernelGGL(k_fill_zero<uint16_t>, dim3(blocks), dim3(256), 0, s,
                         (uint16_t*)out_feat, n);
    else
      hipLaunchKernelGGL(k_fill_zero<float>, dim3(blocks), dim3(256), 0, s, (float*)out_feat, n);
  }
  const int nchunks = feat_on ? (g.C + GSFF_MAX_CHANNELS_PER_PASS - 1) / GSFF_MAX_CHANNELS_PER_PASS
                              : 1;
  for (int k = 0; k < nchunks; ++k) {
    const int c0 = k * GSFF_MAX_CHANNELS_PER_PASS;
    const int cn = feat_on ? min(GSFF_MAX_CHANNELS_PER_PASS, g.C - c0) : 0;
    const int wg = (k == 0);
    const bool obf = out_feat_dtype == GSFF_DTYPE_BF16;
    if (g.feat_dtype == GSFF_DTYPE_BF16) {
      if (obf)
        launch_fwd_dispatch<uint16_t, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth,
                                                out_alpha, out_feat, wg, s);
      else
        launch_fwd_dispatch<uint16_t, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
    } else if (g.feat_dtype == GSFF_DTYPE_F16) {
      if (obf)
        launch_fwd_dispatch<_Float16, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth,
                                                out_alpha, out_feat, wg, s);
      else
        launch_fwd_dispatch<_Float16, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
    } else {
      if (obf)
        launch_fwd_dispatch<float, uint16_t>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                             out_feat, wg, s);
      else
        launch_fwd_dispatch<float, float>(cn, st, g, L, w, c0, out_rgb, out_depth, out_alpha,
                                          out_feat, wg, s);
    }
  }
  return hipGetLastError();
}

// ----------------------------------------------------------- backward -----

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}


constexpr int kBwdNB = 16;              // Gaussians per batch = rows of the contraction
constexpr int kBwdStride = kBlock + 4;  // LDS row stride (floats) of the per-pair products
constexpr int kBwdGeoChannels = 32;     // feature channels carried by the geometry pass
constexpr int kBwdMaxChannels = 64;     // feature channels of a feature-only pass


// Upstream gradient formed inside the adjoint for the L1 losses of the
// method (Eqs. 6, 8, 11 are weighted sums of L1 terms):
//   L = sum_k w_k * mean|out_k - target_k|  over the groups rgb, depth, alpha,
// feature; the per-element gradient is (w_k / numel_k) sign(out - target).
// A group with a NULL target does not enter the loss.
struct L1Upstream {
  const float* out_rgb;
  const float* out_depth;
  const float* out_alpha;
  const float* out_feat;
  const float* t_rgb;
  const float* t_depth;
  const float* t_alpha;
  const float* t_feat;
  float s_rgb, s_depth, s_alpha, s_feat;  // w_k / numel_k
  float* loss;                            // += the loss (may be NULL)
  const uint8_t* mask_v;                  // zero: no colour or depth term here
  const uint8_t* mask_e;                  // zero: no colour term here
};

// The L1 upstream of every pixel in 2-bit codes (0: zero, 1: +1, 2: -1),
// formed once per adjoint call: plane 0 holds r, g, b, depth, alpha at bits
// 0-9, plane 1 + k the feature channels 16 k .. 16 k + 15.  Groups without a
// target are zero, and so are the colour and depth groups of a pixel the
// tracking masks leave out (Eq. 6: m_v m_e on colour, m_v on depth).  The
// pass also adds the loss.
//
// The same launch does the adjoint's other set-up, which shares no data with
// the codes: its first workgroup builds the work items and its second scans
// the slot bases (each a workgroup of dependent steps, which would otherwise
// be a launch of its own on the critical path); for a call that does not
// accumulate, the first sets the loss to zero (loss_zero; the adjoint then
// adds it) while the code workgroups clear the feature gradient (n_zero
// floats at zero).
__device__ __forceinline__ uint32_t l1_code(float o, float t, float scale, float& l) {
  const float d = o - t;
  l += fabsf(d) * scale;
  return d > 0.f ? 1u : (d < 0.f ? 2u : 0u);
}
__device__ __forceinline__ float l1_decode(uint32_t word, int slot) {
  const uint32_t c = (word >> (2 * slot)) & 3u;
  return c == 1u ? 1.f : (c == 2u ? -1.f : 0.f);
}
__global__ __launch_bounds__(256) void k_l1_codes(L1Upstream l1, int64_t HW, int C,
                                                  uint32_t* __restrict__ codes,
                                                  float* __restrict__ loss_part, WsView w,
                                                  int ntiles, uint32_t max_pairs,
                                                  float* __restrict__ zero, int64_t n_zero,
                                                  float* __restrict__ loss_zero, int nslot_blk) {
  __shared__ float s_l[4];
  __shared__ ItemScratch s_items;
  if (blockIdx.x == 0) {  // uniform
    if (loss_zero && threadIdx.x == 0) *loss_zero = 0.f;
    build_adjoint_items<256>(w, ntiles, max_pairs, s_items);
    return;
  }
  if (blockIdx.x == 1) {  // uniform
    scan_slot_blocks<256>(w, nslot_blk, s_items.part);
    return;
  }
  const int64_t wg = (int64_t)blockIdx.x - 2, nwg = (int64_t)gridDim.x - 2;
  const int64_t p = wg * 256 + threadIdx.x;
  float loss = 0.f;
  if (p < HW) {
    // every load of the pixel is issued before any code is formed
    float o[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, t[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (l1.t_rgb) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        o[k] = l1.out_rgb[k * HW + p];
        t[k] = l1.t_rgb[k * HW + p];
      }
    }
    if (l1.t_depth) {
      o[3] = l1.out_depth[p];
      t[3] = l1.t_depth[p];
    }
    if (l1.t_alpha) {
      o[4] = l1.out_alpha[p];
      t[4] = l1.t_alpha[p];
    }
    const bool feat = l1.t_feat != nullptr && C > 0;
    float fo[16], ft[16];
    if (feat) {  // the first 16 channels with the rest (channels past C read channel C - 1)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t q = (int64_t)min(j, C - 1) * HW + p;
        fo[j] = l1.out_feat[q];
        ft[j] = l1.t_feat[q];
      }
    }
    const bool in_v = !l1.mask_v || l1.mask_v[p] != 0;
    const bool in_c = in_v && (!l1.mask_e || l1.mask_e[p] != 0);
    uint32_t w0 = 0u;
    if (l1.t_rgb && in_c) {
#pragma unroll
      for (int k = 0; k < 3; ++k) w0 |= l1_code(o[k], t[k], l1.s_rgb, loss) << (2 * k);
    }
    if (l1.t_depth && in_v) w0 |= l1_code(o[3], t[3], l1.s_depth, loss) << 6;
    if (l1.t_alpha) w0 |= l1_code(o[4], t[4], l1.s_alpha, loss) << 8;
    codes[p] = w0;
    if (feat) {
      for (int cb = 0; cb < C; cb += 16) {
        if (cb > 0) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int64_t q = (int64_t)min(cb + j, C - 1) * HW + p;
            fo[j] = l1.out_feat[q];
            ft[j] = l1.t_feat[q];
          }
        }
        uint32_t wf = 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          float l = 0.f;
          const uint32_t c = l1_code(fo[j], ft[j], l1.s_feat, l);
          if (cb + j < C) {
            wf |= c << (2 * j);
            loss += l;
          }
        }
        codes[(int64_t)(1 + cb / 16) * HW + p] = wf;
      }
    }
  }
  for (int64_t q = p; q < n_zero; q += nwg * 256) zero[q] = 0.f;
  // the workgroup's share of the loss; the adjoint's first workgroup adds
  // the shares up (one atomic instead of one per workgroup on one address)
  if (l1.loss && wg * 256 < HW) {  // uniform
    const float v = wave_sum(loss);
    if ((threadIdx.x & 63) == 0) s_l[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[wg] = (s_l[0] + s_l[1]) + (s_l[2] + s_l[3]);
  }
}


// The per-pixel adjoint of a tile, with the per-Gaussian sums as matrix
// products on the matrix cores.
//
// Every gradient a Gaussian i receives from a tile is a sum over the tile's
// pixels p of one of two per-pair values times a per-pixel quantity:
//   colour, depth, feature k : sum_p w_ip g_k(p)           (w = blending weight)
//   image-space mean, conic  : sums of dL/dpower_ip times 1, x, y, x^2, xy, y^2
//                              (pixel centre relative to the tile centre),
//                              from which du, dv, dA, dB, dC follow in closed form
//   opacity                  : sum_p dL/dpower_ip / o_i
// For a batch of 16 Gaussians these are the products W (16 x 256) * G
// (256 x channels) and DP (16 x 256) * M (256 x 6).
//
// Per batch (back to front over the tile's list):
//  phase A  one thread per pixel walks the 16 Gaussians back to front,
//           recovering T_i = T_{i+1} / (1 - alpha_i) from the final
//           transmittance, and writes w_ip and dL/dpower_ip (zero where the
//           pixel does not use Gaussian i, or alpha is clamped) to LDS.  With
//           D = sum over the contributors behind i of w_m (g . c_m),
//             dL/dalpha_i = T_i (g . c_i) + (g_alpha T_final - D) / (1 - alpha_i).
//  phase B  one wave per 16-column output block runs the K = 256 contraction
//           with 16x16x32 BF16 MFMA: the FP32 left operand is split as hi + lo
//           (both BF16), the right operand is either exact in BF16 (L1 signs,
//           moments of half-integer coordinates) or split the same way, so
//           every product is kept to about 2^-16 relative; accumulation is FP32.
//           The accumulator lanes then add their (Gaussian, channel) results
//           to the global gradients.
// Geometry terms come only from the colour, depth and opacity upstream; the
// feature upstream only enters the feature sums (Sec. 3.1, last paragraph).
// Register budget: four waves per SIMD (four workgroups per CU, which the
// LDS use also allows); the explicit-upstream variant keeps twice the right
// operands in registers and runs three.

template <int CP, bool GEO, bool L1>
__global__ __attribute__((amdgpu_flat_work_group_size(kBlock, kBlock),
                          amdgpu_waves_per_eu(L1 ? 4 : 3))) void k_composite_bwd(
    DevSettings st, int64_t P, int C, int c0, int W, int H, int tiles_x, int ntiles,
    int rank_bits, uint32_t max_pairs, WsView w, const float* __restrict__ g_rgb,
    const float* __restrict__ g_depth, const float* __restrict__ g_alpha,
    const float* __restrict__ g_feat, float* __restrict__ d_feat, L1Upstream l1, int first_pass,
    int zero_geo, int zero_feat) {
  constexpr int NL = (GEO ? 4 : 0) + CP;      // linear channels: r, g, b, depth, features
  constexpr int NCB = (NL + 15) / 16;         // 16-column blocks of W * G
  constexpr int NT = NCB + (GEO ? 1 : 0);     // output blocks (+ the moments block)
  static_assert(NT <= kBlock / 64, "one wave per output block");
  static_assert(NL > 0, "nothing to differentiate");
  __shared__ __attribute__((aligned(16))) float s_W[kBwdNB][kBwdStride];
  __shared__ __attribute__((aligned(16))) float s_DP[GEO ? kBwdNB : 1][GEO ? kBwdStride : 4];
  __shared__ float4 s_r0[2][kBwdNB], s_r1[2][kBwdNB], s_r2[2][kBwdNB];
  __shared__ uint32_t s_gid[2][kBwdNB];
  __shared__ float s_mom[kBwdNB][8];
  if (L1 && first_pass && l1.loss && blockIdx.x == 0) {
    // the L1 loss: the shares the code pass left, one per 256 pixels
    __shared__ float s_part[kBlock / 64];
    const int nparts = (W * H + 255) / 256;
    float v = 0.f;
    for (int i = threadIdx.x; i < nparts; i += kBlock) v += w.loss_part[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
      if (t != 0.f) unsafeAtomicAdd(l1.loss, t);
    }
  }
  // work item: a segment [q1, q2) of a tile's walked list (longest first)
  if (blockIdx.x >= min(w.seg_n[0], (uint32_t)ntiles * (uint32_t)kMaxSeg)) return;
  const uint4 item = w.seg_order[blockIdx.x];
  const int tile = (int)(item.x & 0xFFFFFFu), seg = (int)((item.x >> 24) & 63u);
  const bool inner = ((item.x >> 30) & 1u) != 0u;  // a later segment follows
  const bool rows_ok = (item.x >> 31) != 0u;       // the tile's rows fit
  const uint32_t q1 = item.y, q2 = item.z;
  const uint32_t rowbase = item.w;  // row of list position p: rowbase + p
  if (!guard(w.status, GSFF_CHECK_ITEM, tile, ntiles)) return;
  if (GSFF_CHECKED) {  // list range inside the walked lists, a recorded state per inner segment
    const uint64_t ccap = min((uint64_t)(kSuper * kSuper) * max_pairs, (uint64_t)0xFFFFFFFFu);
    if (!GSFF_CHECK(w.status, GSFF_CHECK_ITEM, q1, (uint64_t)q2 + 1u) ||
        !GSFF_CHECK(w.status, GSFF_CHECK_ITEM, q2, ccap + 1u) ||
        (inner && !GSFF_CHECK(w.status, GSFF_CHECK_ITEM, (uint64_t)seg, (uint64_t)(kMaxSeg - 1))))
      return;
  }
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, lq = lane >> 4, lj = lane & 15;
  const int px = tx * kTile + (tid & (kTile - 1));
  const int py = ty * kTile + (tid / kTile);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const int cn = CP > 0 ? min(CP, C - c0) : 0;
  const int64_t HW = (int64_t)W * H;
  const int64_t p = (int64_t)py * W + px;

  // Batches run back to front: [b0, b1), then [nb0, nb1 = b0), then
  // [mb0, mb1 = nb0), ...; only the front-most one can be shorter than 16.
  // Loads are pipelined: while batch b is processed, the records of b+1
  // (whose ids arrived during b-1) and the ids of b+2 are in flight.
  const uint32_t rx = q1;
  auto batch_start = [rx](uint32_t end) {
    return end > rx ? end - min((uint32_t)kBwdNB, end - rx) : end;
  };
  // The loads are issued by the first 16 lanes of the last wave, which has no
  // output block when NT < 4 (its memory queue then holds no gradient atomics).
  // Ids stay unchecked until use: load_record and the atomics test id < P.
  // The ids of the first two batches are the first loads of the item.
  const int pf = tid - (kBlock - 64);
  const bool pf_lane = pf >= 0 && pf < kBwdNB;
  uint32_t b1 = q2, b0 = batch_start(b1);
  uint32_t nb1 = b0, nb0 = batch_start(nb1);
  uint32_t gid0 = (uint32_t)P, g_next = (uint32_t)P;  // per prefetch lane
  if (pf_lane) {
    if (b0 + pf < b1) gid0 = w.clist[b0 + pf];
    if (nb0 + pf < nb1) g_next = w.clist[nb0 + pf];
    if (GSFF_CHECKED) {  // every walked entry is a Gaussian id
      if (b0 + pf < b1) GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, gid0, (uint64_t)P);
      if (nb0 + pf < nb1) GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, g_next, (uint64_t)P);
    }
  }


  // ---- per-pixel state and upstream gradients
  float Tfin = 1.f;
  uint32_t pend = q1;
  float gr = 0.f, gg = 0.f, gb = 0.f, gd = 0.f, ga = 0.f;  // geometry upstream (scaled)
  float ur = 0.f, ug = 0.f, ub = 0.f, ud = 0.f;           // same, as contraction operands
  // Every per-pixel load is issued up front, unconditionally (a pixel
  // outside the image reads pixel 0 and masks the value), so the loads are
  // in flight together instead of one round trip each.
  const int64_t pq = inside ? p : 0;
  {
    const float tf = w.pix_T[pq];
    const uint32_t pe = w.pix_end[pq];
    Tfin = inside ? tf : 1.f;
    pend = inside ? pe : q1;
  }
  // the feature upstream of the first staging round (RS 16-column blocks),
  // issued with the per-pixel loads: channels past cn and pixels outside the
  // image read channel c0 / pixel 0, masked where the values are formed
  constexpr int RS = GEO ? 2 : 1;
  float fo[RS][16];
  auto load_round = [&](int r) {
#pragma unroll
    for (int u = 0; u < RS; ++u)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        fo[u][j] = 0.f;
      }
    if constexpr (CP > 0 && L1) {
      // the block's channels lie in two code planes at most: both loaded
#pragma unroll
      for (int u = 0; u < RS; ++u) {
        const int first = c0 + 16 * (r * RS + u) - (GEO ? 4 : 0);  // channel of column 0
        const int plane = (first > 0 ? first : 0) >> 4;
        const uint32_t wa = w.l1_codes[(int64_t)(1 + plane) * HW + pq];
        const uint32_t wb = (plane + 1) * 16 < C ? w.l1_codes[(int64_t)(2 + plane) * HW + pq] : 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = 16 * (r * RS + u) + j;
          const int c = k - (GEO ? 4 : 0);
          if (k < NL && c >= 0) {
            const int gch = c0 + c;
            fo[u][j] = l1_decode((gch >> 4) == plane ? wa : wb, gch & 15);
          }
        }
      }
    } else if constexpr (CP > 0) {  // (launched with CP > 0 only when cn >= 1)
#pragma unroll
      for (int u = 0; u < RS; ++u)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = 16 * (r * RS + u) + j;
          const int c = k - (GEO ? 4 : 0);
          if (k < NL && c >= 0) {
            const int64_t q = (int64_t)(c0 + (c < cn ? c : 0)) * HW + pq;
            fo[u][j] = g_feat[q];
          }
        }
    }
  };
  load_round(0);
  // the records of the first batch, once their ids (the first loads) arrive:
  // every lane loads, with no branch to hold the wait (lanes that stage no
  // record and ids past the end read Gaussian 0, masked where staged)
  const int64_t g0 = gid0 < (uint32_t)P ? (int64_t)gid0 : 0;
  const float4 f0 = w.rec[g0], f1 = w.rec[P + g0], f2 = w.rec[2 * P + g0];
  // the state at this segment's end as the forward recorded it (when a later
  // segment follows): T and the colour and depth blended in front of it, and
  // the tile's final colour and depth
  float sst[5] = {1.f, 0.f, 0.f, 0.f, 0.f}, sfin[4] = {0.f, 0.f, 0.f, 0.f};
  if (inner) {
    const float* q = w.seg_state + ((int64_t)tile * (kMaxSeg - 1) + seg) * 5 * kBlock + tid;
    const float* f = w.seg_final + (int64_t)tile * 4 * kBlock + tid;
#pragma unroll
    for (int k = 0; k < 5; ++k) sst[k] = q[k * kBlock];
#pragma unroll
    for (int k = 0; k < 4; ++k) sfin[k] = f[k * kBlock];
  }
  if constexpr (GEO) {
    if constexpr (L1) {
      const uint32_t w0 = w.l1_codes[pq];
      const float m = inside ? 1.f : 0.f;
      ur = m * l1_decode(w0, 0);
      ug = m * l1_decode(w0, 1);
      ub = m * l1_decode(w0, 2);
      ud = m * l1_decode(w0, 3);
      ga = m * l1_decode(w0, 4) * l1.s_alpha;
      gr = ur * l1.s_rgb;
      gg = ug * l1.s_rgb;
      gb = ub * l1.s_rgb;
      gd = ud * l1.s_depth;
    } else {
      const float a0 = g_rgb[pq], a1 = g_rgb[HW + pq], a2 = g_rgb[2 * HW + pq];
      const float a3 = g_depth[pq], a4 = g_alpha[pq];
      gr = ur = inside ? a0 : 0.f;
      gg = ug = inside ? a1 : 0.f;
      gb = ub = inside ? a2 : 0.f;
      gd = ud = inside ? a3 : 0.f;
      ga = inside ? a4 : 0.f;
    }
  }
  // transmittance and D at the segment's end: the final values for the last
  // segment, the recorded ones for the others
  float T = Tfin, D = 0.f;
  if (inner) {
    T = inside ? sst[0] : 1.f;
    if constexpr (GEO)
      D = inside ? gr * (sfin[0] - sst[1]) + gg * (sfin[1] - sst[2]) + gb * (sfin[2] - sst[3]) +
                       gd * (sfin[3] - sst[4])
                 : 0.f;
  }

  // ---- right operands, kept in registers for the tile: wave b < NCB holds
  // G[pixels 32s + 8 lq .. +7][channel 16 b + lj] for s = 0..7, the moments
  // wave (b = NCB) the moment values of the same pixels.
  // The per-pixel values are staged through LDS, RS 16-channel blocks at a
  // time (s_W, and s_DP when the geometry terms are on).
  bf16x8 bh[8], bl[8];
#pragma unroll
  for (int r = 0; r < (NCB + RS - 1) / RS; ++r) {
    if (r > 0) {
      load_round(r);
      lds_barrier();  // the staging rows are free again
    }
#pragma unroll
    for (int u = 0; u < RS; ++u) {
      float* rows_u = u == 0 ? &s_W[0][0] : &s_DP[0][0];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = 16 * (r * RS + u) + j;
        float v = 0.f;
        if (k < NL) {
          if (GEO && k < 4) {
            v = k == 0 ? ur : (k == 1 ? ug : (k == 2 ? ub : ud));
          } else {
            const int c = k - (GEO ? 4 : 0);
            const bool on = inside && c < cn;
            v = on ? fo[u][j] : 0.f;
          }
        }
        if (r * RS + u < NCB) rows_u[j * kBwdStride + tid] = v;
      }
    }
    if (r == 0 && pf_lane) {  // the first batch's records have arrived by now
      const bool ok = gid0 < (uint32_t)P;
      s_gid[0][pf] = gid0;
      s_r0[0][pf] = scaled_r0(keep4(ok, f0));
      s_r1[0][pf] = scaled_r1(keep4(ok, f1));
      s_r2[0][pf] = keep4(ok, f2);
    }
    lds_barrier();
    if (wave >= r * RS && wave < r * RS + RS && wave < NCB) {
      const float* rows_w = wave == r * RS ? &s_W[0][0] : &s_DP[0][0];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const float* src = rows_w + lj * kBwdStride + 32 * s + 8 * lq;
        const float4 a = *reinterpret_cast<const float4*>(src);
        const float4 b = *reinterpret_cast<const float4*>(src + 4);
        if (L1) {
          bh[s] = to_bf16x8(a, b);  // signs: exact
        } else {
          split8(a, b, bh[s], bl[s]);
        }
      }
    }
  }
  if constexpr (GEO) {
    // the moments wave: right operand M[pixel][j] = 1, x, y, x^2, xy, y^2 for
    // j = lj (zero for lj >= 6), pixel 32 s + 8 lq + t at x = 8 (lq & 1) + t - 7.5,
    // y = 2 s + lq / 2 - 7.5 relative to the tile centre; products of
    // half-integers below 8 in magnitude, so exact in BF16
    if (wave == NCB) {
      const float c0 = lj == 0 ? 1.f : 0.f, c1 = lj == 1 ? 1.f : 0.f;
      const float c2 = lj == 2 ? 1.f : 0.f, c3 = lj == 3 ? 1.f : 0.f;
      const float c4 = lj == 4 ? 1.f : 0.f, c5 = lj == 5 ? 1.f : 0.f;
      const float x0 = (float)(8 * (lq & 1)) - 7.5f;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const float y = (float)(2 * s + (lq >> 1)) - 7.5f;
        const float base = __builtin_fmaf(y, __builtin_fmaf(c5, y, c2), c0);
        const float lin = __builtin_fmaf(c4, y, c1);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float x = x0 + (float)t;
          bh[s][t] = (__bf16)__builtin_fmaf(x, __builtin_fmaf(c3, x, lin), base);
        }
      }
    }
  }
  lds_barrier();
  if (q1 >= q2) return;  // uniform: an empty segment
  // The tile's results go to one row per walked list position (the rows of
  // the tiles follow each other in tile order) when they fit; otherwise they
  // are added to the per-Gaussian gradients with atomics.
  const int RW = w.row_width;

  const float gaT = ga * Tfin;
  const float tcx = (float)(tx * kTile) + 0.5f * kTile, tcy = (float)(ty * kTile) + 0.5f * kTile;
  int buf = 0;
  while (true) {
    const bool more = nb1 > rx;  // another batch follows this one
    // records of the next batch, ids of the one after
    const uint32_t pgid = g_next;
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0;
    bool pok = false;
    const uint32_t mb1 = nb0, mb0 = batch_start(mb1);
    if (pf_lane) {
      if (more) pok = fetch_record(w, pgid, P, p0, p1, p2);
      g_next = (more && mb0 + pf < mb1) ? w.clist[mb0 + pf] : (uint32_t)P;
      if (GSFF_CHECKED && more && mb0 + pf < mb1)
        GSFF_CHECK(w.status, GSFF_CHECK_LIST_ID, g_next, (uint64_t)P);
    }

    // ---- phase A: per-pixel products, back to front
    const bool wave_any = __ballot(inside && pend > b0) != 0ull;
    if (wave_any) {
      // Branch-free: every value is computed for every (pixel, Gaussian) and
      // masked, so the record reads of later Gaussians can be issued early.
#pragma unroll
      for (int jj = kBwdNB - 1; jj >= 0; --jj) {
        const float4 r0 = s_r0[buf][jj], r1 = s_r1[buf][jj];
        const AlphaEval e = eval_alpha(r0, r1, pxc, pyc, st.alpha_max);
        const bool act = (b0 + (uint32_t)jj < pend) && (e.alpha >= st.alpha_min);
        // a pair the pixel does not use gets alpha 0: then 1 / (1 - alpha) is
        // exactly 1, T passes through and the weight is 0
        const float al = act ? e.alpha : 0.f;
        float gc = 0.f;
        if constexpr (GEO) {
          const float4 r2 = s_r2[buf][jj];
          gc = gr * r2.x + gg * r2.y + gb * r2.z + gd * r1.z;
        }
        float wv, dal;
        back_step(al, gc, gaT, T, D, wv, dal);  // rcp(1) = 1 exactly
        if constexpr (GEO) {
          const float og = (act && e.oG < st.alpha_max) ? e.oG : 0.f;
          s_DP[jj][tid] = dal * og;
        }
        s_W[jj][tid] = wv;
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < kBwdNB; ++jj) {
        s_W[jj][tid] = 0.f;
        if constexpr (GEO) s_DP[jj][tid] = 0.f;
      }
    }
    lds_barrier();

    // ---- phase B: contraction over the tile's pixels on the matrix cores
    if (wave < NCB) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const float* src = &s_W[lj][32 * s + 8 * lq];
        bf16x8 ah, al;
        split8(*reinterpret_cast<const float4*>(src), *reinterpret_cast<const float4*>(src + 4),
               ah, al);
        acc = mfma16(ah, bh[s], acc);
        acc = mfma16(al, bh[s], acc);
        if (!L1) acc = mfma16(ah, bl[s], acc);
      }
      // acc[r]: Gaussian 4 lq + r of the batch, channel 16 wave + lj
      const int k = 16 * wave + lj;
      float scale = 1.f;
      int col = -1;  // column in a row: du dv dA dB dC do dr dg db dz, then features
      float* dst = nullptr;
      int64_t stride = 0;
      if (k < NL) {
        if (GEO && k < 4) {
          if (L1) scale = k < 3 ? l1.s_rgb : l1.s_depth;
          col = k < 3 ? 6 + k : 9;
          dst = w.grad2d + col;
          stride = 10;
        } else {
          const int c = k - (GEO ? 4 : 0);
          if (c < cn) {
            if (L1) scale = l1.s_feat;
            col = 10 + c0 + c;
            dst = d_feat + c0 + c;
            stride = C;
          }
        }
      }
      if (rows_ok) {
        const uint32_t nb = b1 - b0;  // Gaussians in this batch
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t g = 4 * lq + r;
          // (the row index is formed modulo 2^32: rowbase may wrap below zero)
          if (g < nb && GSFF_CHECK(w.status, GSFF_CHECK_ROW, rowbase + b0 + g, w.row_cap)) {
            float* row = w.rows + (int64_t)(rowbase + b0 + g) * RW;
            if (col >= 0) row[col] = acc[r] * scale;
            if (wave == 0 && first_pass) {  // columns no pass of this call writes
              if (zero_geo && lj < 10) row[lj] = 0.f;
              if (zero_feat)
                for (int cc = lj; cc < C; cc += 16) row[10 + cc] = 0.f;
            }
          }
        }
      } else if (dst) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t gid = s_gid[buf][4 * lq + r];
          const float v = acc[r] * scale;
          if (gid < (uint32_t)P && v != 0.f) unsafeAtomicAdd(dst + (int64_t)gid * stride, v);
        }
      }
    } else if constexpr (GEO) {
      if (wave == NCB) {
        // moments of dL/dpower (the right operand, in bh, holds the moments)
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const float* src = &s_DP[lj][32 * s + 8 * lq];
          bf16x8 ah, al;
          split8(*reinterpret_cast<const float4*>(src), *reinterpret_cast<const float4*>(src + 4),
                 ah, al);
          acc = mfma16(ah, bh[s], acc);
          acc = mfma16(al, bh[s], acc);
        }
        if (lj < 6) {
#pragma unroll
          for (int r = 0; r < 4; ++r) s_mom[4 * lq + r][lj] = acc[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < kBwdNB) {
          const uint32_t gid = s_gid[buf][lane];
          if (gid < (uint32_t)P && (rows_ok ? (uint32_t)lane < b1 - b0 : true)) {
            const float4 r0 = s_r0[buf][lane], r1 = s_r1[buf][lane];
            const float cA = r0.z * kConAInv, cB = r0.w * kConBInv, cC = r1.x * kConAInv;
            const float M[6] = {s_mom[lane][0], s_mom[lane][1], s_mom[lane][2],
                                s_mom[lane][3], s_mom[lane][4], s_mom[lane][5]};
            const float udx = r0.x - tcx, vdy = r0.y - tcy;  // mean relative to the tile centre
            float geo[6];
            geo_from_moments(cA, cB, cC, r1.y, udx, vdy, M, geo);
            if (rows_ok) {
              if (GSFF_CHECK(w.status, GSFF_CHECK_ROW, rowbase + b0 + (uint32_t)lane, w.row_cap)) {
                float* row = w.rows + (int64_t)(rowbase + b0 + (uint32_t)lane) * RW;
#pragma unroll
                for (int f = 0; f < 6; ++f) row[f] = geo[f];
              }
            } else {
              float* dst = w.grad2d + (int64_t)gid * 10;
#pragma unroll
              for (int f = 0; f < 6; ++f)
                if (geo[f] != 0.f) unsafeAtomicAdd(dst + f, geo[f]);
            }
          }
        }
      }
    }
    // the first pass files each valid Gaussian's row in the Gaussian's slots
    // (a Gaussian has a slot per tile of its rectangle and meets each tile once)
    // and opens a reduction work item at every 64th slot; in the deterministic
    // mode the row goes to the slot of this tile's place in the rectangle and
    // the reduction visits every Gaussian's slots in order instead
    if (first_pass && rows_ok && pf_lane) {
      const uint32_t gid = s_gid[buf][pf];
      if ((uint32_t)pf < b1 - b0 && gid < (uint32_t)P) {
        const uint32_t row = rowbase + b0 + (uint32_t)pf;
        const uint32_t sbase = w.slot_blk[gid >> 8] + w.slot_local[gid];
        if (st.deterministic) {
          const ushort4 rc = w.rects[gid];
          // the tile lies in the rectangle (its list holds the Gaussian)
          const bool in_rect = tx >= rc.x && tx <= rc.z && ty >= rc.y && ty <= rc.w;
          if (GSFF_CHECKED && !in_rect)
            check_failed(w.status, GSFF_CHECK_SLOT, (uint64_t)tile, (uint64_t)gid);
          if (in_rect) {
            const uint32_t sl = sbase + (uint32_t)(ty - rc.y) * (uint32_t)(rc.z - rc.x + 1) +
                                (uint32_t)(tx - rc.x);
            if (guard(w.status, GSFF_CHECK_SLOT, sl, w.slot_cap)) w.slots[sl] = row;
          }
        } else {
          const uint32_t k = atomicAdd(&w.nslot[gid], 1u);
          const uint32_t sl = sbase + k;
          if (GSFF_CHECKED) {  // a Gaussian meets each tile of its rectangle once
            const ushort4 rc = w.rects[gid];
            const uint64_t nt = (rc.x <= rc.z && rc.y <= rc.w)
                                    ? (uint64_t)(rc.z - rc.x + 1) * (uint64_t)(rc.w - rc.y + 1)
                                    : 0ull;
            GSFF_CHECK(w.status, GSFF_CHECK_SLOT, k, nt);
          }
          if (guard(w.status, GSFF_CHECK_SLOT, sl, w.slot_cap)) w.slots[sl] = row;
          if ((k & 63u) == 0u) {
            const uint32_t t = atomicAdd(w.item_n, 1u);
            if (guard(w.status, GSFF_CHECK_REDUCE, t, w.item_cap))
              w.items[t] = make_uint2(gid, k);
          }
        }
      }
    }
    if (more && pf_lane) {
      settle_record(pok, p0, p1, p2);
      s_gid[buf ^ 1][pf] = pgid;
      s_r0[buf ^ 1][pf] = scaled_r0(p0);
      s_r1[buf ^ 1][pf] = scaled_r1(p1);
      s_r2[buf ^ 1][pf] = p2;
    }
    lds_barrier();  // products consumed, next records visible
    if (!more) break;
    b1 = nb1;
    b0 = nb0;
    nb1 = mb1;
    nb0 = mb0;
    buf ^= 1;
  }
}

// Which columns of the adjoint rows a pass writes beyond its own: the first
// pass of a call links the rows and writes zeros where no pass writes.
struct PassFlags {
  int first, zero_geo, zero_feat;
};

template <int CP, bool GEO, bool L1>
static void launch_bwd_t(const DevSettings& st, const DevGaussians& g, const Layout& L,
                         const WsView& w, int c0, const float* g_rgb, const float* g_depth,
                         const float* g_alpha, const float* g_feat, float* d_feat,
                         const L1Upstream& l1, const PassFlags& pf, hipStream_t s) {
  const int grid = (int)L.ntiles * kMaxSeg;  // work items beyond the filed ones return
  hipLaunchKernelGGL((k_composite_bwd<CP, GEO, L1>), dim3(grid), dim3(kBlock), 0, s, st, g.P,
                     g.C, c0, L.W, L.H, L.tiles_x, L.ntiles, L.rank_bits, (uint32_t)L.max_pairs,
                     w, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf.first, pf.zero_geo,
                     pf.zero_feat);
}

template <bool GEO, bool L1>
static void launch_bwd_dispatch(int cn, const DevSettings& st, const DevGaussians& g,
                                const Layout& L, const WsView& w, int c0, const float* g_rgb,
                                const float* g_depth, const float* g_alpha, const float* g_feat,
                                float* d_feat, const L1Upstream& l1, const PassFlags& pf,
                                hipStream_t s) {
  if (cn <= 0) {
    if constexpr (GEO)
      launch_bwd_t<0, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf,
                               s);
  } else if (cn <= 8) {
    launch_bwd_t<8, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf, s);
  } else if (cn <= 16) {
    launch_bwd_t<16, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf,
                              s);
  } else if (cn <= 32) {
    launch_bwd_t<32, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf,
                              s);
  } else {
    if constexpr (!GEO)
      launch_bwd_t<64, GEO, L1>(st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat, d_feat, l1, pf,
                                s);
  }
}

// l1 == nullptr: explicit upstream gradients; otherwise the L1 upstream is
// formed inside the kernel (feature group on iff l1->t_feat is set).
// Channel passes: the geometry pass carries up to kBwdGeoChannels feature
// channels, every further pass up to kBwdMaxChannels; each pass recomputes
// the blending weights.
hipError_t launch_composite_bwd_impl(const DevGaussians& g, const DevSettings& st,
                                     const Layout& L, const WsView& w, const float* g_rgb,
                                     const float* g_depth, const float* g_alpha,
                                     const float* g_feat, bool geometry, float* d_feat,
                                     int32_t accumulate, const L1Upstream* l1, hipStream_t s) {
  const bool has_gf = l1 ? (l1->t_feat != nullptr && l1->out_feat != nullptr) : g_feat != nullptr;
  const bool feat_on = st.render_features && g.C > 0 && has_gf && d_feat != nullptr;
  // grad2d is zero here: the forward preprocess clears it and the preprocess
  // adjoint clears it again after consuming it
  if (d_feat && !accumulate && L.P > 0 && g.C > 0 && !l1) {  // the L1 code pass clears it
    const int64_t n = L.P * g.C;
    hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       d_feat, n);
  }
  if (L.P == 0 && !l1) return hipGetLastError();
  if (st.deterministic && L.P > 0)
    hipLaunchKernelGGL(k_fill_slots, dim3(1024), dim3(256), 0, s, w, (int)L.pose_blocks);
  L1Upstream none{};
  const L1Upstream& u = l1 ? *l1 : none;
  const int C = feat_on ? g.C : 0;
  int c0 = 0;
  bool geo = geometry;
  bool first = true;
  while (geo || c0 < C) {
    const int cn = min(geo ? kBwdGeoChannels : kBwdMaxChannels, C - c0);
    // rows hold 10 + g.C columns; the first pass zeroes the ones no pass writes
    const PassFlags pf{first ? 1 : 0, (first && !geometry) ? 1 : 0,
                       (first && C == 0 && g.C > 0) ? 1 : 0};
    if (geo) {
      if (l1)
        launch_bwd_dispatch<true, true>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                        d_feat, u, pf, s);
      else
        launch_bwd_dispatch<true, false>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                         d_feat, u, pf, s);
    } else {
      if (l1)
        launch_bwd_dispatch<false, true>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                         d_feat, u, pf, s);
      else
        launch_bwd_dispatch<false, false>(cn, st, g, L, w, c0, g_rgb, g_depth, g_alpha, g_feat,
                                          d_feat, u, pf, s);
    }
    c0 += cn;
    geo = false;
    first = false;
  }
  return hipGetLastError();
}

hipError_t launch_composite_bwd(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                const WsView& w, const float* g_rgb, const float* g_depth,
                                const float* g_alpha, const float* g_feat, bool geometry,
                                float* d_feat, int32_t accumulate, hipStream_t s) {
  return launch_composite_bwd_impl(g, st, L, w, g_rgb, g_depth, g_alpha, g_feat, geometry, d_feat,
                                   accumulate, nullptr, s);
}

hipError_t launch_composite_bwd_l1(const DevGaussians& g, const DevSettings& st, const Layout& L,
                                   const WsView& w, const L1Args& a, bool geometry, float* d_feat,
                                   int32_t accumulate, hipStream_t s) {
  const double HW = (double)L.W * L.H;
  L1Upstream u;
  u.out_rgb = a.out_rgb;
  u.out_depth = a.out_depth;
  u.out_alpha = a.out_alpha;
  u.out_feat = a.out_feat;
  u.t_rgb = a.t_rgb;
  u.t_depth = a.t_depth;
  u.t_alpha = a.t_alpha;
  u.t_feat = a.t_feat;
  u.s_rgb = (float)(a.w_rgb / (3.0 * HW));
  u.s_depth = (float)(a.w_depth / HW);
  u.s_alpha = (float)(a.w_alpha / HW);
  u.s_feat = (float)(g.C > 0 ? a.w_feat / ((double)g.C * HW) : 0.0);
  u.loss = a.loss;
  u.mask_v = a.mask_v;
  u.mask_e = a.mask_e;
  // the upstream codes and the loss, once for every channel pass, with the
  // work items and the cleared feature gradient
  const int64_t npx = (int64_t)L.W * L.H;
  const int64_t n_zero = (d_feat && !accumulate && L.P > 0 && g.C > 0) ? L.P * g.C : 0;
  // (at least one code workgroup, for the clearing)
  const int64_t ncode = npx > 0 ? (npx + 255) / 256 : 1;
  hipLaunchKernelGGL(k_l1_codes, dim3((unsigned)(2 + ncode)), dim3(256), 0, s, u,
                     npx, g.C, w.l1_codes, w.loss_part, w, L.ntiles, (uint32_t)L.max_pairs,
                     d_feat, n_zero, accumulate ? nullptr : a.loss,
                     (int)(L.P > 0 ? L.pose_blocks : 0));
  return launch_composite_bwd_impl(g, st, L, w, nullptr, nullptr, nullptr, nullptr, geometry,
                                   d_feat, accumulate, &u, s);
}

// ---------------------------------------------------------------- L1 ------

__device__ __forceinline__ float l1_elem(float x, float y, float scale, float& l) {
  const float d = x - y;
  l += fabsf(d);
  return d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
}

// grad = scale * sign(x - y), loss += scale * sum |x - y|.  VEC: four
// elements per thread per step (16-byte loads and stores) plus a scalar tail;
// grid-stride, one loss atomic per workgroup.
template <bool VEC>
__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ x,
                                                 const float* __restrict__ y, int64_t n,
                                                 float scale, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  __shared__ float s_part[4];
  float l = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t done = 0;
  if (VEC) {
    const int64_t n4 = n / 4;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
    float4* g4 = reinterpret_cast<float4*>(grad);
    for (int64_t i = t0; i < n4; i += stride) {
      const float4 a = x4[i], b = y4[i];
      float4 g;
      g.x = l1_elem(a.x, b.x, scale, l);
      g.y = l1_elem(a.y, b.y, scale, l);
      g.z = l1_elem(a.z, b.z, scale, l);
      g.w = l1_elem(a.w, b.w, scale, l);
      g4[i] = g;
    }
    done = 4 * n4;
  }
  for (int64_t i = done + t0; i < n; i += stride) grad[i] = l1_elem(x[i], y[i], scale, l);
  if (!loss) return;  // uniform
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float t = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
    if (t != 0.f) unsafeAtomicAdd(loss, t * scale);
  }
}

hipError_t launch_l1_grad(const float* x, const float* y, int64_t n, float scale, float* grad,
                          float* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool aligned = (((uintptr_t)x | (uintptr_t)y | (uintptr_t)grad) & 15u) == 0;
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 2048) blocks = 2048;  // grid-stride; bounds the loss atomics
  if (aligned)
    hipLaunchKernelGGL(k_l1_grad<true>, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, scale,
                       grad, loss);
  else
    hipLaunchKernelGGL(k_l1_grad<false>, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, scale,
                       grad, loss);
  return hipGetLastError();
}

}  // namespace gsff
