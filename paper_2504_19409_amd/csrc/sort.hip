// Depth sort, tile binning and per-tile lists (Sec. 3.1: the projected
// Gaussians are sorted by depth and blended front to back, per screen tile).
//
// Order of work:
//   1. LSD radix sort of the P depth keys (float32 bits of camera z, culled
//      Gaussians keyed 0xFFFFFFFF), values = Gaussian ids, stable, so equal
//      keys keep index order: one histogram kernel for all four 8-bit digits,
//      then one single-sweep kernel per digit (in-workgroup stable ranking,
//      decoupled look-back across workgroups); see the depth sort section.
//   2. Binning in depth-rank order (tile grids whose cursors fit in LDS).
//      Ranks are cut into blocks of kBinBlock.  Each wave of 64 ranks builds
//      coverage masks (one 64-bit word per tile column and per tile row) with
//      ballots; a rank covers a tile iff its bit is set in both words, so a
//      block's pair count per tile is a few popcounts.  The counts are
//      scanned along the blocks for every tile and then across tiles, which
//      gives every tile its [start, end) and every block its cursor inside
//      each tile.  The scatter then writes every (rank, tile) pair at cursor +
//      (set bits of the tile's mask below the rank's lane): every tile's list
//      comes out in depth order, the pairs never sorted.
//   3. Other tile grids fall back to emitting (tile << rank_bits | rank) keys
//      in rank order, a stable LSD radix sort on the tile bits, a binary search
//      for the tile ranges and a final rank -> id conversion.
// Either way the pair buffer ends up holding Gaussian ids grouped by tile.
//
// Radix passes of the pair sort: every wave owns a chunk of 64 * IPT consecutive
// keys (1024).
//   hist    : per-chunk digit histogram (LDS atomics) -> hist[digit][chunk]
//   rowscan : one block per digit, exclusive scan along the chunk axis,
//             digit totals -> hist_tot
//   scatter : each wave walks its chunk in order; lanes with equal digits find
//             each other with one ballot per digit bit, take their rank among
//             lower lanes, and write to base + running count (stable).
#include <hip/hip_runtime.h>

#include <atomic>

#include "gsff_internal.h"

namespace gsff {

// Workgroup barrier that orders LDS only: global loads issued before it stay
// in flight (__syncthreads() also waits for every outstanding global access).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive wave scan (wave64) of a 32-bit value.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Exclusive block scan (256 threads).  Returns the exclusive prefix; *total
// receives the block sum.  Uses s_tmp[4].
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* s_tmp,
                                                       uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v, lane);
  if (lane == 63) s_tmp[wv] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t t = s_tmp[k];
    if (k < wv) base += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// ---------------------------------------------------------------- radix ----

template <int IPT>
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ n_dev,
                                                    uint32_t n_static, int shift, int nbits,
                                                    uint32_t* __restrict__ hist, int nchunks,
                                                    uint32_t cap) {
  __shared__ uint32_t s_hist[4][256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int chunk = blockIdx.x * 4 + wv;
  const uint32_t n = min(n_dev ? *n_dev : n_static, cap);  // never past the key buffer
  const uint32_t nbins = 1u << nbits, mask = nbins - 1u;
  for (uint32_t d = lane; d < nbins; d += 64) s_hist[wv][d] = 0u;
  __syncthreads();
  if (chunk < nchunks) {
    const uint64_t base = (uint64_t)chunk * (64 * IPT);
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      const uint64_t idx = base + (uint64_t)it * 64 + lane;
      if (idx < n) atomicAdd(&s_hist[wv][(keys[idx] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  if (chunk < nchunks)
    for (uint32_t d = lane; d < nbins; d += 64) hist[(uint64_t)d * nchunks + chunk] = s_hist[wv][d];
}

__global__ __launch_bounds__(256) void k_radix_rowscan(uint32_t* __restrict__ hist, int nchunks,
                                                       uint32_t* __restrict__ hist_tot) {
  __shared__ uint32_t s_tmp[4];
  const int d = blockIdx.x;
  uint32_t* row = hist + (uint64_t)d * nchunks;
  uint32_t carry = 0;
  for (int b = 0; b < nchunks; b += 256) {
    const int i = b + threadIdx.x;
    const uint32_t v = (i < nchunks) ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, s_tmp, &tot);
    if (i < nchunks) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) hist_tot[d] = carry;
}

template <int IPT, bool HasVals>
__global__ __launch_bounds__(256) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_dev, uint32_t n_static, int shift, int nbits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ hist_tot, int nchunks,
    uint32_t cap, uint32_t* status) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_cnt[4][256];
  __shared__ uint32_t s_tmp[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int chunk = blockIdx.x * 4 + wv;
  const uint32_t n = min(n_dev ? *n_dev : n_static, cap);  // never past either buffer
  const uint32_t nbins = 1u << nbits, mask = nbins - 1u;
  // digit bases: exclusive scan of the digit totals (nbins <= 256)
  {
    const uint32_t v = (threadIdx.x < nbins) ? hist_tot[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, s_tmp, &tot);
    s_base[threadIdx.x] = ex;
  }
  __syncthreads();
  if (chunk >= nchunks) return;  // whole wave; no barrier follows
  for (uint32_t d = lane; d < nbins; d += 64)
    s_cnt[wv][d] = s_base[d] + hist[(uint64_t)d * nchunks + chunk];
  const uint64_t base = (uint64_t)chunk * (64 * IPT);
  uint32_t k[IPT];
  uint32_t v[IPT];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const uint64_t idx = base + (uint64_t)it * 64 + lane;
    k[it] = (idx < n) ? keys_in[idx] : 0u;
    if (HasVals) v[it] = (idx < n) ? vals_in[idx] : 0u;
  }
  const uint64_t lt = lanemask_lt(lane);
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const uint64_t idx = base + (uint64_t)it * 64 + lane;
    const bool valid = idx < n;
    const uint32_t d = (k[it] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t start = s_cnt[wv][d];
    // cap: output capacity, never exceeded
    if (valid && guard(status, GSFF_CHECK_PAIR_DEST, start + rank, cap)) {
      keys_out[start + rank] = k[it];
      if (HasVals) vals_out[start + rank] = v[it];
    }
    // the lowest lane of each digit group advances the running count
    if (valid && (peers & lt) == 0ull) s_cnt[wv][d] = start + (uint32_t)__popcll(peers);
  }
}

// One stable LSD pass over nbits digits at `shift`; chunks of 64 * IPT keys.
template <int IPT>
static hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                             uint32_t* vout, const uint32_t* n_dev, uint32_t n_static,
                             int shift, int nbits, int nchunks, uint32_t cap, const WsView& w,
                             hipStream_t s) {
  const unsigned blocks = (unsigned)((nchunks + 3) / 4);
  hipLaunchKernelGGL(k_radix_hist<IPT>, dim3(blocks), dim3(256), 0, s, kin, n_dev, n_static,
                     shift, nbits, w.hist, nchunks, cap);
  hipLaunchKernelGGL(k_radix_rowscan, dim3(1u << nbits), dim3(256), 0, s, w.hist, nchunks,
                     w.hist_tot);
  if (vin)
    hipLaunchKernelGGL((k_radix_scatter<IPT, true>), dim3(blocks), dim3(256), 0, s, kin, vin,
                       kout, vout, n_dev, n_static, shift, nbits, w.hist, w.hist_tot, nchunks,
                       cap, w.status);
  else
    hipLaunchKernelGGL((k_radix_scatter<IPT, false>), dim3(blocks), dim3(256), 0, s, kin,
                       nullptr, kout, nullptr, n_dev, n_static, shift, nbits, w.hist, w.hist_tot,
                       nchunks, cap, w.status);
  return hipGetLastError();
}

// ------------------------------------------------------- depth sort ----
//
// Single-sweep LSD radix sort of the P depth keys, four passes of 8 bits:
//   k_sort_hist4 : all four digit histograms in one read of the keys, as
//                  kSortHistBlocks per-workgroup partials (nothing to clear
//                  first); it also clears the look-back words.
//   k_sort_pass  : workgroup b ranks the keys of chunk b stably in LDS (one
//                  ballot per digit bit per wave, as the radix scatter),
//                  publishes its digit counts and then finds each digit's
//                  count in chunks 0..b-1 in two levels: the chunks are
//                  grouped kLbGroup at a time; b reads the counts of the
//                  chunks of its own group before it, and the totals of the
//                  earlier groups, to which every chunk adds its counts with
//                  one atomic per digit (the word's top bits count the
//                  chunks that have added).  This is the single-pass prefix
//                  scan of Merrill and Garland (2016) with the serial
//                  look-back chain replaced by a two-level reduction: no
//                  chunk waits for another chunk's prefix, so every chunk
//                  waits about one round trip after its predecessors have
//                  ranked.  Every workgroup publishes before it waits, and
//                  waits a bounded number of polls: a workgroup whose
//                  predecessors have not all published by then (they may not
//                  have been dispatched yet) counts their digits itself from
//                  the pass's input, so every wait ends and the result does
//                  not depend on the order workgroups are dispatched in.
// Chunk word: bit 30 set once published, bits 29-0 the count.
// Group word: bits 29-24 the chunks added, bits 23-0 their count.
constexpr uint32_t kLbAgg = 1u << 30, kLbMask = (1u << 30) - 1u;
constexpr uint32_t kLbArrive = 1u << 24, kLbGroupMask = kLbArrive - 1u;
constexpr int kLbGroup = kSortLbGroup;
static_assert((uint64_t)kLbGroup * 256 * kSortIptMax <= kLbGroupMask && kLbGroup < 64,
              "a group's count and arrivals fit their fields");

// Sum of the words words[k * 256], k in [lo, hi), W at a time, polling the
// first one not yet complete: chunk words (GROUP false) once published,
// group words once all kLbGroup chunks have added.  Stops (stalled = true)
// once polls reaches spin.
template <int W, bool GROUP>
__device__ __forceinline__ uint32_t lb_sum(const uint32_t* words, int lo, int hi, uint32_t spin,
                                           uint32_t& polls, bool& stalled) {
  constexpr uint32_t kDone = GROUP ? (uint32_t)kLbGroup * kLbArrive : kLbAgg;
  uint32_t s = 0;
  int k = lo;
  while (k < hi && !stalled) {
    uint32_t x[W];
#pragma unroll
    for (int j = 0; j < W; ++j)
      x[j] = k + j < hi ? __hip_atomic_load(&words[(int64_t)(k + j) * 256], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : kDone;
    int used = W;  // words consumed before one that is not complete
#pragma unroll
    for (int j = 0; j < W; ++j) {
      if (used == W) {
        const bool done = GROUP ? (x[j] & ~kLbGroupMask) == kDone : (x[j] & kLbAgg) != 0u;
        if (!done) used = j;
        else s += x[j] & (GROUP ? kLbGroupMask : kLbMask);
      }
    }
    k += used;
    if (used < W) {
      if (++polls >= spin) stalled = true;
      else __builtin_amdgcn_s_sleep(1);
    }
  }
  return s;
}

__global__ __launch_bounds__(256) void k_sort_hist4(const uint32_t* __restrict__ keys, uint32_t n,
                                                    WsView w, uint32_t lb_words) {
  __shared__ uint32_t s_h[1024];
  for (int j = threadIdx.x; j < 1024; j += 256) s_h[j] = 0u;
  __syncthreads();
  // 16 keys per thread are loaded before any is counted: one round trip
  // per 16 grid strides instead of one per stride
  constexpr int KB = 16;
  const uint32_t stride = gridDim.x * 256;
  for (uint64_t i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += (uint64_t)KB * stride) {
    uint32_t k[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const uint64_t i = i0 + (uint64_t)j * stride;
      k[j] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (i0 + (uint64_t)j * stride < n) {
#pragma unroll
        for (int p = 0; p < 4; ++p) atomicAdd(&s_h[256 * p + ((k[j] >> (8 * p)) & 255u)], 1u);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < 1024; j += 256) w.sort_part[blockIdx.x * 1024 + j] = s_h[j];
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < lb_words; i += gridDim.x * 256)
    w.sort_lb[i] = 0u;
}

template <int IPT>
__global__ __launch_bounds__(256) void k_sort_pass(const uint32_t* __restrict__ kin,
                                                   const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout,
                                                   uint32_t* __restrict__ vout, uint32_t n,
                                                   int pass, uint32_t spin, WsView w) {
  __shared__ uint32_t s_cnt[4][256];  // per-wave digit counts, then per-wave digit offsets
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_tmp[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int shift = 8 * pass;
  const int nch = (int)gridDim.x, ngr = (nch + kLbGroup - 1) / kLbGroup;
  uint32_t* lb = w.sort_lb + (uint64_t)pass * (uint64_t)(nch + ngr) * 256;  // chunk counts
  uint32_t* glb = lb + (uint64_t)nch * 256;                                  // group totals
  const uint32_t b = blockIdx.x;
  const uint64_t base = (uint64_t)b * (256 * IPT) + (uint64_t)wv * (64 * IPT);
  uint32_t k[IPT], v[IPT], rank[IPT];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const uint64_t idx = base + (uint64_t)it * 64 + lane;
    k[it] = idx < n ? kin[idx] : 0u;
    v[it] = idx < n ? vin[idx] : 0u;
  }
  // this pass's digit totals (thread = digit), from the histogram partials
  uint32_t part[kSortHistBlocks];
#pragma unroll
  for (int g = 0; g < kSortHistBlocks; ++g) part[g] = w.sort_part[g * 1024 + 256 * pass + tid];
#pragma unroll
  for (int k = 0; k < 4; ++k) s_cnt[k][tid] = 0u;
  lds_barrier();  // the zeroed counts; the loads stay in flight
  // stable rank of every key among the wave's keys of its digit
  const uint64_t lt = lanemask_lt(lane);
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const bool valid = base + (uint64_t)it * 64 + lane < n;
    const uint32_t d = (k[it] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const uint32_t start = s_cnt[wv][d];
    rank[it] = start + (uint32_t)__popcll(peers & lt);
    if (valid && (peers & lt) == 0ull) s_cnt[wv][d] = start + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // thread = digit: the chunk's count, published, then the earlier chunks' count
  const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
  const uint32_t cnt = c0 + c1 + c2 + c3;
  const int grp = (int)b / kLbGroup, first = grp * kLbGroup;
  __hip_atomic_store(&lb[b * 256 + tid], kLbAgg | cnt, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(&glb[grp * 256 + tid], kLbArrive | cnt, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  // the digits' first places (independent of the earlier chunks) while the
  // neighbours publish
  uint32_t tot = 0u;
#pragma unroll
  for (int g = 0; g < kSortHistBlocks; ++g) tot += part[g];
  uint32_t all;
  const uint32_t dbase = block_excl_scan256(tot, s_tmp, &all);
  uint32_t polls = 0;
  bool stalled = spin == 0u && b > 0u;  // (a zero limit: every workgroup counts)
  uint32_t excl = lb_sum<kLbGroup, false>(lb + tid, first, (int)b, spin, polls, stalled);
  excl += lb_sum<32, true>(glb + tid, 0, grp, spin, polls, stalled);
  if (__syncthreads_or(stalled ? 1 : 0)) {  // uniform: count chunks 0..b-1 from the input
    s_base[tid] = 0u;
    __syncthreads();
    const uint64_t end = (uint64_t)b * (256 * IPT);  // (those chunks are full)
#pragma unroll 8
    for (uint64_t i = tid; i < end; i += 256) atomicAdd(&s_base[(kin[i] >> shift) & 255u], 1u);
    __syncthreads();
    excl = s_base[tid];
    __syncthreads();
    if (tid == 0) atomicOr(&w.status[0], GSFF_FLAG_SORT_RECOUNT);
  }
  s_base[tid] = dbase + excl;
  s_cnt[0][tid] = 0u;
  s_cnt[1][tid] = c0;
  s_cnt[2][tid] = c0 + c1;
  s_cnt[3][tid] = c0 + c1 + c2;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    if (base + (uint64_t)it * 64 + lane < n) {
      const uint32_t d = (k[it] >> shift) & 255u;
      const uint32_t pos = s_base[d] + s_cnt[wv][d] + rank[it];
      if (guard(w.status, GSFF_CHECK_SORT_DEST, pos, n)) {
        kout[pos] = k[it];
        vout[pos] = v[it];
      }
    }
  }
}

static std::atomic<uint32_t> g_sort_wait_limit{kSortWaitPolls};

void set_sort_wait_limit(uint32_t polls) { g_sort_wait_limit.store(polls); }

hipError_t launch_sort_depth(const Layout& L, const WsView& w, hipStream_t s) {
  if (L.P == 0) return hipSuccess;
  const uint32_t spin = g_sort_wait_limit.load();
  const uint32_t n = (uint32_t)L.P;
  const int64_t groups = (L.sort_blocks + kSortLbGroup - 1) / kSortLbGroup;
  hipLaunchKernelGGL(k_sort_hist4, dim3(kSortHistBlocks), dim3(256), 0, s, w.dkeys_a, n, w,
                     (uint32_t)(4 * 256 * (L.sort_blocks + groups)));
  uint32_t* ka = w.dkeys_a;
  uint32_t* kb = w.dkeys_b;
  uint32_t* va = w.dids_a;
  uint32_t* vb = w.dids_b;
  for (int pass = 0; pass < 4; ++pass) {
    const dim3 grid((unsigned)L.sort_blocks);
    if (L.sort_ipt == 4)
      hipLaunchKernelGGL(k_sort_pass<4>, grid, dim3(256), 0, s, ka, va, kb, vb, n, pass, spin, w);
    else if (L.sort_ipt == 8)
      hipLaunchKernelGGL(k_sort_pass<8>, grid, dim3(256), 0, s, ka, va, kb, vb, n, pass, spin, w);
    else
      hipLaunchKernelGGL(k_sort_pass<kSortIptMax>, grid, dim3(256), 0, s, ka, va, kb, vb, n, pass,
                         spin, w);
    uint32_t* t = ka;
    ka = kb;
    kb = t;
    t = va;
    va = vb;
    vb = t;
  }
  return hipGetLastError();  // four passes: the result is back in dkeys_a / dids_a
}

hipError_t launch_sort_tiles(const Layout& L, const WsView& w, hipStream_t s) {
  if (L.direct_bin || L.P == 0 || L.tile_bits == 0 || L.max_pairs == 0) return hipSuccess;
  const int n1 = (L.tile_bits + 1) / 2, n2 = L.tile_bits - n1;
  hipError_t e = radix_pass<kRadixIpt>(w.pkeys_a, nullptr, w.pkeys_b, nullptr, w.status + 2, 0u,
                            L.rank_bits, n1, (int)L.pair_chunks, (uint32_t)L.max_pairs, w, s);
  if (e != hipSuccess) return e;
  // second pass (possibly 0 bits: a stable copy) brings the keys back to pkeys_a
  return radix_pass<kRadixIpt>(w.pkeys_b, nullptr, w.pkeys_a, nullptr, w.status + 2, 0u,
                    L.rank_bits + n1, n2, (int)L.pair_chunks, (uint32_t)L.max_pairs, w, s);
}

// ------------------------------------------------------------- binning ----

// rectangle of the Gaussian at depth rank r (empty if the stored id is not valid)
__device__ __forceinline__ ushort4 ranked_rect(const WsView& w, int64_t r, int64_t P) {
  const uint32_t gid = w.dids_a[r];
  return guard(w.status, GSFF_CHECK_RANK_ID, gid, (uint32_t)P) ? w.rects[gid]
                                                               : make_ushort4(1, 1, 0, 0);
}

__device__ __forceinline__ uint32_t rect_count(ushort4 r) {
  if (r.x > r.z || r.y > r.w) return 0u;
  return (uint32_t)(r.z - r.x + 1) * (uint32_t)(r.w - r.y + 1);
}

// Binning works on super-tiles of kSuper x kSuper tiles (the bin grid):
// a tile rectangle's range of super-tiles (empty stays empty) ...
__device__ __forceinline__ ushort4 super_rect(ushort4 r) {
  if (r.x > r.z || r.y > r.w) return make_ushort4(1, 1, 0, 0);
  return make_ushort4(r.x / kSuper, r.y / kSuper, r.z / kSuper, r.w / kSuper);
}

// ... and the tiles of super-tile (X, Y) that it covers: bit 4 (ty % 4) + (tx % 4)
__device__ __forceinline__ uint32_t super_mask(ushort4 r, uint32_t X, uint32_t Y) {
  const int xa = max((int)r.x - (int)(kSuper * X), 0), xb = min((int)r.z - (int)(kSuper * X), 3);
  const int ya = max((int)r.y - (int)(kSuper * Y), 0), yb = min((int)r.w - (int)(kSuper * Y), 3);
  if (xa > xb || ya > yb) return 0u;
  const uint32_t cols = ((2u << xb) - 1u) & ~((1u << xa) - 1u);
  uint32_t m = 0;
#pragma unroll
  for (int y = 0; y < 4; ++y) m |= (y >= ya && y <= yb) ? cols << (4 * y) : 0u;
  return m;
}

// per-block sums of tile counts, ranks in depth order
__global__ __launch_bounds__(256) void k_count_reduce(WsView w, int64_t P) {
  __shared__ uint32_t s_tmp[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanBlock / 256; ++k) {
    const int64_t r = base + k * 256 + threadIdx.x;
    if (r < P) sum += rect_count(super_rect(ranked_rect(w, r, P)));
  }
  uint32_t tot;
  block_excl_scan256(sum, s_tmp, &tot);
  if (threadIdx.x == 0) w.scan_part[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums; pair count and overflow flag
__global__ __launch_bounds__(1024) void k_count_top(WsView w, int nblocks, uint64_t max_pairs) {
  __shared__ uint64_t s_w[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t carry = 0;
  for (int b = 0; b < nblocks; b += 1024) {
    const int i = b + threadIdx.x;
    uint64_t v = (i < nblocks) ? (uint64_t)w.scan_part[i] : 0ull;
    uint64_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t t = __shfl_up(inc, off, 64);
      if (lane >= off) inc += t;
    }
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) pre += s_w[k];
      tot += s_w[k];
    }
    __syncthreads();
    if (i < nblocks) w.scan_part[i] = (uint32_t)(carry + pre + inc - v);
    carry += tot;
  }
  if (threadIdx.x == 0) {
    const bool over = carry > max_pairs;
    if (over) atomicOr(&w.status[0], GSFF_FLAG_PAIR_OVERFLOW);
    w.status[1] = (uint32_t)(carry > 0xFFFFFFFFull ? 0xFFFFFFFFull : carry);
    w.status[2] = over ? 0u : (uint32_t)carry;  // pairs the later stages use
  }
}

// Offsets and pair emission: key = (super-tile << rank_bits) | rank.  After the
// block scan every lane holds the offset, count and rectangle of its own rank;
// each wave then walks its 64 ranks in order, broadcasting one rank's values
// with readlane, and all lanes write consecutive keys of that rank's run.
__global__ __launch_bounds__(256) void k_emit(WsView w, int64_t P, int tiles_x, int rank_bits,
                                              uint32_t max_pairs) {
  __shared__ uint32_t s_tmp[4];
  const bool ok = (w.status[2] != 0u || w.status[1] == 0u) && w.status[2] <= max_pairs;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  const int lane = threadIdx.x & 63;
  uint32_t carry = w.scan_part[blockIdx.x];
  for (int k = 0; k < kScanBlock / 256; ++k) {
    const int64_t r = base + k * 256 + threadIdx.x;
    ushort4 rc = make_ushort4(1, 1, 0, 0);
    if (r < P) rc = super_rect(ranked_rect(w, r, P));
    const uint32_t cnt = rect_count(rc);
    uint32_t tot;
    const uint32_t off = carry + block_excl_scan256(cnt, s_tmp, &tot);
    carry += tot;
    if (r < P) w.offsets[r] = off;
    if (!ok) continue;
    const uint32_t x0 = rc.x, y0 = rc.y, wd = (uint32_t)(rc.z - rc.x) + 1u;
    const uint32_t rank0 = (uint32_t)(r - lane);
    for (int src = 0; src < 64; ++src) {
      const uint32_t n = __builtin_amdgcn_readlane(cnt, src);
      if (n == 0u) continue;  // uniform
      const uint32_t o = __builtin_amdgcn_readlane(off, src);
      const uint32_t bx = __builtin_amdgcn_readlane(x0, src);
      const uint32_t by = __builtin_amdgcn_readlane(y0, src);
      const uint32_t bw = __builtin_amdgcn_readlane(wd, src);
      const uint32_t rk = rank0 + (uint32_t)src;
      for (uint32_t j = lane; j < n; j += 64) {
        const uint32_t ty = by + j / bw, tx = bx + j % bw;
        if (GSFF_CHECK(w.status, GSFF_CHECK_PAIR_DEST, o + j, w.status[2]))
          w.pkeys_a[o + j] = ((ty * (uint32_t)tiles_x + tx) << rank_bits) | rk;
      }
    }
  }
}

// ------------------------------------------------------ direct binning ----

// Coverage masks of the 64 consecutive depth ranks held by a wave's lanes:
// bit L of col[x] is set when lane L's rectangle spans tile column x, bit L of
// row[y] when it spans tile row y.  A rectangle is the product of its column
// and row ranges, so lane L covers tile (x, y) exactly when bit L is set in
// col[x] & row[y]: the wave's pair count on a tile is the popcount of that
// word, and a pair's place among the wave's pairs of its tile (rank order) is
// the popcount of the bits below its lane.  One ballot per tile column / row.
__device__ __forceinline__ void wave_cover_masks(ushort4 rc, int tiles_x, int tiles_y,
                                                 uint64_t* __restrict__ col,
                                                 uint64_t* __restrict__ row) {
  const int lane = threadIdx.x & 63;
  const uint32_t x0 = rc.x, x1 = rc.z, y0 = rc.y, y1 = rc.w;
  for (int b = 0; b < tiles_x; b += 64) {
    uint64_t mine = 0;
    const int nb = tiles_x - b < 64 ? tiles_x - b : 64;
    for (int k = 0; k < nb; ++k) {
      const uint32_t x = (uint32_t)(b + k);
      const uint64_t m = __ballot(x0 <= x && x <= x1);
      mine = lane == k ? m : mine;
    }
    if (lane < nb) col[b + lane] = mine;
  }
  for (int b = 0; b < tiles_y; b += 64) {
    uint64_t mine = 0;
    const int nb = tiles_y - b < 64 ? tiles_y - b : 64;
    for (int k = 0; k < nb; ++k) {
      const uint32_t y = (uint32_t)(b + k);
      const uint64_t m = __ballot(y0 <= y && y <= y1);
      mine = lane == k ? m : mine;
    }
    if (lane < nb) row[b + lane] = mine;
  }
}

// rectangle of the Gaussian at depth rank r, and its id (empty past the end)
__device__ __forceinline__ ushort4 rank_rect(const WsView& w, int64_t r, int64_t P,
                                             uint32_t* gid) {
  ushort4 rc = make_ushort4(1, 1, 0, 0);
  *gid = 0u;
  if (r < P) {
    *gid = w.dids_a[r];
    if (guard(w.status, GSFF_CHECK_RANK_ID, *gid, (uint32_t)P)) rc = w.rects[*gid];
  }
  return rc;
}

__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Per-block, per-super-tile pair counts -> binhist[cell][block], from the
// masks; the kernels below take the bin grid (cells = super-tiles) as
// tiles_x x tiles_y / ntiles.
__global__ __launch_bounds__(256) void k_bin_hist(WsView w, int64_t P, int ntiles, int tiles_x,
                                                  int tiles_y, int nblk) {
  extern __shared__ uint64_t s_m[];  // [4][tiles_x + tiles_y]
  const int wv = threadIdx.x >> 6, TM = tiles_x + tiles_y;
  uint32_t gid;
  const ushort4 rc =
      super_rect(rank_rect(w, (int64_t)blockIdx.x * kBinBlock + threadIdx.x, P, &gid));
  wave_cover_masks(rc, tiles_x, tiles_y, s_m + wv * TM, s_m + wv * TM + tiles_x);
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += 256) {
    const int y = t / tiles_x, x = t - y * tiles_x;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c += __popcll(s_m[k * TM + x] & s_m[k * TM + tiles_x + y]);
    w.binhist[(int64_t)t * nblk + blockIdx.x] = c;
  }
}

// One wave per tile: exclusive scan of its counts along the blocks, written
// block-major to curbase[block][tile] so each scatter block reads its row
// contiguously; tile totals.
__global__ __launch_bounds__(256) void k_bin_colscan(WsView w, int ntiles, int nblk) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;  // whole wave
  const uint32_t* col = w.binhist + (int64_t)t * nblk;
  constexpr int G = 16;  // 64-block rows loaded together before they are scanned
  uint32_t carry = 0;
  for (int g0 = 0; g0 < nblk; g0 += 64 * G) {
    uint32_t v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int b = g0 + 64 * k + lane;
      v[k] = b < nblk ? col[b] : 0u;
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int b = g0 + 64 * k + lane;
      const uint32_t inc = wave_incl_scan(v[k], lane);
      if (b < nblk) w.curbase[(int64_t)b * ntiles + t] = carry + inc - v[k];
      carry += __shfl(inc, 63, 64);
    }
  }
  if (lane == 0) w.tile_tot[t] = carry;
}

// Stable scatter of Gaussian ids into their tiles' segments.  Every
// workgroup first scans the tile totals itself (a few hundred words) for the
// tiles' first pairs; workgroup (0, 0) also writes the tile ranges, the pair
// count and the overflow flag (an overflowing frame renders empty: every
// range collapses and nothing is written).  Wave wv owns the block's ranks
// [64 wv, 64 wv + 64); its cursors start after the pairs of lower waves, and
// every pair's place follows from the coverage masks, so each lane walks its
// own rectangle with no ordering between lanes.  The rank chunk's tile rows
// are split into gridDim.y bands, one workgroup each: the nearest chunks hold
// the largest rectangles, and a band is a fraction of their walk.
__global__ __launch_bounds__(256) void k_bin_scatter(WsView w, int64_t P, int ntiles,
                                                     int tiles_x, int tiles_y, int nblk,
                                                     uint32_t max_pairs) {
  // [4][tiles_x + tiles_y] masks, then [4][band tiles] cursors, then [ntiles] starts
  extern __shared__ uint64_t s_m[];
  __shared__ uint64_t s_wsum[4];
  const int wv = threadIdx.x >> 6, TM = tiles_x + tiles_y, lane = threadIdx.x & 63;
  const int nband = (int)gridDim.y;
  const int band_rows = (tiles_y + nband - 1) / nband;
  uint32_t* s_c = reinterpret_cast<uint32_t*>(s_m + 4 * TM);
  uint32_t* s_st = s_c + 4 * band_rows * tiles_x;
  // the tiles' first pairs: an exclusive scan of the tile totals
  uint64_t carry = 0;
  for (int b0 = 0; b0 < ntiles; b0 += 256) {
    const int i = b0 + (int)threadIdx.x;
    const uint64_t v = i < ntiles ? (uint64_t)w.tile_tot[i] : 0ull;
    uint64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t t = __shfl_up(inc, off, 64);
      if (lane >= off) inc += t;
    }
    if (lane == 63) s_wsum[wv] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < wv) pre += s_wsum[k];
      tot += s_wsum[k];
    }
    __syncthreads();
    if (i < ntiles) s_st[i] = (uint32_t)(carry + pre + inc - v);
    carry += tot;
  }
  __syncthreads();
  const bool over = carry > (uint64_t)max_pairs;
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    for (int i = threadIdx.x; i < ntiles; i += 256)
      w.tile_ranges[i] = over ? make_uint2(0u, 0u) : make_uint2(s_st[i], s_st[i] + w.tile_tot[i]);
    if (threadIdx.x == 0) {
      if (over) atomicOr(&w.status[0], GSFF_FLAG_PAIR_OVERFLOW);
      w.status[1] = (uint32_t)(carry > 0xFFFFFFFFull ? 0xFFFFFFFFull : carry);
      w.status[2] = over ? 0u : (uint32_t)carry;
    }
  }
  if (carry == 0 || over) return;  // nothing to write, or overflow (uniform)
  const int y_lo = (int)blockIdx.y * tiles_y / nband, y_hi = ((int)blockIdx.y + 1) * tiles_y / nband;
  const int t_lo = y_lo * tiles_x, nbt = (y_hi - y_lo) * tiles_x;
  if (nbt == 0) return;  // uniform
  uint32_t gid;
  const ushort4 trc = rank_rect(w, (int64_t)blockIdx.x * kBinBlock + threadIdx.x, P, &gid);
  const ushort4 rc = super_rect(trc);
  const uint64_t* col = s_m + wv * TM;
  const uint64_t* row = col + tiles_x;
  wave_cover_masks(rc, tiles_x, tiles_y, s_m + wv * TM, s_m + wv * TM + tiles_x);
  __syncthreads();
  for (int b = threadIdx.x; b < nbt; b += 256) {
    const int t = t_lo + b;
    const int y = t / tiles_x, x = t - y * tiles_x;
    uint32_t cur = s_st[t] + w.curbase[(int64_t)blockIdx.x * ntiles + t];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_c[k * nbt + b] = cur;
      cur += __popcll(s_m[k * TM + x] & s_m[k * TM + tiles_x + y]);
    }
  }
  __syncthreads();
  // this lane's rectangle, rows clipped to the band
  const uint32_t ya = max((uint32_t)rc.y, (uint32_t)y_lo), yb = min((uint32_t)rc.w, (uint32_t)(y_hi - 1));
  if (rc.x > rc.z || ya > yb) return;
  const uint32_t cnt = (uint32_t)(rc.z - rc.x + 1) * (yb - ya + 1);
  const uint32_t* cw = s_c + wv * nbt - t_lo;
  const uint32_t x0 = rc.x, x1 = rc.z;
  uint32_t x = x0, y = ya;
  uint64_t rm = row[y];
  for (uint32_t j = 0; j < cnt; ++j) {
    const uint32_t t = y * (uint32_t)tiles_x + x;
    const uint32_t pos = cw[t] + bits_below_lane(col[x] & rm);
    // (carry <= max_pairs here: the frame did not overflow)
    if (guard(w.status, GSFF_CHECK_PAIR_DEST, pos, (uint32_t)carry)) {
      w.pkeys_a[pos] = gid;
      w.pmask[pos] = (uint16_t)super_mask(trc, x, y);
    }
    const bool wrap = x == x1;
    x = wrap ? x0 : x + 1u;
    y = wrap && y < yb ? y + 1u : y;
    rm = row[y];
  }
}

// fallback path: sorted (super-tile | rank) keys -> Gaussian ids and tile
// masks, after the ranges
__global__ __launch_bounds__(256) void k_keys_to_ids(WsView w, uint32_t rmask, int rank_bits,
                                                     int64_t P, int super_x, uint32_t max_pairs) {
  const uint32_t n = min(w.status[2], max_pairs);
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint32_t key = w.pkeys_a[i];
    const uint32_t r = key & rmask;
    const uint32_t cell = rank_bits >= 32 ? 0u : key >> rank_bits;
    const uint32_t gid =
        guard(w.status, GSFF_CHECK_RANK_ID, r, (uint32_t)P) ? w.dids_a[r] : (uint32_t)P;
    uint32_t m = 0u;
    if (guard(w.status, GSFF_CHECK_RANK_ID, gid, (uint32_t)P))
      m = super_mask(w.rects[gid], cell % (uint32_t)super_x, cell / (uint32_t)super_x);
    w.pkeys_a[i] = gid;
    w.pmask[i] = (uint16_t)m;
  }
}

hipError_t launch_bin(const Layout& L, const WsView& w, hipStream_t s) {
  if (L.P == 0) {
    return hipSuccess;  // status was zeroed by the preprocess kernel
  }
  if (L.direct_bin) {
    // the bin grid is the super-tile grid; scatter bands split its rows over
    // kBinBands workgroups per rank chunk
    const int nband = L.super_y < kBinBands ? L.super_y : kBinBands;
    const int band_rows = (L.super_y + nband - 1) / nband;
    const size_t lds_m = 32ull * (L.super_x + L.super_y);
    const size_t lds_c = lds_m + 16ull * band_rows * L.super_x + 4ull * L.nsuper;
    hipLaunchKernelGGL(k_bin_hist, dim3((unsigned)L.bin_blocks), dim3(256), lds_m, s, w, L.P,
                       L.nsuper, L.super_x, L.super_y, (int)L.bin_blocks);
    hipLaunchKernelGGL(k_bin_colscan, dim3((unsigned)((L.nsuper + 3) / 4)), dim3(256), 0, s, w,
                       L.nsuper, (int)L.bin_blocks);
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)L.bin_blocks, (unsigned)nband), dim3(256),
                       lds_c, s, w, L.P, L.nsuper, L.super_x, L.super_y, (int)L.bin_blocks,
                       (uint32_t)L.max_pairs);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_count_reduce, dim3((unsigned)L.scan_blocks), dim3(256), 0, s, w, L.P);
  hipLaunchKernelGGL(k_count_top, dim3(1), dim3(1024), 0, s, w, (int)L.scan_blocks,
                     (uint64_t)L.max_pairs);
  hipLaunchKernelGGL(k_emit, dim3((unsigned)L.scan_blocks), dim3(256), 0, s, w, L.P, L.super_x,
                     L.rank_bits, (uint32_t)L.max_pairs);
  return hipGetLastError();
}

// ------------------------------------------------------------- ranges -----

__device__ __forceinline__ uint32_t lower_bound_u64(const uint32_t* a, uint32_t n, uint64_t key) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_tile_ranges(WsView w, int ntiles, int rank_bits,
                                                     uint32_t max_pairs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const uint32_t n = min(w.status[2], max_pairs);
  const uint32_t a = lower_bound_u64(w.pkeys_a, n, (uint64_t)t << rank_bits);
  const uint32_t b = lower_bound_u64(w.pkeys_a, n, (uint64_t)(t + 1) << rank_bits);
  w.tile_ranges[t] = make_uint2(a, b);
}

hipError_t launch_tile_ranges(const Layout& L, const WsView& w, hipStream_t s) {
  if (L.direct_bin && L.P > 0) return hipSuccess;  // ranges came with the binning
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((L.nsuper + 255) / 256)), dim3(256), 0, s, w,
                     L.nsuper, L.rank_bits, (uint32_t)L.max_pairs);
  if (L.P > 0 && L.max_pairs > 0) {
    const uint32_t rmask = (L.rank_bits >= 32) ? 0xFFFFFFFFu : ((1u << L.rank_bits) - 1u);
    int64_t blocks = (L.max_pairs + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_keys_to_ids, dim3((unsigned)blocks), dim3(256), 0, s, w, rmask,
                       L.rank_bits, L.P, L.super_x, (uint32_t)L.max_pairs);
  }
  return hipGetLastError();
}

}  // namespace gsff
