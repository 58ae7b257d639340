// Tile binning: stable LSD radix sort of the key words on their tile id,
// carrying the emission index and the record id, with the key count read
// from device memory (so the host never synchronises), and the per-tile
// [start, end) ranges.  Digits are at most 8 bits (256 per pass), or, for
// small inputs whose tile id has at most 10 bits, the whole tile id in one
// pass (up to 1024 digits).
#include "ug_kernels.h"

namespace ug {

constexpr int kSortThreads = 256;
constexpr uint32_t kSortMaxBlocks = 2048;
constexpr uint32_t kWideMaxBlocks = 256;  // one wide pass only up to this many blocks

// Contiguous chunk of the n keys owned by block b of G (multiple of 256).
__device__ __forceinline__ void sort_chunk(uint32_t n, uint32_t G, uint32_t b, uint32_t& s, uint32_t& e) {
  uint64_t C = ((uint64_t)n + G - 1) / G;
  C = (C + 255) & ~(uint64_t)255;
  const uint64_t s64 = (uint64_t)b * C;
  s = (uint32_t)(s64 < n ? s64 : n);
  const uint64_t e64 = s64 + C;
  e = (uint32_t)(e64 < n ? e64 : n);
}

// Per-block digit histogram, block-major: cnt[b * D + d] (D digit slots).
template <int D>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const Ctrl* __restrict__ ctrl,
                                                              const uint32_t* __restrict__ keys, uint32_t G,
                                                              int shift, uint32_t dmask, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[4][D];
  for (int j = threadIdx.x; j < 4 * D; j += kSortThreads) (&h[0][0])[j] = 0u;
  __syncthreads();
  uint32_t s, e;
  sort_chunk(ctrl->n_key_eff, G, blockIdx.x, s, e);
  const int wave = threadIdx.x >> 6;
  // eight loads in flight per thread, then their counts
  for (uint32_t i0 = s + threadIdx.x; i0 < e; i0 += 8 * kSortThreads) {
    uint32_t kv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t i = i0 + (uint32_t)(j * kSortThreads);
      kv[j] = i < e ? keys[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (i0 + (uint32_t)(j * kSortThreads) < e) atomicAdd(&h[wave][(kv[j] >> shift) & dmask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < D; d += kSortThreads)
    cnt[(size_t)blockIdx.x * D + d] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// One block per digit d: exclusive scan of column d over the G blocks
// (in place), and the column total coltot[d].  G <= 4096.
constexpr int kColPer = 16;
template <int D>
__global__ __launch_bounds__(256) void k_radix_colscan(uint32_t* __restrict__ cnt, uint32_t G,
                                                       uint32_t* __restrict__ coltot) {
  __shared__ uint32_t sh[4];
  const uint32_t d = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  uint32_t v[kColPer];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kColPer; ++j) {
    const uint32_t b = kColPer * t + j;
    v[j] = b < G ? cnt[(size_t)b * D + d] : 0u;
    sum += v[j];
  }
  uint32_t x = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += sh[w];
    total += sh[w];
  }
  uint32_t run = before + x - sum;
#pragma unroll
  for (int j = 0; j < kColPer; ++j) {
    const uint32_t b = kColPer * t + j;
    if (b < G) cnt[(size_t)b * D + d] = run;
    run += v[j];
  }
  if (t == 0) coltot[d] = total;
}

// Stable scatter.  The block's chunk is walked in rounds of up to 4096 keys;
// in a round wave w owns the w-th quarter of the round's keys (rounded up to
// whole loads of 64), loaded 64 at a time.  Each wave ranks its keys on its own: lanes holding
// the same digit are found with one ballot per digit bit, and a per-wave digit counter
// in LDS orders the wave's loads.  One block step then orders the waves and
// the digits, the round is reordered by digit in LDS and written out as
// contiguous runs per digit, so the global writes coalesce.
// kItems keys per thread and round: 8 for small inputs (more blocks, less
// LDS), 16 when every block walks several rounds.

// Every key carries two payload words (emission index, record id).  They
// are loaded with the keys (coalesced, in flight during the ranking) and
// follow them through the same LDS slots one word at a time: the keys are
// reordered and written, then the emission indices, then the record ids.
struct SortSet {
  uint32_t* key;
  uint32_t* val;  // emission index; generated (= position) in the first pass
  uint32_t* rec;
};

template <int kItems, int D>
__device__ __forceinline__ void radix_scatter(const Ctrl* __restrict__ ctrl, SortSet in,
                                                                SortSet out, bool gen_val,
                                                                const uint32_t* __restrict__ cnt,
                                                                const uint32_t* __restrict__ coltot, uint32_t G,
                                                                int shift, int dbits, uint32_t* __restrict__ tile_start,
                                                                uint32_t T) {
  constexpr int kRound = kSortThreads * kItems;
  const uint32_t* __restrict__ kin = in.key;
  __shared__ uint32_t s_key[kRound];  // the round reordered by digit: keys, then each payload word
  constexpr int kPer = D / kSortThreads;  // digits per thread, consecutive
  __shared__ uint32_t run[D];      // global output position of the next key of each digit
  __shared__ uint32_t loc[D];      // first LDS slot of each digit in this round
  __shared__ uint32_t rcnt[D];     // keys of each digit in this round
  __shared__ uint32_t wcnt[4][D];  // per-wave digit counts, then the waves' prefixes
  __shared__ uint32_t sh[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t dmask = (1u << dbits) - 1u;
  uint32_t s, e;
  sort_chunk(ctrl->n_key_eff, G, blockIdx.x, s, e);
  {
    uint32_t tot[kPer], sum = 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      tot[k] = coltot[tid * kPer + k];
      sum += tot[k];
    }
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += sh[w];
    uint32_t at = before + x - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = tid * kPer + k;
      // one pass over the whole tile id: a digit's first output position is
      // its tile's start
      if (tile_start && blockIdx.x == 0 && (uint32_t)d < T) tile_start[d] = at;
      run[d] = at + cnt[(size_t)blockIdx.x * D + d];
      at += tot[k];
    }
    if (tile_start && blockIdx.x == 0 && tid == 0) tile_start[T] = ctrl->n_key_eff;
  }
  for (uint32_t base = s; base < e; base += kRound) {
    // ---- per wave: ranks of its 512 keys among its own keys of each digit
#pragma unroll
    for (int j = 0; j < D / 64; ++j) wcnt[wave][lane + 64 * j] = 0u;
    wave_lds_sync();
    // the round's keys split evenly over the waves, in whole loads of 64
    const uint32_t n_round = min((uint32_t)kRound, e - base);
    const uint32_t seg = ((n_round + 255u) / 256u) * 64u;
    uint32_t kk[kItems], rr[kItems], vv[kItems], rc[kItems];
    // all of the round's loads first: the ranking's wave fences would
    // otherwise keep each load behind the previous key's LDS update
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const uint32_t i = base + (uint32_t)wave * seg + (uint32_t)(it * 64 + lane);
      const bool valid = (uint32_t)(it * 64) < seg && i < e;
      kk[it] = valid ? kin[i] : 0u;
      vv[it] = gen_val ? i : (valid ? in.val[i] : 0u);
      rc[it] = valid ? in.rec[i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const uint32_t i = base + (uint32_t)wave * seg + (uint32_t)(it * 64 + lane);
      const bool valid = (uint32_t)(it * 64) < seg && i < e;
      const uint32_t k = kk[it];
      const uint32_t d = (k >> shift) & dmask;
      unsigned long long peers = __ballot(valid);
      for (int bit = 0; bit < dbits; ++bit) {
        const bool on = (d >> bit) & 1u;
        const unsigned long long bm = __ballot(on);
        peers &= on ? bm : ~bm;
      }
      const uint32_t before = valid ? wcnt[wave][d] : 0u;
      wave_lds_sync();
      if (valid && lanemask_lt_popc(peers) == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
      wave_lds_sync();
      rr[it] = valid ? before + lanemask_lt_popc(peers) : 0xffffffffu;
    }
    __syncthreads();
    // ---- per digit: the waves' prefixes and the round's count
    {
      uint32_t c[kPer], sum = 0u;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int d = tid * kPer + k;
        const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
        wcnt[0][d] = 0u;
        wcnt[1][d] = c0;
        wcnt[2][d] = c0 + c1;
        wcnt[3][d] = c0 + c1 + c2;
        c[k] = c0 + c1 + c2 + c3;
        rcnt[d] = c[k];
        sum += c[k];
      }
      uint32_t x = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane == 63) sh[wave] = x;
      __syncthreads();
      uint32_t before = 0;
      for (int w = 0; w < wave; ++w) before += sh[w];
      uint32_t at = before + x - sum;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        loc[tid * kPer + k] = at;
        at += c[k];
      }
    }
    __syncthreads();
    // slot of each of the thread's keys in the reordered round
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      if (rr[it] != 0xffffffffu) {
        const uint32_t d = (kk[it] >> shift) & dmask;
        rr[it] += loc[d] + wcnt[wave][d];
        s_key[rr[it]] = kk[it];
      }
    }
    __syncthreads();
    // keys out, as contiguous runs per digit; each slot's output position is
    // kept for the payload words
    uint32_t opos[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t i = (uint32_t)tid + (uint32_t)(j * kSortThreads);
      opos[j] = 0xffffffffu;
      if (i < n_round) {
        const uint32_t k = s_key[i];
        const uint32_t d = (k >> shift) & dmask;
        opos[j] = run[d] + (i - loc[d]);
        out.key[opos[j]] = k;
      }
    }
    // the two payload words through the same slots
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kItems; ++it)
        if (rr[it] != 0xffffffffu) s_key[rr[it]] = w == 0 ? vv[it] : rc[it];
      __syncthreads();
      uint32_t* __restrict__ dst = w == 0 ? out.val : out.rec;
#pragma unroll
      for (int j = 0; j < kItems; ++j)
        if (opos[j] != 0xffffffffu) dst[opos[j]] = s_key[(uint32_t)tid + (uint32_t)(j * kSortThreads)];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) run[tid * kPer + k] += rcnt[tid * kPer + k];
    __syncthreads();
  }
}

// Kernels around the scatter body.  The large-input variant (16 keys per
// thread and round, 256 digits) is held to four workgroups per CU, which its
// LDS allows; the compiler would otherwise give it more registers and three.
template <int kItems, int D>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const Ctrl* __restrict__ ctrl, SortSet in,
                                                                SortSet out, bool gen_val,
                                                                const uint32_t* __restrict__ cnt,
                                                                const uint32_t* __restrict__ coltot, uint32_t G,
                                                                int shift, int dbits, uint32_t* __restrict__ tile_start,
                                                                uint32_t T) {
  radix_scatter<kItems, D>(ctrl, in, out, gen_val, cnt, coltot, G, shift, dbits, tile_start, T);
}

__global__ __launch_bounds__(kSortThreads, 4) void k_radix_scatter_large(
    const Ctrl* __restrict__ ctrl, SortSet in, SortSet out, bool gen_val, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ coltot, uint32_t G, int shift, int dbits, uint32_t* __restrict__ tile_start,
    uint32_t T) {
  radix_scatter<16, 256>(ctrl, in, out, gen_val, cnt, coltot, G, shift, dbits, tile_start, T);
}

// tile_start[t] = first sorted key index whose tile id is >= t (t in [0, T]).
// Eight consecutive keys per thread (two 16-byte loads; the grid covers the
// key capacity); the key before a thread's first comes from its neighbour
// lane.  Each key writes the starts of the tiles after the previous key's
// tile up to its own.
constexpr uint32_t kRangeKeys = 8;
__global__ __launch_bounds__(256) void k_tile_ranges(const Ctrl* __restrict__ ctrl,
                                                     const uint32_t* __restrict__ skeys, uint32_t T, uint32_t tmask,
                                                     uint32_t* __restrict__ tile_start) {
  const uint32_t n = ctrl->n_key_eff;
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) {
    for (uint32_t t = g; t <= T; t += gridDim.x * blockDim.x) tile_start[t] = 0u;
    return;
  }
  const uint32_t i0 = g * kRangeKeys;
  uint32_t k[kRangeKeys];
  if (i0 + kRangeKeys <= n) {
    const uint4* p = reinterpret_cast<const uint4*>(skeys + i0);  // i0 is a multiple of 8: 32-byte aligned
    const uint4 a = p[0], b = p[1];
    k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
    k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
  } else {
#pragma unroll
    for (uint32_t j = 0; j < kRangeKeys; ++j) k[j] = i0 + j < n ? skeys[i0 + j] : 0u;
  }
#pragma unroll
  for (uint32_t j = 0; j < kRangeKeys; ++j) k[j] = min(k[j] & tmask, T - 1);  // tiles are < T; keeps writes in bounds
  uint32_t kp = __shfl_up(k[kRangeKeys - 1], 1, 64);
  if ((threadIdx.x & 63) == 0 && i0 > 0 && i0 < n) kp = min(skeys[i0 - 1] & tmask, T - 1);
  if (i0 >= n) return;
#pragma unroll
  for (uint32_t j = 0; j < kRangeKeys; ++j) {
    const uint32_t i = i0 + j;
    if (i < n) {
      const uint32_t t0 = i ? kp + 1u : 0u;
      for (uint32_t t = t0; t <= k[j]; ++t) tile_start[t] = i;
      if (i == n - 1)
        for (uint32_t t = k[j] + 1; t <= T; ++t) tile_start[t] = n;
      kp = k[j];
    }
  }
}

// Blocks of the sort: chunks of at least 2048 keys (half a round), at most
// 2048 blocks (larger inputs walk several full rounds per block).
uint32_t sort_blocks_for(uint32_t key_cap) {
  uint32_t g = (key_cap + 2047u) / 2048u;
  if (g < 1) g = 1;
  if (g > kSortMaxBlocks) g = kSortMaxBlocks;
  return g;
}

// Digit width of every pass: the whole tile id in one pass when it has at
// most 10 bits and the input is small (at most kWideMaxBlocks blocks, so the
// block-major histograms stay small); otherwise the bits split evenly over
// passes of at most 8 bits, so small tile counts get fewer digits and longer
// runs per digit.
int sort_digit_bits(int bits, uint32_t G) {
  if (bits < 1) bits = 1;
  if (bits <= 10 && G <= kWideMaxBlocks) return bits;
  const int p = (bits + 7) / 8;
  return (bits + p - 1) / p;
}

int sort_passes(int bits, uint32_t G) {
  if (bits < 1) bits = 1;
  const int d = sort_digit_bits(bits, G);
  return (bits + d - 1) / d;
}

uint32_t sort_digit_slots(int bits, uint32_t G) { return sort_digit_bits(bits, G) > 8 ? 1024u : 256u; }

hipError_t launch_radix_hist(const Ctrl* ctrl, const uint32_t* keys, uint32_t* hist, uint32_t G, int bits, int pass,
                             hipStream_t s) {
  const int db = sort_digit_bits(bits, G);
  if (db > 8)
    hipLaunchKernelGGL(k_radix_hist<1024>, dim3(G), dim3(kSortThreads), 0, s, ctrl, keys, G, db * pass,
                       (1u << db) - 1u, hist);
  else
    hipLaunchKernelGGL(k_radix_hist<256>, dim3(G), dim3(kSortThreads), 0, s, ctrl, keys, G, db * pass,
                       (1u << db) - 1u, hist);
  return hipGetLastError();
}

hipError_t launch_radix_colscan(uint32_t* hist, uint32_t G, int bits, hipStream_t s) {
  const uint32_t D = sort_digit_slots(bits, G);
  if (D == 1024u)
    hipLaunchKernelGGL(k_radix_colscan<1024>, dim3(D), dim3(256), 0, s, hist, G, hist + (size_t)D * G);
  else
    hipLaunchKernelGGL(k_radix_colscan<256>, dim3(D), dim3(256), 0, s, hist, G, hist + (size_t)D * G);
  return hipGetLastError();
}

hipError_t launch_radix_scatter(const Ctrl* ctrl, const uint32_t* const in[3], uint32_t* const out[3],
                                const uint32_t* hist, uint32_t G, int bits, int pass, uint32_t* tile_start,
                                uint32_t num_tiles, hipStream_t s) {
  const int db = sort_digit_bits(bits, G);
  const uint32_t D = sort_digit_slots(bits, G);
  const SortSet si{const_cast<uint32_t*>(in[0]), const_cast<uint32_t*>(in[1]), const_cast<uint32_t*>(in[2])};
  const SortSet so{out[0], out[1], out[2]};
  const uint32_t* coltot = hist + (size_t)D * G;
  if (D == 1024u)  // only for G <= kWideMaxBlocks
    hipLaunchKernelGGL((k_radix_scatter<8, 1024>), dim3(G), dim3(kSortThreads), 0, s, ctrl, si, so, pass == 0,
                       hist, coltot, G, db * pass, db, tile_start, num_tiles);
  else if (G >= kSortMaxBlocks)
    hipLaunchKernelGGL(k_radix_scatter_large, dim3(G), dim3(kSortThreads), 0, s, ctrl, si, so, pass == 0,
                       hist, coltot, G, db * pass, db, tile_start, num_tiles);
  else
    hipLaunchKernelGGL((k_radix_scatter<8, 256>), dim3(G), dim3(kSortThreads), 0, s, ctrl, si, so, pass == 0,
                       hist, coltot, G, db * pass, db, tile_start, num_tiles);
  return hipGetLastError();
}

hipError_t launch_tile_ranges(const Ctrl* ctrl, const uint32_t* skeys, uint32_t num_tiles, uint32_t key_cap,
                              int mask_shift, uint32_t* tile_start, hipStream_t s) {
  const uint32_t tmask = mask_shift >= 32 ? 0xffffffffu : (1u << mask_shift) - 1u;
  const uint32_t blocks = (key_cap + 256u * kRangeKeys - 1u) / (256u * kRangeKeys);
  hipLaunchKernelGGL(k_tile_ranges, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, s, ctrl, skeys, num_tiles, tmask,
                     tile_start);
  return hipGetLastError();
}

}  // namespace ug
