// Stable LSD radix sort passes (8-bit digits) of (uint32 key, uint32 value)
// pairs, used twice per frame by the binning stage: on the depth keys of the
// drawn Gaussians and on the tile keys of the emitted (tile, Gaussian) pairs.
// The last tile pass writes the 64-bit (tile << 32 | float32 depth bits) keys.
//
// Each pass is reduce-then-scan, with no inter-workgroup waiting:
//   upsweep  - per 2048-key tile, a 256-bin digit histogram;
//   scan     - one workgroup per digit scans that digit's counts over tiles;
//   scatter  - each tile ranks its keys stably in LDS (per-wave ballot match
//              on the 8 digit bits, wave-private running counters), stages
//              keys and values in LDS in digit order, and writes each digit
//              run contiguously to its global position.
// The item count lives in device memory (written by the previous stage); the
// grids are sized from the capacity and tiles past the count exit at once.
#include "rara_internal.h"

namespace rara {

namespace {

constexpr int kWaves = kSortThreads / 64;
// kItems keys per thread: a sort tile holds kSortThreads * kItems keys and
// each wave owns 64 * kItems consecutive ones

__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sort tile of workgroup b.  Workgroups go to the 8 XCDs round robin (b mod 8)
// and every XCD takes one contiguous run of the live tiles, so neighbouring
// tiles -- whose histogram entries share cache lines and whose digit runs are
// written next to each other -- are merged in one L2.  The grid is a multiple
// of 8; -1 for a workgroup without a tile.
__device__ inline int64_t sort_tile_of_block(int64_t b, int64_t tiles)
{
    const int64_t per = (tiles + 7) / 8;
    const int64_t j = b >> 3;
    const int64_t t = (b & 7) * per + j;
    return (j < per && t < tiles) ? t : -1;
}

// Lanes of the wave whose (valid) digit equals this lane's digit.
__device__ inline uint64_t match_digit(uint32_t digit, bool valid)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// kFilter (first depth pass): item i is Gaussian i, taken when it is drawn
// (tiles_touched > 0), its key the bits of its positive depth; the kernel also
// resets the tile ranges of the frame (start 0xffffffff, end 0: no pair yet).
template <bool kFilter, int kItems>
__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(
    const uint32_t* __restrict__ keys, const int64_t* __restrict__ num_items, const int32_t* __restrict__ overflow,
    int shift, uint32_t* __restrict__ hist, int64_t stride, const float* __restrict__ depth,
    const uint32_t* __restrict__ tt, int64_t n_items, uint32_t* __restrict__ ranges, int64_t range_words)
{
    if (kFilter)
        for (int64_t w = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; w < range_words;
             w += (int64_t)gridDim.x * kSortThreads)
            ranges[w] = (w & 1) ? 0u : 0xffffffffu;
    if (overflow && *overflow) return;
    constexpr int kTileKeys = kSortThreads * kItems;
    const int64_t P = kFilter ? n_items : *num_items;
    const int64_t tile = sort_tile_of_block(blockIdx.x, (P + kTileKeys - 1) / kTileKeys);
    if (tile < 0) return;
    const int64_t base = tile * kTileKeys;
    __shared__ uint32_t counts[kWaves][kRadix];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kWaves * kRadix; k += kSortThreads) (&counts[0][0])[k] = 0u;
    __syncthreads();
    const int64_t wbase = base + (int64_t)wave * 64 * kItems;
    // every load of the wave first (the filter's depth and tile-count loads
    // together), then the counts
    uint32_t key[kItems];
    bool valid[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool in = idx < P;
        if (kFilter) {
            // unconditional loads (a clamped index; P >= 1 here), so that none waits for another
            const int64_t ic = in ? idx : P - 1;
            const uint32_t t = tt[ic];
            const uint32_t k = __float_as_uint(depth[ic]);
            valid[r] = in && t > 0u;
            key[r] = in ? k : 0u;
        } else {
            valid[r] = in;
            key[r] = in ? keys[idx] : 0u;
        }
    }
    // a histogram needs no ranks: one LDS atomic per key into the wave's own row
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (valid[r]) atomicAdd(&counts[wave][(key[r] >> shift) & (kRadix - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += counts[w][d];
        hist[(int64_t)d * stride + tile] = t;
    }
}

// One workgroup per digit: exclusive scan of hist[d][0..tiles) in place and the
// digit's total.  The item count is *num_items, or n_items without it.  The
// row is scanned in chunks of 4096 counts: coalesced loads (16 per thread, all
// in flight) into LDS, a serial scan of 16 consecutive counts per thread (the
// LDS rows are padded to 17 words, so the 64 lanes hit distinct banks), a
// block scan of the thread totals, and coalesced stores.
constexpr int kScanPer = 16;
constexpr int kScanChunk = 256 * kScanPer;

__device__ inline int scan_slot(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(256) void radix_scan_kernel(uint32_t* __restrict__ hist, int64_t stride,
                                                         const int64_t* __restrict__ num_items, int64_t n_items,
                                                         const int32_t* __restrict__ overflow,
                                                         uint32_t* __restrict__ digit_totals, int tile_keys)
{
    if (overflow && *overflow) return;
    const int64_t P = num_items ? *num_items : n_items;
    const int64_t tiles = (P + tile_keys - 1) / tile_keys;
    uint32_t* row = hist + (int64_t)blockIdx.x * stride;
    __shared__ uint32_t buf[kScanChunk + kScanChunk / kScanPer];
    __shared__ uint32_t wave_tot[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += kScanChunk) {
        const int m = (int)(tiles - c0 < kScanChunk ? tiles - c0 : kScanChunk);
        uint32_t v[kScanPer];
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = j * 256 + t;
            v[j] = i < m ? row[c0 + i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) buf[scan_slot(j * 256 + t)] = v[j];
        __syncthreads();
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = acc;
            acc += buf[t * (kScanPer + 1) + k];
        }
        // inclusive scan of the thread totals within the wave, then across waves
        uint32_t inc = acc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t up = __shfl_up(inc, off, 64);
            if (lane >= off) inc += up;
        }
        if (lane == 63) wave_tot[wave] = inc;
        __syncthreads();
        uint32_t before = carry, chunk = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            before += w < wave ? wave_tot[w] : 0u;
            chunk += wave_tot[w];
        }
        const uint32_t excl = before + inc - acc;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) buf[t * (kScanPer + 1) + k] = excl + v[k];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kScanPer; ++j) {
            const int i = j * 256 + t;
            if (i < m) row[c0 + i] = buf[scan_slot(i)];
        }
        carry += chunk;
        __syncthreads();   // buf and wave_tot are rewritten by the next chunk
    }
    if (t == 0) digit_totals[blockIdx.x] = carry;
}

// kFinal: keys_out is ignored and the 64-bit (key << 32 | depth bits of the
// value's Gaussian) key is written to final_keys instead (when not null).  kFilter: the input
// of radix_upsweep_kernel<true>; the pass also writes the number of drawn
// Gaussians to count_out.  last.ranges (optional): the tile ranges of
// SortLastPass.
template <bool kFinal, bool kFilter, int kItems>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const int64_t* __restrict__ num_items, const int32_t* __restrict__ overflow,
    int shift, const uint32_t* __restrict__ hist, int64_t stride, const uint32_t* __restrict__ digit_totals,
    uint64_t* __restrict__ final_keys, const float* __restrict__ depth, const uint32_t* __restrict__ tt,
    int64_t n_items, int64_t* __restrict__ count_out, SortLastPass last)
{
    if (overflow && *overflow) return;
    constexpr int kTileKeys = kSortThreads * kItems;
    const int64_t P = kFilter ? n_items : *num_items;
    const int64_t tile = sort_tile_of_block(blockIdx.x, (P + kTileKeys - 1) / kTileKeys);
    if (tile < 0) return;
    const int64_t base = tile * kTileKeys;

    __shared__ uint32_t s_keys[kTileKeys];
    __shared__ uint32_t s_vals[kTileKeys];
    __shared__ uint32_t counts[kWaves][kRadix];   // running per-wave digit counts, then per-wave starts
    __shared__ uint32_t local_start[kRadix];      // start of each digit run inside the tile
    __shared__ uint32_t global_start[kRadix];     // global position of that run
    __shared__ uint32_t wave_sum[kWaves];
    __shared__ uint32_t wave_gsum[kWaves];
    __shared__ uint32_t s_count;                  // keys of this tile

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this tile's digit offsets do not depend on the keys: issue their loads first
    const uint32_t gtot = digit_totals[tid];
    const uint32_t tile_off = hist[(int64_t)tid * stride + tile];
    for (int k = tid; k < kWaves * kRadix; k += kSortThreads) (&counts[0][0])[k] = 0u;
    __syncthreads();

    // 1. stable rank of every key within (wave, digit)
    const int64_t wbase = base + (int64_t)wave * 64 * kItems;
    uint32_t key[kItems];
    uint32_t val[kItems];
    uint32_t packed[kItems];   // digit | rank-within-wave-digit << 8 ; 0xffffffff = invalid
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool in = idx < P;
        bool valid;
        if (kFilter) {
            const int64_t ic = in ? idx : P - 1;   // unconditional loads, as in the upsweep
            const uint32_t t = tt[ic];
            const uint32_t k = __float_as_uint(depth[ic]);
            key[r] = in ? k : 0u;
            val[r] = (uint32_t)idx;
            valid = in && t > 0u;
        } else {
            key[r] = in ? keys_in[idx] : 0u;
            val[r] = in ? vals_in[idx] : 0u;
            valid = in;
        }
        packed[r] = valid ? 0u : 0xffffffffu;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const bool valid = packed[r] == 0u;
        const uint32_t d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(d, valid);
        uint32_t rank = 0;
        if (valid) {
            const uint32_t below = lanes_below(peers);
            rank = counts[wave][d] + below;
            // every peer has read the running count before the group's first lane updates it
            __builtin_amdgcn_wave_barrier();
            if (below == 0) counts[wave][d] += (uint32_t)__popcll(peers);
        } else {
            __builtin_amdgcn_wave_barrier();
        }
        packed[r] = valid ? (d | (rank << 8)) : 0xffffffffu;
    }
    __syncthreads();

    // 2. per-digit totals over the four waves, exclusive scan over digits
    uint32_t dtot = 0;
    {
        const int d = tid;   // kSortThreads == kRadix
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = counts[w][d];
            counts[w][d] = run;   // exclusive start of wave w inside digit d
            run += c;
        }
        dtot = run;
    }
    // exclusive scans over the 256 digits (4 waves x 64 lanes): local digit
    // starts from dtot, global digit bases from the pass-wide digit totals
    {
        uint32_t incl = dtot, gincl = gtot;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, 64);
            const uint32_t go = __shfl_up(gincl, off, 64);
            if (lane >= off) { incl += o; gincl += go; }
        }
        if (lane == 63) { wave_sum[wave] = incl; wave_gsum[wave] = gincl; }
        __syncthreads();
        uint32_t before = 0, gbefore = 0;
        for (int w = 0; w < wave; ++w) { before += wave_sum[w]; gbefore += wave_gsum[w]; }
        local_start[tid] = before + incl - dtot;
        global_start[tid] = gbefore + gincl - gtot + tile_off;
        if (tid == kRadix - 1) {
            s_count = before + incl;
            if (kFilter && tile == 0) *count_out = (int64_t)(gbefore + gincl);   // all drawn Gaussians
        }
    }
    __syncthreads();

    // 3. stage keys and values in LDS in digit order
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (packed[r] != 0xffffffffu) {
            const uint32_t d = packed[r] & 0xffu;
            const uint32_t pos = local_start[d] + counts[wave][d] + (packed[r] >> 8);
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();

    // 4. write each digit run contiguously
    const int cnt = (int)s_count;
    for (int k = tid; k < cnt; k += kSortThreads) {
        const uint32_t kk = s_keys[k];
        const uint32_t d = (kk >> shift) & (kRadix - 1);
        const uint32_t g = global_start[d] + ((uint32_t)k - local_start[d]);
        const uint32_t v = s_vals[k];
        if (!kFinal)
            keys_out[g] = kk;
        else if (final_keys)
            final_keys[g] = ((uint64_t)kk << 32) | (uint64_t)__float_as_uint(depth[v]);
        vals_out[g] = v;
        // equal keys are consecutive in s_keys and in the output: the first and
        // last of each group here bound the key's range (every workgroup's
        // groups of one key together form one interval)
        if (last.ranges && kk < last.num_tiles) {
            if (k == 0 || s_keys[k - 1] != kk) atomicMin(&last.ranges[2 * kk], g);
            if (k == cnt - 1 || s_keys[k + 1] != kk) atomicMax(&last.ranges[2 * kk + 1], g + 1u);
        }
    }
}

}  // namespace

namespace {

template <int kItems>
hipError_t sort_passes_t(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int passes, const int64_t* count,
                         const int32_t* overflow, int64_t blocks, uint32_t* hist, uint32_t* digit_totals,
                         uint64_t* final_keys, uint32_t* final_vals, const float* depth, const SortFirstPass* first,
                         const SortLastPass* last, hipStream_t s)
{
    constexpr int kTileKeys = kSortThreads * kItems;
    const SortLastPass none{nullptr, 0u};
    // pass p reads (ka, va) when p is even and (kb, vb) when odd; with final_vals
    // the last pass writes (final_keys, final_vals) instead of the other buffer
    // (final_keys may be null: no keys written);
    // with `first`, pass 0 reads the drawn Gaussians instead of (ka, va) and
    // writes their number to first->count_out (the `count` of later passes)
    const unsigned grid = (unsigned)((blocks + 7) / 8 * 8);   // see sort_tile_of_block
    for (int p = 0; p < passes; ++p) {
        const bool even = (p & 1) == 0;
        const uint32_t* kin = even ? ka : kb;
        const uint32_t* vin = even ? va : vb;
        uint32_t* kout = even ? kb : ka;
        uint32_t* vout = even ? vb : va;
        const int shift = p * kRadixBits;
        const bool filter = first && p == 0;
        const SortLastPass lp = (last && p == passes - 1) ? *last : none;
        const dim3 g(grid), t(kSortThreads);
        if (filter) {
            hipLaunchKernelGGL((radix_upsweep_kernel<true, kItems>), g, t, 0, s, nullptr, nullptr, overflow, shift,
                               hist, blocks, first->depth, first->tt, first->n, first->ranges, first->range_words);
            hipLaunchKernelGGL(radix_scan_kernel, dim3(kRadix), dim3(256), 0, s, hist, blocks, nullptr, first->n,
                               overflow, digit_totals, kTileKeys);
            hipLaunchKernelGGL((radix_scatter_kernel<false, true, kItems>), g, t, 0, s, nullptr, nullptr, kout, vout,
                               nullptr, overflow, shift, hist, blocks, digit_totals, nullptr, first->depth, first->tt,
                               first->n, first->count_out, lp);
            continue;
        }
        hipLaunchKernelGGL((radix_upsweep_kernel<false, kItems>), g, t, 0, s, kin, count, overflow, shift, hist,
                           blocks, nullptr, nullptr, (int64_t)0, nullptr, (int64_t)0);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(kRadix), dim3(256), 0, s, hist, blocks, count, (int64_t)0,
                           overflow, digit_totals, kTileKeys);
        if (final_vals && p == passes - 1)
            hipLaunchKernelGGL((radix_scatter_kernel<true, false, kItems>), g, t, 0, s, kin, vin, kout, final_vals,
                               count, overflow, shift, hist, blocks, digit_totals, final_keys, depth, nullptr,
                               (int64_t)0, nullptr, lp);
        else
            hipLaunchKernelGGL((radix_scatter_kernel<false, false, kItems>), g, t, 0, s, kin, vin, kout, vout, count,
                               overflow, shift, hist, blocks, digit_totals, nullptr, nullptr, nullptr, (int64_t)0,
                               nullptr, lp);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t sort_passes(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int passes, int items,
                       const int64_t* count, const int32_t* overflow, int64_t blocks, uint32_t* hist,
                       uint32_t* digit_totals, uint64_t* final_keys, uint32_t* final_vals, const float* depth,
                       const SortFirstPass* first, const SortLastPass* last, hipStream_t s)
{
    if (items == kDepthSortItems)
        return sort_passes_t<kDepthSortItems>(ka, va, kb, vb, passes, count, overflow, blocks, hist, digit_totals,
                                              final_keys, final_vals, depth, first, last, s);
    return sort_passes_t<kSortItems>(ka, va, kb, vb, passes, count, overflow, blocks, hist, digit_totals, final_keys,
                                     final_vals, depth, first, last, s);
}

}  // namespace rara
