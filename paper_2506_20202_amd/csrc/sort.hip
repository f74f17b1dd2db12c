// Stable LSD radix sort of (uint64 tile|depth key, uint32 index) pairs, 8-bit
// digits, only over the significant key bits (31 depth bits -- depths are
// positive floats -- plus ceil(log2(tiles)) tile bits).
//
// Each pass is reduce-then-scan, with no inter-workgroup waiting:
//   upsweep  - per 4096-key tile, a 256-bin digit histogram;
//   scan     - one workgroup per digit scans that digit's counts over tiles;
//   scatter  - each tile ranks its keys stably in LDS (per-wave ballot match
//              on the 8 digit bits, wave-private running counters), stages
//              keys and values in LDS in digit order, and writes each digit
//              run contiguously to its global position.
// The pair count lives in device memory (written by the binning stage); the
// grids are sized from the capacity and tiles past the count exit at once.
#include "rara_internal.h"

namespace rara {

namespace {

constexpr int kWaves = kSortThreads / 64;
constexpr int kWaveKeys = kSortTile / kWaves;   // consecutive keys owned by one wave

__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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

__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint64_t* __restrict__ keys,
                                                                     const int64_t* __restrict__ num_pairs,
                                                                     const int32_t* __restrict__ overflow, int shift,
                                                                     uint32_t* __restrict__ hist, int64_t stride)
{
    if (*overflow) return;
    const int64_t P = *num_pairs;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    if (base >= P) return;
    __shared__ uint32_t counts[kWaves][kRadix];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kWaves * kRadix; k += kSortThreads) (&counts[0][0])[k] = 0u;
    __syncthreads();
    const int64_t wbase = base + (int64_t)wave * kWaveKeys;
    for (int r = 0; r < kWaveKeys / 64; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool valid = idx < P;
        const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & (kRadix - 1) : 0u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && lanes_below(peers) == 0) counts[wave][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += counts[w][d];
        hist[(int64_t)d * stride + blockIdx.x] = t;
    }
}

// One workgroup per digit: exclusive scan of hist[d][0..tiles) in place and the
// digit's total.
__global__ __launch_bounds__(256) void radix_scan_kernel(uint32_t* __restrict__ hist, int64_t stride,
                                                         const int64_t* __restrict__ num_pairs,
                                                         const int32_t* __restrict__ overflow,
                                                         uint32_t* __restrict__ digit_totals)
{
    if (*overflow) return;
    const int64_t P = *num_pairs;
    const int64_t tiles = (P + kSortTile - 1) / kSortTile;
    uint32_t* row = hist + (int64_t)blockIdx.x * stride;
    __shared__ uint32_t part[256];
    const int t = threadIdx.x;
    const int64_t per = (tiles + 255) / 256;
    const int64_t lo = t * per, hi = lo + per < tiles ? lo + per : tiles;
    uint32_t acc = 0;
    for (int64_t k = lo; k < hi; ++k) acc += row[k];
    part[t] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int64_t k = lo; k < hi; ++k) {
        const uint32_t v = row[k];
        row[k] = run;
        run += v;
    }
    if (t == 255) digit_totals[blockIdx.x] = part[255];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint64_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const int64_t* __restrict__ num_pairs, const int32_t* __restrict__ overflow,
    int shift, const uint32_t* __restrict__ hist, int64_t stride, const uint32_t* __restrict__ digit_totals)
{
    if (*overflow) return;
    const int64_t P = *num_pairs;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    if (base >= P) return;

    __shared__ uint64_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t counts[kWaves][kRadix];   // running per-wave digit counts, then per-wave starts
    __shared__ uint32_t local_start[kRadix];      // start of each digit run inside the tile
    __shared__ uint32_t global_start[kRadix];     // global position of that run
    __shared__ uint32_t wave_sum[kWaves];
    __shared__ uint32_t wave_gsum[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < kWaves * kRadix; k += kSortThreads) (&counts[0][0])[k] = 0u;
    __syncthreads();

    // 1. stable rank of every key within (wave, digit)
    const int64_t wbase = base + (int64_t)wave * kWaveKeys;
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t packed[kSortItems];   // digit | rank-within-wave-digit << 8 ; 0xffffffff = invalid
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool valid = idx < P;
        key[r] = valid ? keys_in[idx] : 0ull;
        val[r] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = wbase + r * 64 + lane;
        const bool valid = idx < P;
        const uint32_t d = (uint32_t)(key[r] >> shift) & (kRadix - 1);
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
        const uint32_t gtot = digit_totals[tid];
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
        global_start[tid] = gbefore + gincl - gtot + hist[(int64_t)tid * stride + blockIdx.x];
    }
    __syncthreads();

    // 3. stage keys and values in LDS in digit order
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (packed[r] != 0xffffffffu) {
            const uint32_t d = packed[r] & 0xffu;
            const uint32_t pos = local_start[d] + counts[wave][d] + (packed[r] >> 8);
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();

    // 4. write each digit run contiguously
    const int64_t cnt64 = P - base < kSortTile ? P - base : kSortTile;
    const int cnt = (int)cnt64;
    for (int k = tid; k < cnt; k += kSortThreads) {
        const uint64_t kk = s_keys[k];
        const uint32_t d = (uint32_t)(kk >> shift) & (kRadix - 1);
        const uint32_t g = global_start[d] + ((uint32_t)k - local_start[d]);
        keys_out[g] = kk;
        vals_out[g] = s_vals[k];
    }
}

}  // namespace

hipError_t launch_sort(const BinWorkspace& ws, int64_t cap, const rara_binned& out, int passes, hipStream_t s)
{
    const int64_t blocks = ws.sort_blocks;
    const int64_t stride = ws.sort_blocks;
    // pass p reads src, writes dst; the last pass lands in out
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        const uint64_t* kin = to_out ? ws.keys_alt : out.keys;
        const uint32_t* vin = to_out ? ws.vals_alt : out.vals;
        uint64_t* kout = to_out ? out.keys : ws.keys_alt;
        uint32_t* vout = to_out ? out.vals : ws.vals_alt;
        const int shift = p * kRadixBits;
        hipLaunchKernelGGL(radix_upsweep_kernel, dim3((unsigned)blocks), dim3(kSortThreads), 0, s, kin, out.num_pairs,
                           out.overflow, shift, ws.hist, stride);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(kRadix), dim3(256), 0, s, ws.hist, stride, out.num_pairs,
                           out.overflow, ws.digit_totals);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)blocks), dim3(kSortThreads), 0, s, kin, vin, kout, vout,
                           out.num_pairs, out.overflow, shift, ws.hist, stride, ws.digit_totals);
    }
    (void)cap;
    return hipGetLastError();
}

}  // namespace rara
