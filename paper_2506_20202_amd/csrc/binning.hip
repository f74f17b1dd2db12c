// Tile binning and the tile|depth sort.
//
// The pairs are ordered by the 64-bit key (tile << 32 | float32 depth bits),
// ties by Gaussian index, with a stable LSD radix sort.  LSD handles the low
// (depth) digits first, and all pairs of one Gaussian share its depth, so the
// depth passes run on the drawn Gaussians before expansion:
//   1-2. four 8-bit LSD passes on the depth bits of the drawn Gaussians (stable:
//      ties stay in index order); the first pass reads all Gaussians in index
//      order and keeps the drawn ones, so no separate compaction runs;
//   3. exclusive scan of tiles_touched in that order and emission of one
//      (tile, index) pair per listed tile (the tiles of the rectangle the
//      Gaussian reaches) -- the pairs are now in depth order;
//   4. ceil(log2(tiles) / 8) stable LSD passes on the tile digits, the last one
//      writing the 64-bit keys;
//   5. per-tile [start, end) ranges and the blend schedule.
// This is the same permutation as sorting the expanded pairs by all their key
// bits, with the four depth passes over ~P / 5 items instead of P.
//
// The pair offsets are a reduce-then-scan over 256-Gaussian chunks of the
// depth order: a sum of the tile counts per chunk, and each emit workgroup
// adds the sums before its chunk to get its first pair (a few KB of reads
// that stay in L2, instead of a kernel that scans the sums).  Inside a chunk
// the prefix is a wavefront-ballot scan: bit b of every lane's count is
// gathered with one 64-lane ballot, and mbcnt (popcount of the ballot below
// the lane) times 2^b is added to the lane's prefix; the loop stops at the
// highest bit any lane still holds.  Four wave totals are combined through
// LDS.
#include "rara_internal.h"

namespace rara {

namespace {

__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Exclusive prefix of v over the 64 lanes of the wave and the wave total.
__device__ inline uint32_t wave_ballot_scan(uint32_t v, uint32_t& total)
{
    uint32_t prefix = 0, tot = 0;
    uint32_t rem = v;
    for (int b = 0; b < 32; ++b) {
        const uint64_t m = __ballot(rem & 1u);
        prefix += lanes_below(m) << b;
        tot += (uint32_t)__popcll(m) << b;
        rem >>= 1;
        if (__ballot(rem != 0u) == 0ull) break;
    }
    total = tot;
    return prefix;
}

// Exclusive prefix over a 256-thread block (4 waves) and the block total.
__device__ inline uint32_t block_ballot_scan(uint32_t v, uint32_t& total)
{
    __shared__ uint32_t wave_tot[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t wt;
    const uint32_t p = wave_ballot_scan(v, wt);
    if (lane == 0) wave_tot[wave] = wt;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    total = wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
    return before + p;
}

// Rectangle (tx0, ty0, tx1, ty1) and area of a tile record.
__device__ inline ushort4 record_rect(const ulonglong2& r)
{
    return make_ushort4((unsigned short)r.x, (unsigned short)(r.x >> 16), (unsigned short)(r.x >> 32),
                        (unsigned short)(r.x >> 48));
}

__device__ inline int rect_area(const ushort4& rc) { return (int)(rc.z - rc.x) * (int)(rc.w - rc.y); }

// Per-chunk sums of the tile counts over the depth order (k < *count), chunk
// b = the 256 Gaussians from b * 256; also gathers each drawn Gaussian's tile
// record (rectangle and listed-tile mask) into depth order (drec[k] =
// tile_rec[order[k]]), so that the emit reads them in sequence instead of
// gathering them again.  The count is the number of listed tiles
// (tiles_touched of a drawn Gaussian).
__global__ __launch_bounds__(256) void chunk_sum_kernel(const ulonglong2* __restrict__ tile_rec,
                                                        const uint32_t* __restrict__ order,
                                                        const int64_t* __restrict__ count,
                                                        uint32_t* __restrict__ chunk_sums,
                                                        ulonglong2* __restrict__ drec)
{
    const int64_t drawn = *count;
    if ((int64_t)blockIdx.x * kScanBlock >= drawn) {   // past the drawn Gaussians: uniform
        if (threadIdx.x == 0) chunk_sums[blockIdx.x] = 0u;
        return;
    }
    const int64_t k = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    uint32_t v = 0u;
    if (k < drawn) {
        const ulonglong2 r = tile_rec[order[k]];
        drec[k] = r;
        v = listed_count(r.y, rect_area(record_rect(r)));
    }
    uint32_t total;
    block_ballot_scan(v, total);
    if (threadIdx.x == 0) chunk_sums[blockIdx.x] = total;
}

// A frame without Gaussians: no pairs, no overflow.
__global__ void no_pairs_kernel(int64_t* __restrict__ num_pairs, int32_t* __restrict__ overflow)
{
    *num_pairs = 0;
    *overflow = 0;
}

// One (tile, index) pair per listed tile, Gaussians taken in depth order.
// A workgroup owns 256 consecutive Gaussians of the depth order (chunk b) and
// the contiguous run of pairs they emit, from the sum of the chunk sums before
// it; the last workgroup also writes the pair count and the overflow flag.  A
// workgroup whose pairs do not all fit the capacity writes none (the frame
// then overflows).  The pairs are expanded cooperatively: thread e of each
// 256-pair step finds the Gaussian that owns pair e by a binary search over
// the workgroup's inclusive pair offsets in LDS, so the work per thread does
// not depend on footprint sizes and the stores of a step are consecutive.
__global__ __launch_bounds__(256) void emit_kernel(const ulonglong2* __restrict__ drec,
                                                   const uint32_t* __restrict__ order,
                                                   const int64_t* __restrict__ count,
                                                   const uint32_t* __restrict__ chunk_sums, int64_t cap,
                                                   int tiles_x, int64_t* __restrict__ num_pairs,
                                                   int32_t* __restrict__ overflow, uint32_t* __restrict__ tkeys,
                                                   uint32_t* __restrict__ tvals, uint32_t* __restrict__ pair_start)
{
    __shared__ uint32_t s_end[kScanBlock];   // inclusive end of each Gaussian's pairs inside the workgroup
    __shared__ uint32_t s_id[kScanBlock];
    __shared__ ushort4 s_rc[kScanBlock];
    __shared__ uint64_t s_mk[kScanBlock];
    __shared__ uint64_t s_part[kScanBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b = blockIdx.x;
    const bool last_block = b == (int64_t)gridDim.x - 1;
    const int64_t drawn = *count;
    // a chunk past the drawn Gaussians emits nothing; the last workgroup still
    // sums every chunk for the pair count
    if (b * kScanBlock >= drawn && !last_block) return;
    // pairs before this chunk: 8 loads per thread in flight per step
    uint64_t before = 0;
    for (int64_t c0 = 0; c0 < b; c0 += 8 * kScanBlock) {
        uint32_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t c = c0 + u * kScanBlock + tid;
            x[u] = chunk_sums[c < b ? c : b - 1];   // unconditional (b >= 1 here): no load waits for another
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) before += c0 + u * kScanBlock + tid < b ? x[u] : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) before += __shfl_xor(before, off, 64);
    const int64_t k = b * kScanBlock + tid;
    const bool valid = k < drawn;
    const uint32_t id = valid ? order[k] : 0u;
    const ulonglong2 rec = valid ? drec[k] : make_ulonglong2(0ull, 0ull);
    const ushort4 rk = valid ? record_rect(rec) : make_ushort4(0, 0, 1, 1);
    const uint64_t mk = rec.y;
    const uint32_t v = valid ? listed_count(mk, rect_area(rk)) : 0u;
    if (lane == 0) s_part[wave] = before;
    uint32_t total;
    const uint32_t pre = block_ballot_scan(v, total);   // its barrier orders s_part
    const uint64_t base64 = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    if (last_block && tid == 0) {
        const uint64_t P = base64 + total;
        *num_pairs = (int64_t)P;
        *overflow = P > (uint64_t)cap ? 1 : 0;
    }
    if (total == 0u || base64 + total > (uint64_t)cap) return;   // uniform over the workgroup
    const uint32_t base = (uint32_t)base64;
    if (pair_start && v) pair_start[id] = base + pre;   // first pair of this Gaussian, emission order
    s_end[tid] = pre + v;
    s_id[tid] = id;
    s_rc[tid] = v ? rk : make_ushort4(0, 0, 1, 1);
    s_mk[tid] = mk;
    __syncthreads();
    for (uint32_t e = (uint32_t)tid; e < total; e += kScanBlock) {
        // owner = number of Gaussians whose pairs all precede e (s_end is non-decreasing, s_end[255] = total)
        int own = 0;
#pragma unroll
        for (int step = kScanBlock / 2; step > 0; step >>= 1)
            if (s_end[own + step - 1] <= e) own += step;
        const uint32_t li = e - (own ? s_end[own - 1] : 0u);
        const ushort4 rc = s_rc[own];
        const uint32_t w = (uint32_t)(rc.z - rc.x);
        const uint32_t pos = listed_tile(s_mk[own], (int)w * (int)(rc.w - rc.y), li);   // in the rectangle
        const uint32_t row = pos / w, col = pos - row * w;
        tkeys[base + e] = (uint32_t)((rc.y + row) * (uint32_t)tiles_x + rc.x + col);
        tvals[base + e] = s_id[own];
    }
}

__global__ __launch_bounds__(256) void ranges_clear_kernel(uint32_t* __restrict__ ranges, int num_tiles)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < num_tiles) reinterpret_cast<uint2*>(ranges)[t] = make_uint2(0u, 0u);
}

// Blend schedule: the tiles whose list has at least kHeavyList entries come
// first, so that the longest walks start earliest, and among them the up to
// kMaxUnitTiles longest (the forward blend gives the first kMaxUnitTiles of
// the group four workgroups each): those of at least L* entries, L* the
// smallest of kHeavyList + kUnitBucket k (k = 0 .. 255) that at most
// kMaxUnitTiles lists reach, from a histogram of the long lists' lengths; then
// the other tiles; each class in tile order.  work[h] = h-th long-list tile,
// work[H + l] = l-th other tile, work[T] = H.  Tiles without pairs (end 0) get
// the empty range (0, 0).
//
// One 1024-thread workgroup, so all of it runs on one CU: the accesses are
// kept coalesced (thread t takes tiles t, t + 1024, ... of each 8192-tile
// block) and the class flags are counted with wave ballots.  A tile's rank in
// its class is the class count of the blocks before it, of the rounds of 1024
// tiles before it in its block, of the waves before it in its round, and of
// the lanes before it in its wave.  A first sweep counts the classes (the
// ranges of the first block stay in registers), the second writes the ranges
// and the schedule.
__device__ inline uint32_t plan_len(uint2 r) { return r.y != 0u ? r.y - r.x : 0u; }
__device__ inline bool plan_heavy(uint2 r) { return plan_len(r) >= kHeavyList; }
// histogram bucket of a long list's length
__device__ inline uint32_t plan_bucket(uint32_t len) { return min(255u, (len - kHeavyList) / kUnitBucket); }

__global__ __launch_bounds__(1024) void plan_kernel(uint2* __restrict__ ranges, int num_tiles,
                                                    uint32_t* __restrict__ work)
{
    constexpr int kRounds = 8, kBlock = kRounds * 1024;
    // per (round, wave): the count of each class (very long, long), then its exclusive prefix
    __shared__ uint32_t s_cnt[2][kRounds * 16];
    __shared__ uint32_t s_tot[2][16];
    __shared__ uint32_t s_hist[256];   // long lists per length bucket
    __shared__ uint32_t s_unit[2];     // L*, V
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto load_block = [&](int b0, uint2* r) {
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const int t = b0 + j * 1024 + tid;
            r[j] = ranges[t < num_tiles ? t : num_tiles - 1];
            if (t >= num_tiles) r[j] = make_uint2(0u, 0u);
        }
    };
    if (tid < 256) s_hist[tid] = 0u;
    __syncthreads();
    // sweep 1: H (all long) and the histogram of the long lists' lengths
    uint2 r0[kRounds];
    load_block(0, r0);
    uint32_t hc = 0;
#pragma unroll
    for (int j = 0; j < kRounds; ++j)
        if (plan_heavy(r0[j])) {
            ++hc;
            atomicAdd(&s_hist[plan_bucket(plan_len(r0[j]))], 1u);
        }
    for (int b0 = kBlock; b0 < num_tiles; b0 += kBlock) {
        uint2 r[kRounds];
        load_block(b0, r);
#pragma unroll
        for (int j = 0; j < kRounds; ++j)
            if (plan_heavy(r[j])) {
                ++hc;
                atomicAdd(&s_hist[plan_bucket(plan_len(r[j]))], 1u);
            }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hc += __shfl_xor(hc, off, 64);
    if (lane == 0) s_tot[1][wave] = hc;
    __syncthreads();
    if (wave == 0) {
        // S(k) = long lists in buckets k.. (non-increasing in k); k* = the smallest k with
        // S(k) <= kMaxUnitTiles (256 when none), L* = kHeavyList + kUnitBucket k*, V = S(k*).
        // Lane l holds buckets 4l .. 4l + 3.
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h[i] = s_hist[4 * lane + i];
            sum += h[i];
        }
        uint32_t suf = sum;   // inclusive suffix over lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_down(suf, off, 64);
            if (lane + off < 64) suf += o;
        }
        uint32_t S[4];
        S[3] = suf - sum + h[3];
        S[2] = S[3] + h[2];
        S[1] = S[2] + h[1];
        S[0] = S[1] + h[0];
        int kl = 4;   // this lane's smallest qualifying bucket, 4 when none
#pragma unroll
        for (int i = 3; i >= 0; --i)
            if (S[i] <= kMaxUnitTiles) kl = i;
        const uint64_t q = __ballot(kl < 4);
        if (q == 0ull) {
            if (lane == 0) {
                s_unit[0] = 0xffffffffu;
                s_unit[1] = 0u;
            }
        } else if (lane == (int)__builtin_ctzll(q)) {
            s_unit[0] = kHeavyList + kUnitBucket * (uint32_t)(4 * lane + kl);
            s_unit[1] = S[kl];
        }
    }
    __syncthreads();
    const uint32_t Lstar = s_unit[0], V = s_unit[1];
    uint32_t H = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) H += s_tot[1][w];
    __syncthreads();   // s_tot is rewritten below
    auto plan_unit = [&](uint2 r) { return plan_len(r) >= Lstar; };
    // sweep 2: ranges and positions, block by block
    uint32_t carry[2] = {0u, 0u};   // tiles of each class in the blocks before
    for (int b0 = 0; b0 < num_tiles; b0 += kBlock) {
        uint2 r[kRounds];
        if (b0 == 0) {
#pragma unroll
            for (int j = 0; j < kRounds; ++j) r[j] = r0[j];
        } else {
            load_block(b0, r);
        }
        uint64_t mv[kRounds], ml[kRounds];
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            mv[j] = __ballot(plan_unit(r[j]));
            ml[j] = __ballot(plan_heavy(r[j]) && !plan_unit(r[j]));
            if (lane == 0) {
                s_cnt[0][j * 16 + wave] = (uint32_t)__popcll(mv[j]);
                s_cnt[1][j * 16 + wave] = (uint32_t)__popcll(ml[j]);
            }
        }
        __syncthreads();
        if (wave < 2) {   // exclusive prefix of each class's 128 counts in (round, wave) order, two per lane
            uint32_t* c = s_cnt[wave];
            const uint32_t c0 = c[2 * lane], c1 = c[2 * lane + 1];
            uint32_t incl = c0 + c1;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t o = __shfl_up(incl, off, 64);
                if (lane >= off) incl += o;
            }
            const uint32_t ex = incl - c0 - c1;
            c[2 * lane] = ex;
            c[2 * lane + 1] = ex + c0;
            if (lane == 63) s_tot[wave][0] = incl;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            const int t = b0 + j * 1024 + tid;
            if (t < num_tiles) {
                const bool very = ((mv[j] >> lane) & 1ull) != 0ull;
                const bool lng = ((ml[j] >> lane) & 1ull) != 0ull;
                const uint32_t vb = carry[0] + s_cnt[0][j * 16 + wave] +
                                    __builtin_amdgcn_mbcnt_hi((uint32_t)(mv[j] >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mv[j], 0u));
                const uint32_t lb = carry[1] + s_cnt[1][j * 16 + wave] +
                                    __builtin_amdgcn_mbcnt_hi((uint32_t)(ml[j] >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)ml[j], 0u));
                ranges[t] = r[j].y == 0u ? make_uint2(0u, 0u) : r[j];
                work[very ? vb : lng ? V + lb : H + (uint32_t)t - vb - lb] = (uint32_t)t;
            }
        }
        carry[0] += s_tot[0][0];
        carry[1] += s_tot[1][0];
        __syncthreads();   // s_cnt and s_tot are rewritten by the next block
    }
    if (tid == 0) work[num_tiles] = H;
}

}  // namespace

hipError_t launch_plan(const rara_binned& out, int num_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, reinterpret_cast<uint2*>(out.ranges), num_tiles,
                       out.work);
    return hipGetLastError();
}

hipError_t launch_bin(const ProjPtrs& proj, int64_t n, const CamParams& cam, int64_t cap, const BinWorkspace& ws,
                      const rara_binned& out, int tile_passes, hipStream_t s)
{
    const int64_t nb = ws.scan_blocks;
    const uint32_t num_tiles = (uint32_t)(cam.tiles_x * cam.tiles_y);
    // 1-2. depth order of the drawn Gaussians: the first of the four passes
    // takes them straight from the preprocess output (and counts them); the
    // result is back in buffer 0
    if (n > 0) {
        const SortFirstPass first{proj.depth, proj.tiles_touched, n, ws.dcount, out.ranges,
                                  (int64_t)num_tiles * 2};
        hipError_t e = sort_passes(ws.dkeys[0], ws.dvals[0], ws.dkeys[1], ws.dvals[1], 4, kDepthSortItems, ws.dcount,
                                   nullptr, ws.depth_blocks, ws.hist, ws.digit_totals, nullptr, nullptr, nullptr,
                                   &first, nullptr, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)nb), dim3(256), 0, s, proj.tile_rec, ws.dvals[0],
                           ws.dcount, ws.block_sums, ws.drec);
    } else {
        hipLaunchKernelGGL(no_pairs_kernel, dim3(1), dim3(1), 0, s, out.num_pairs, out.overflow);
    }
    // the last tile pass must read the workspace buffer, never out.keys, which
    // it writes; the other buffer lives in out.keys (cap x (u32, u32) fits)
    uint32_t* alias_k = reinterpret_cast<uint32_t*>(out.keys);
    uint32_t* alias_v = alias_k + cap;
    const bool last_reads_a = ((tile_passes - 1) & 1) == 0;
    uint32_t* ka = last_reads_a ? ws.tkeys : alias_k;
    uint32_t* va = last_reads_a ? ws.tvals : alias_v;
    uint32_t* kb = last_reads_a ? alias_k : ws.tkeys;
    uint32_t* vb = last_reads_a ? alias_v : ws.tvals;
    // 3. pair offsets in depth order, pair count, overflow flag, emission
    if (n > 0)
        hipLaunchKernelGGL(emit_kernel, dim3((unsigned)nb), dim3(256), 0, s, ws.drec, ws.dvals[0],
                           ws.dcount, ws.block_sums, cap, cam.tiles_x, out.num_pairs, out.overflow, ka, va,
                           out.pair_start);
    // 4. tile digits; the last pass writes the 64-bit keys and the values, and
    // the tile ranges (tiles without pairs keep (0xffffffff, 0) for plan_kernel)
    const SortLastPass last{n > 0 ? out.ranges : nullptr, num_tiles};
    return sort_passes(ka, va, kb, vb, tile_passes, kSortItems, out.num_pairs, out.overflow, ws.tile_blocks, ws.hist,
                       ws.digit_totals, out.keys_scratch ? nullptr : out.keys, out.vals, proj.depth, nullptr, &last,
                       s);
}

hipError_t launch_ranges_clear(const rara_binned& out, int num_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(ranges_clear_kernel, dim3((num_tiles + 255) / 256), dim3(256), 0, s, out.ranges, num_tiles);
    return hipGetLastError();
}

}  // namespace rara
