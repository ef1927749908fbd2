// Binning: device-wide exclusive scan, instance emission, a stable LSD radix
// sort of (key, value) pairs and the per-tile ranges of the sorted instances.
//
// Ordering strategy.  The per-pixel order is ascending (depth, Gaussian id)
// (eq. 1 of the paper orders primitives by the depth of their centres; ties
// are broken by id).  Instead of sorting one 64-bit (tile | depth) key per
// Gaussian-tile instance, the Gaussian-views are sorted once by their 32-bit
// depth key (stable, so equal depths keep id order), instances are emitted in
// that order, and a stable radix sort on the tile id alone (13-20 bits) groups
// them by tile without disturbing the depth order inside a tile.
#include "internal.h"

namespace rgs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItemsPerThread = 8;
constexpr int kTile = kThreads * kItemsPerThread;  // items per block
constexpr int kBins = 256;                         // 8-bit digits

// Element count of a device-sized array: a frame whose instance count
// overflowed the capacity is treated as empty downstream (its status reports
// the overflow), so no kernel ever reads entries that were not written.
__device__ __forceinline__ int64_t clamp_count(const int64_t *n_dev, int64_t n_max)
{
    if (!n_dev) return n_max;
    const int64_t n = *n_dev;
    return n <= n_max ? n : 0;
}

// Inclusive scan across a 256-thread block (4 waves); returns the inclusive
// prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t x, uint32_t *smem /*[kWaves]*/, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    if (lane == 63) smem[wave] = v;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = smem[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + v;
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n_max,
                                                         const int64_t *__restrict__ n_dev, int shift, int bits,
                                                         uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t cnt[kWaves][kBins];
    const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const int64_t n = clamp_count(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint32_t mask = (1u << bits) - 1u;
    if (base < n) {
#pragma unroll
        for (int j = 0; j < kItemsPerThread; ++j) {
            const int64_t idx = base + (int64_t)j * kThreads + tid;
            if (idx < n) atomicAdd(&cnt[wave][(keys[idx] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
}

// Exclusive scan of each digit's row hist[d][0..nblocks) (one block per digit).
__global__ __launch_bounds__(kThreads) void k_radix_scan_rows(uint32_t *__restrict__ hist, int nblocks,
                                                              uint32_t *__restrict__ row_total)
{
    __shared__ uint32_t smem[kWaves];
    uint32_t *row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int base = 0; base < nblocks; base += kThreads) {
        const int i = base + threadIdx.x;
        const uint32_t x = i < nblocks ? row[i] : 0u;
        uint32_t tot;
        const uint32_t inc = block_inclusive_scan(x, smem, &tot);
        if (i < nblocks) row[i] = carry + inc - x;
        carry += tot;
    }
    if (threadIdx.x == 0) row_total[blockIdx.x] = carry;
}

// Stable scatter of one block's items by digit.  Each wave ranks 8 rounds of
// 64 consecutive items: lanes holding the same digit are found with one ballot
// per digit bit, ranked by popcount of the lower peers, and a per-wave LDS
// counter per digit carries the rank across rounds.  Items are then staged in
// LDS in block-local sorted order and written out in runs of equal digits.
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, int64_t n_max, const int64_t *__restrict__ n_dev, int shift, int bits,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ row_total, int nblocks)
{
    __shared__ uint32_t wave_cnt[kWaves][kBins];
    __shared__ uint32_t block_start[kBins];
    __shared__ uint32_t out_base[kBins];
    __shared__ uint32_t s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t smem[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = clamp_count(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) return;  // uniform per block
    const uint32_t mask = (1u << bits) - 1u;

    // digit bases: exclusive scan of the row totals (thread = digit)
    uint32_t dig_total;
    const uint32_t rt = row_total[tid];
    const uint32_t dig_base = block_inclusive_scan(rt, smem, &dig_total) - rt;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();

    uint32_t my_key[kItemsPerThread], my_val[kItemsPerThread], my_rank[kItemsPerThread];
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kItemsPerThread; ++r) {
        const int64_t idx = base + (int64_t)wave * (kTile / kWaves) + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t key = valid ? keys_in[idx] : 0u;
        my_key[r] = key;
        my_val[r] = valid ? vals_in[idx] : 0u;
        const uint32_t d = (key >> shift) & mask;
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        const uint32_t prior = valid ? wave_cnt[wave][d] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wave_cnt[wave][d] = prior + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        my_rank[r] = valid ? prior + rank : 0xffffffffu;
    }
    __syncthreads();
    {
        // prefix over waves for digit tid, then block-local digit starts
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wave_cnt[w][tid];
            wave_cnt[w][tid] = run;
            run += c;
        }
        uint32_t tot;
        const uint32_t start = block_inclusive_scan(run, smem, &tot) - run;
        block_start[tid] = start;
        out_base[tid] = dig_base + hist[(size_t)tid * nblocks + blockIdx.x] - start;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItemsPerThread; ++r) {
        if (my_rank[r] == 0xffffffffu) continue;
        const uint32_t d = (my_key[r] >> shift) & mask;
        const uint32_t pos = block_start[d] + wave_cnt[wave][d] + my_rank[r];
        s_keys[pos] = my_key[r];
        s_vals[pos] = my_val[r];
    }
    __syncthreads();
    const int count = (int)((n - base) < kTile ? (n - base) : kTile);
    for (int p = tid; p < count; p += kThreads) {
        const uint32_t key = s_keys[p];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t dst = out_base[d] + (uint32_t)p;
        if ((int64_t)dst < n) {
            keys_out[dst] = key;
            vals_out[dst] = s_vals[p];
        }
    }
}

// ---------------------------------------------------------------------- scan
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ counts,
                                                          const uint32_t *__restrict__ gather, int64_t n,
                                                          unsigned long long *__restrict__ block_sums)
{
    __shared__ unsigned long long part[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    unsigned long long acc = 0;
#pragma unroll
    for (int j = 0; j < kItemsPerThread; ++j) {
        const int64_t idx = base + (int64_t)j * kThreads + threadIdx.x;
        if (idx < n) acc += counts[gather ? gather[idx] : idx];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) block_sums[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Single-block exclusive scan of the block sums; writes the grand total.
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long *__restrict__ block_sums, int nb,
                                                   int64_t *__restrict__ total)
{
    __shared__ unsigned long long wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const unsigned long long x = i < nb ? block_sums[i] : 0ull;
        unsigned long long v = x;
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long y = __shfl_up(v, d, 64);
            if (lane >= d) v += y;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        unsigned long long before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) before += wsum[w];
            all += wsum[w];
        }
        __syncthreads();
        if (i < nb) block_sums[i] = carry + before + v - x;
        carry += all;
    }
    if (threadIdx.x == 0) *total = (int64_t)carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t *__restrict__ counts,
                                                         const uint32_t *__restrict__ gather, int64_t n,
                                                         const unsigned long long *__restrict__ block_sums,
                                                         uint32_t *__restrict__ offsets)
{
    __shared__ uint32_t smem[kWaves];
    // blocked arrangement: thread t owns items base + t*8 .. +7
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItemsPerThread;
    uint32_t c[kItemsPerThread];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kItemsPerThread; ++j) {
        const int64_t idx = base + j;
        c[j] = idx < n ? counts[gather ? gather[idx] : idx] : 0u;
        local += c[j];
    }
    uint32_t tot;
    const uint32_t before = block_inclusive_scan(local, smem, &tot) - local;
    unsigned long long run = block_sums[blockIdx.x] + before;
#pragma unroll
    for (int j = 0; j < kItemsPerThread; ++j) {
        const int64_t idx = base + j;
        if (idx < n) offsets[idx] = run > 0xffffffffull ? 0xffffffffu : (uint32_t)run;
        run += c[j];
    }
}

// ---------------------------------------------------------------- emission
// One lane per sorted Gaussian-view writes its (tile, id) instances in
// row-major tile order at its scanned offset.  Rectangles of more than
// kEmitSolo tiles are queued in LDS and written by the whole wave, 64 tiles
// per step, so one large Gaussian does not serialise a lane.
constexpr uint32_t kEmitSolo = 16;

__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t *__restrict__ order,
                                                   const uint32_t *__restrict__ offsets,
                                                   const uint32_t *__restrict__ tile_counts,
                                                   const uint2 *__restrict__ rects, const DevView *__restrict__ views,
                                                   int64_t n, int64_t n_total, int64_t capacity,
                                                   uint32_t *__restrict__ inst_tiles, uint32_t *__restrict__ inst_ids)
{
    __shared__ uint32_t big[kWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t id = 0, cnt = 0;
    if (k < n_total) {
        id = order[k];
        cnt = tile_counts[id];
    }
    const bool solo = cnt > 0 && cnt <= kEmitSolo;
    if (solo) {
        const int v = (int)(id / (uint32_t)n);
        const uint2 r = rects[id];
        const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff, ty1 = r.y >> 16;
        const int tiles_x = views[v].tiles_x;
        const uint32_t tbase = (uint32_t)views[v].tile_base;
        int64_t pos = offsets[k];
        if (pos + cnt <= capacity) {  // overflow: the scan total reports it
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx, ++pos) {
                    inst_tiles[pos] = tbase + (uint32_t)(ty * tiles_x + tx);
                    inst_ids[pos] = id;
                }
        }
    }
    // queue the large rectangles of this wave and write them cooperatively
    const bool large = cnt > kEmitSolo;
    const unsigned long long mask = __ballot(large);
    if (large) big[wave][__popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)(k - (int64_t)blockIdx.x * kThreads);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nbig = __popcll(mask);
    for (int b = 0; b < nbig; ++b) {
        const int64_t kk = (int64_t)blockIdx.x * kThreads + big[wave][b];
        const uint32_t bid = order[kk];
        const uint32_t bcnt = tile_counts[bid];
        const int64_t base = offsets[kk];
        if (base + bcnt > capacity) continue;
        const int v = (int)(bid / (uint32_t)n);
        const uint2 r = rects[bid];
        const int tx0 = r.x & 0xffff, ty0 = r.x >> 16, tx1 = r.y & 0xffff;
        const uint32_t nx = (uint32_t)(tx1 - tx0 + 1);
        const int tiles_x = views[v].tiles_x;
        const uint32_t tbase = (uint32_t)views[v].tile_base;
        for (uint32_t j = lane; j < bcnt; j += 64) {
            const int ty = ty0 + (int)(j / nx), tx = tx0 + (int)(j % nx);
            inst_tiles[base + j] = tbase + (uint32_t)(ty * tiles_x + tx);
            inst_ids[base + j] = bid;
        }
    }
}

// ------------------------------------------------------------ tile ranges
__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ __launch_bounds__(kThreads) void k_tile_ranges(const uint32_t *__restrict__ inst_tiles,
                                                          const int64_t *__restrict__ counters, int64_t capacity,
                                                          int64_t total_tiles, uint2 *__restrict__ ranges)
{
    const int64_t m = clamp_count(counters, capacity);
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const uint32_t t = inst_tiles[p];
    if (t >= total_tiles) return;
    if (p == 0 || inst_tiles[p - 1] != t) ranges[t].x = (uint32_t)p;
    if (p == m - 1 || inst_tiles[p + 1] != t) ranges[t].y = (uint32_t)(p + 1);
}

// -------------------------------------------------------- tile scheduling
// Work order of the compositing kernels: tiles sorted by decreasing list
// length (coarse buckets of 4 entries, order inside a bucket arbitrary), so
// the longest tiles start first and the persistent grid drains evenly.
constexpr int kSchedBuckets = 256;

__device__ __forceinline__ uint32_t work_bucket(uint2 r)
{
    const uint32_t len = r.y - r.x;
    return min(len >> 2, (uint32_t)(kSchedBuckets - 1));
}

__global__ __launch_bounds__(kThreads) void k_sched_hist(const uint2 *__restrict__ ranges, int64_t total_tiles,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[kSchedBuckets];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t < total_tiles) atomicAdd(&cnt[work_bucket(ranges[t])], 1u);
    __syncthreads();
    if (cnt[threadIdx.x]) atomicAdd(&hist[threadIdx.x], cnt[threadIdx.x]);
}

__global__ __launch_bounds__(kThreads) void k_sched_scatter(const uint2 *__restrict__ ranges, int64_t total_tiles,
                                                            const uint32_t *__restrict__ hist,
                                                            uint32_t *__restrict__ cursor,
                                                            uint32_t *__restrict__ tile_order)
{
    __shared__ uint32_t smem[kWaves];
    __shared__ uint32_t base[kSchedBuckets];
    __shared__ uint32_t cnt[kSchedBuckets];
    // buckets in decreasing order: bucket b starts after all tiles of buckets > b
    const uint32_t hb = hist[kSchedBuckets - 1 - threadIdx.x];
    uint32_t tot;
    const uint32_t before = block_inclusive_scan(hb, smem, &tot) - hb;
    base[kSchedBuckets - 1 - threadIdx.x] = before;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t b = 0, rank = 0;
    if (t < total_tiles) {
        b = work_bucket(ranges[t]);
        rank = atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    if (cnt[threadIdx.x]) base[threadIdx.x] += atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (t < total_tiles) tile_order[base[b] + rank] = (uint32_t)t;
}

}  // namespace

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

size_t radix_hist_entries(int64_t n_max) { return (size_t)kBins * (size_t)((n_max + kTile - 1) / kTile + 1); }

hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n_max,
                      const int64_t *n_dev, int bits, uint32_t *hist, uint32_t *row_total, hipStream_t stream)
{
    const int nblocks = (int)((n_max + kTile - 1) / kTile);
    if (nblocks == 0 || bits <= 0) return hipSuccess;
    const int passes = radix_passes(bits);
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        // spread the bits evenly over the passes (each <= 8)
        const int pbits = (bits - shift + (passes - p) - 1) / (passes - p);
        k_radix_hist<<<nblocks, kThreads, 0, stream>>>(ki, n_max, n_dev, shift, pbits, hist, nblocks);
        k_radix_scan_rows<<<kBins, kThreads, 0, stream>>>(hist, nblocks, row_total);
        k_radix_scatter<<<nblocks, kThreads, 0, stream>>>(ki, vi, ko, vo, n_max, n_dev, shift, pbits, hist,
                                                          row_total, nblocks);
        shift += pbits;
        uint32_t *t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    return hipGetLastError();
}

size_t scan_block_entries(int64_t n) { return (size_t)((n + kTile - 1) / kTile + 1); }

hipError_t exclusive_scan_gather(const uint32_t *counts, const uint32_t *gather, uint32_t *offsets, int64_t n,
                                 unsigned long long *block_sums, int64_t *total, hipStream_t stream)
{
    const int nb = (int)((n + kTile - 1) / kTile);
    if (nb == 0) {
        k_fill_u32<<<1, kThreads, 0, stream>>>(reinterpret_cast<uint32_t *>(total), 0u, 2);
        return hipGetLastError();
    }
    k_scan_reduce<<<nb, kThreads, 0, stream>>>(counts, gather, n, block_sums);
    k_scan_top<<<1, 1024, 0, stream>>>(block_sums, nb, total);
    k_scan_apply<<<nb, kThreads, 0, stream>>>(counts, gather, n, block_sums, offsets);
    return hipGetLastError();
}

hipError_t launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *tile_counts, const uint2 *rects,
                       const DevView *views, int64_t n, int n_views, int64_t capacity, uint32_t *inst_tiles,
                       uint32_t *inst_ids, hipStream_t stream)
{
    const int64_t total = n * n_views;
    if (total == 0) return hipSuccess;
    k_emit<<<(unsigned)((total + kThreads - 1) / kThreads), kThreads, 0, stream>>>(
        order, offsets, tile_counts, rects, views, n, total, capacity, inst_tiles, inst_ids);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    k_fill_u32<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, stream>>>(p, value, n);
    return hipGetLastError();
}

size_t sched_words() { return 4 + 2 * kSchedBuckets; }

hipError_t launch_tile_ranges(const uint32_t *inst_tiles, const int64_t *counters, int64_t capacity,
                              int64_t total_tiles, uint2 *ranges, uint32_t *sched, uint32_t *tile_order,
                              hipStream_t stream)
{
    // empty ranges; the work-queue heads and scheduling histograms start at zero
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, 2 * total_tiles, stream);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(sched, 0u, (int64_t)sched_words(), stream);
    if (e != hipSuccess) return e;
    if (capacity > 0)
        k_tile_ranges<<<(unsigned)((capacity + kThreads - 1) / kThreads), kThreads, 0, stream>>>(inst_tiles, counters,
                                                                                                 capacity, total_tiles, ranges);
    const unsigned nb = (unsigned)((total_tiles + kThreads - 1) / kThreads);
    uint32_t *hist = sched + 4, *cursor = sched + 4 + kSchedBuckets;
    k_sched_hist<<<nb, kThreads, 0, stream>>>(ranges, total_tiles, hist);
    k_sched_scatter<<<nb, kThreads, 0, stream>>>(ranges, total_tiles, hist, cursor, tile_order);
    return hipGetLastError();
}

}  // namespace rgs
