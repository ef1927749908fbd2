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
#include <algorithm>

#include "internal.h"

namespace rgs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Binning scan: items per thread (4 or 8) chosen from the item count, as for
// the radix passes below.
constexpr int kScanItemsMin = 4;
constexpr int scan_tile(int items) { return kThreads * items; }
constexpr int kScanSelfPrefixBlocks = 1024;
// Scans of at least this many blocks write the row owner map in row order.
constexpr int kScanRowOrderBlocks = 4096;
// Radix sort: the keys per thread of a pass (ITEMS: 4, 8 or 16) are chosen
// per sort from its size.  More keys per workgroup amortise a workgroup's
// per-digit work on large sorts; fewer give small sorts enough workgroups to
// fill the CUs and a shorter serial ranking chain.
constexpr int kRadixItemsMin = 4;
constexpr int radix_tile(int items) { return kThreads * items; }
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
// Digit histogram of one block's items; with `drop`, keys equal to drop_key
// are left out (they leave the sort in this pass).  Blocks past the
// device-side count write nothing: the row scan and the scatter only look at
// the first ceil(n / (256 ITEMS)) blocks.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n_max,
                                                         const int64_t *__restrict__ n_dev, int shift, int bits,
                                                         bool drop, uint32_t drop_key, uint32_t *__restrict__ hist,
                                                         int nblocks)
{
    __shared__ uint32_t cnt[kWaves][kBins];
    const int tid = threadIdx.x, wave = tid >> 6;
    const int64_t n = clamp_count(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * radix_tile(ITEMS);
    if (base >= n) return;  // uniform per block
#pragma unroll
    for (int w = 0; w < kWaves; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t idx = base + (int64_t)j * kThreads + tid;
            if (idx < n) {
                const uint32_t key = keys[idx];
                if (!(drop && key == drop_key)) atomicAdd(&cnt[wave][(key >> shift) & mask], 1u);
            }
        }
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
}

// Exclusive scan of each digit's row hist[d][0..nb) (one block per digit)
// over the nb = ceil(n / tile) blocks that hold items (tile = keys per block).
__global__ __launch_bounds__(kThreads) void k_radix_scan_rows(uint32_t *__restrict__ hist, int nblocks,
                                                              int64_t n_max, const int64_t *__restrict__ n_dev,
                                                              int tile, uint32_t *__restrict__ row_total)
{
    __shared__ uint32_t smem[kWaves];
    const int64_t n = clamp_count(n_dev, n_max);
    const int nb = (int)std::min<int64_t>((n + tile - 1) / tile, nblocks);
    uint32_t *row = hist + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kThreads) {
        const int i = base + threadIdx.x;
        const uint32_t x = i < nb ? row[i] : 0u;
        uint32_t tot;
        const uint32_t inc = block_inclusive_scan(x, smem, &tot);
        if (i < nb) row[i] = carry + inc - x;
        carry += tot;
    }
    if (threadIdx.x == 0) row_total[blockIdx.x] = carry;
}

// Stable scatter of one block's items by digit.  Each wave ranks 8 rounds of
// 64 consecutive items: lanes holding the same digit are found with one ballot
// per digit bit, ranked by popcount of the lower peers, and a per-wave LDS
// counter per digit carries the rank across rounds.  Items are then staged in
// LDS in block-local sorted order and written out in runs of equal digits.
// With `drop`, keys equal to drop_key are not written, and block 0 stores
// the number of items kept (the sum of the digit totals) in *kept_out.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, int64_t n_max, const int64_t *__restrict__ n_dev, int shift, int bits,
    bool drop, uint32_t drop_key, int64_t *__restrict__ kept_out, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ row_total, int nblocks)
{
    __shared__ uint32_t wave_cnt[kWaves][kBins];
    __shared__ uint32_t block_start[kBins];
    __shared__ uint32_t out_base[kBins];
    __shared__ uint32_t s_keys[radix_tile(ITEMS)];
    __shared__ uint32_t s_vals[radix_tile(ITEMS)];
    __shared__ uint32_t smem[kWaves];
    __shared__ uint32_t block_valid;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = clamp_count(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * radix_tile(ITEMS);
    if (base >= n) {  // uniform per block
        if (drop && blockIdx.x == 0 && tid == 0) *kept_out = 0;
        return;
    }
    const uint32_t mask = (1u << bits) - 1u;

    // digit bases: exclusive scan of the row totals (thread = digit)
    uint32_t dig_total;
    const uint32_t rt = row_total[tid];
    const uint32_t dig_base = block_inclusive_scan(rt, smem, &dig_total) - rt;
    if (drop && blockIdx.x == 0 && tid == 0) *kept_out = (int64_t)dig_total;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();

    uint32_t my_key[ITEMS], my_val[ITEMS], my_rank[ITEMS];
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t idx = base + (int64_t)wave * (radix_tile(ITEMS) / kWaves) + r * 64 + lane;
        const uint32_t key = idx < n ? keys_in[idx] : 0u;
        const bool valid = idx < n && !(drop && key == drop_key);
        my_key[r] = key;
        my_val[r] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
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
        if (tid == 0) block_valid = tot;
        out_base[tid] = dig_base + hist[(size_t)tid * nblocks + blockIdx.x] - start;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (my_rank[r] == 0xffffffffu) continue;
        const uint32_t d = (my_key[r] >> shift) & mask;
        const uint32_t pos = block_start[d] + wave_cnt[wave][d] + my_rank[r];
        s_keys[pos] = my_key[r];
        s_vals[pos] = my_val[r];
    }
    __syncthreads();
    const int count = (int)block_valid;  // items of this block that stay in the sort
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
// Binning scan over the depth-sorted Gaussian-views: each item carries two
// counts, the tiles of its binning box (instances) and the tile rows of that
// box; both are scanned at once (block sums hold the pair as two uint64).
// A culled view (sorted key 0xffffffff, all at the end) counts nothing and
// costs no gather; a kept one reads its box.
__device__ __forceinline__ void scan_item(const uint32_t *__restrict__ keys, const uint2 *__restrict__ boxes,
                                          const uint32_t *__restrict__ order, int64_t idx, int TW, int TH,
                                          uint32_t &tiles, uint32_t &rows, uint2 &box)
{
    tiles = rows = 0u;
    box = make_uint2(0u, 0u);
    if (keys[idx] != 0xffffffffu) {
        box = boxes[order[idx]];
        const PixelBox pb = unpack_box(box);
        rows = (uint32_t)(pb.y1 / TH - pb.y0 / TH + 1);
        tiles = rows * (uint32_t)(pb.x1 / TW - pb.x0 / TW + 1);
    }
}

// Gathers each sorted item's two counts once (into `tiles` and `rows`, read
// back by k_scan_apply, which scans them in place) and reduces them per block.
// The gathered binning box is also stored in depth order (`sorted_boxes`), so
// the emission kernel reads it coalesced instead of gathering it again.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ keys,
                                                          const uint2 *__restrict__ boxes,
                                                          const uint32_t *__restrict__ order, int64_t n_max,
                                                          const int64_t *__restrict__ n_dev, int TW, int TH,
                                                          uint32_t *__restrict__ tiles, uint32_t *__restrict__ rows,
                                                          uint2 *__restrict__ sorted_boxes,
                                                          unsigned long long *__restrict__ block_sums)
{
    const int64_t n = clamp_count(n_dev, n_max);
    __shared__ unsigned long long part[2][kWaves];
    const int64_t base = (int64_t)blockIdx.x * scan_tile(ITEMS);
    unsigned long long at = 0, ar = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = base + (int64_t)j * kThreads + threadIdx.x;
        if (idx < n) {
            uint32_t t, r;
            uint2 box;
            scan_item(keys, boxes, order, idx, TW, TH, t, r, box);
            tiles[idx] = t;
            rows[idx] = r;
            sorted_boxes[idx] = box;
            at += t;
            ar += r;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        at += __shfl_xor(at, d, 64);
        ar += __shfl_xor(ar, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = at;
        part[1][threadIdx.x >> 6] = ar;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const unsigned long long *p = part[threadIdx.x];
        block_sums[2 * blockIdx.x + threadIdx.x] = p[0] + p[1] + p[2] + p[3];
    }
}

// Single-block exclusive scan of the block-sum pairs; writes the two totals
// to counters[0] (instances) and counters[2] (tile rows).
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long *__restrict__ block_sums, int nb,
                                                   int64_t *__restrict__ counters)
{
    __shared__ unsigned long long wsum[2][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long carry[2] = {0, 0};
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        unsigned long long x[2], v[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            x[c] = i < nb ? block_sums[2 * i + c] : 0ull;
            v[c] = x[c];
        }
        for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const unsigned long long y = __shfl_up(v[c], d, 64);
                if (lane >= d) v[c] += y;
            }
        }
        if (lane == 63) {
            wsum[0][wave] = v[0];
            wsum[1][wave] = v[1];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            unsigned long long before = 0, all = 0;
            for (int w = 0; w < 16; ++w) {
                if (w < wave) before += wsum[c][w];
                all += wsum[c][w];
            }
            if (i < nb) block_sums[2 * i + c] = carry[c] + before + v[c] - x[c];
            carry[c] += all;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counters[0] = (int64_t)carry[0];
        counters[2] = (int64_t)carry[1];
    }
}

// Sums of the (tiles, rows) block-sum pairs of the blocks before `block`
// (pre) and of all nb blocks (all), the same in every thread.
__device__ void block_prefix_pairs(const unsigned long long *__restrict__ block_sums, int nb, int block,
                                   unsigned long long (&pre)[2], unsigned long long (&all)[2])
{
    __shared__ unsigned long long part[4][kWaves];
    unsigned long long v[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        const unsigned long long t = block_sums[2 * i], r = block_sums[2 * i + 1];
        v[2] += t;
        v[3] += r;
        if (i < block) {
            v[0] += t;
            v[1] += r;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        for (int d = 32; d >= 1; d >>= 1) v[c] += __shfl_xor(v[c], d, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) part[c][threadIdx.x >> 6] = v[c];
    __syncthreads();
    pre[0] = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    pre[1] = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    all[0] = part[2][0] + part[2][1] + part[2][2] + part[2][3];
    all[1] = part[3][0] + part[3][1] + part[3][2] + part[3][3];
}

// Offsets of every sorted item, scanned in place over the counts k_scan_reduce
// left in `offsets` (box tiles) and `row_offsets` (tile rows), plus the owner
// map of the tile rows (row_owner[r] = sorted position owning row r) when the
// instances fit.  The map is written per item (each thread the rows of its
// own items) or, with `rows_in_order`, in row order by consecutive threads,
// each looking its row's owner up in the block's item table.  Row order
// coalesces the stores, which pays off at tens of millions of items; with a
// few hundred blocks the lookups' latency is exposed and per item is faster.
// With `self_prefix` (few blocks), block_sums still holds every block's raw
// pair: each block sums the pairs before its own and all of them, block 0
// writes the totals to counters[0] and counters[2], and k_scan_top is not
// launched.  Otherwise k_scan_top has turned block_sums into exclusive
// prefixes and written the totals.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_scan_apply(int64_t n_max, const int64_t *__restrict__ n_dev,
                                                         int64_t capacity,
                                                         const unsigned long long *__restrict__ block_sums,
                                                         int64_t *__restrict__ counters, bool self_prefix,
                                                         bool rows_in_order, uint32_t *__restrict__ offsets,
                                                         uint32_t *__restrict__ row_offsets,
                                                         uint32_t *__restrict__ row_owner)
{
    static_assert(ITEMS % 4 == 0, "whole 16-byte loads per thread");
    __shared__ uint32_t smem[kWaves];
    const int64_t n = clamp_count(n_dev, n_max);
    // blocked arrangement: thread t owns items base + t*ITEMS .. (aligned 16-byte groups)
    const int64_t base = (int64_t)blockIdx.x * scan_tile(ITEMS) + (int64_t)threadIdx.x * ITEMS;
    uint32_t c[ITEMS], r[ITEMS];
    if (base + ITEMS <= n) {
        const uint4 *pc = reinterpret_cast<const uint4 *>(offsets + base);
        const uint4 *pr = reinterpret_cast<const uint4 *>(row_offsets + base);
#pragma unroll
        for (int v = 0; v < ITEMS / 4; ++v) {
            const uint4 cv = pc[v], rv = pr[v];
            c[4 * v] = cv.x; c[4 * v + 1] = cv.y; c[4 * v + 2] = cv.z; c[4 * v + 3] = cv.w;
            r[4 * v] = rv.x; r[4 * v + 1] = rv.y; r[4 * v + 2] = rv.z; r[4 * v + 3] = rv.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool in = base + j < n;
            c[j] = in ? offsets[base + j] : 0u;
            r[j] = in ? row_offsets[base + j] : 0u;
        }
    }
    uint32_t lt = 0, lr = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        lt += c[j];
        lr += r[j];
    }
    uint32_t tot;
    const uint32_t bt = block_inclusive_scan(lt, smem, &tot) - lt;
    const uint32_t br = block_inclusive_scan(lr, smem, &tot) - lr;
    unsigned long long pre[2], all[2];
    if (self_prefix) {
        block_prefix_pairs(block_sums, (int)gridDim.x, (int)blockIdx.x, pre, all);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            counters[0] = (int64_t)all[0];
            counters[2] = (int64_t)all[1];
        }
    } else {
        pre[0] = block_sums[2 * blockIdx.x];
        pre[1] = block_sums[2 * blockIdx.x + 1];
        all[0] = (unsigned long long)counters[0];
    }
    const uint32_t block_rows = tot;  // tile rows of the block's items
    const bool fits = all[0] <= (unsigned long long)capacity;
    unsigned long long rt = pre[0] + bt;
    unsigned long long rr = pre[1] + br;
    // first row of each of the block's items, relative to the block's first row
    __shared__ uint32_t row_start[scan_tile(ITEMS)];
    uint32_t lr0 = br;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int64_t idx = base + j;
        if (idx < n) {
            offsets[idx] = rt > 0xffffffffull ? 0xffffffffu : (uint32_t)rt;
            row_offsets[idx] = rr > 0xffffffffull ? 0xffffffffu : (uint32_t)rr;
            // rows <= instances, so every row index lies below capacity
            if (fits && !rows_in_order)
                for (uint32_t q = 0; q < r[j]; ++q) row_owner[rr + q] = (uint32_t)idx;
        }
        row_start[threadIdx.x * ITEMS + j] = lr0;
        rt += c[j];
        rr += r[j];
        lr0 += r[j];
    }
    if (!fits || !rows_in_order) return;  // uniform over the grid
    __syncthreads();
    // owner map of the block's rows, written in row order by consecutive
    // threads: the owner of row q is the last item whose first row is <= q
    // (items without rows share the first row of the next item)
    const int64_t block_base = (int64_t)blockIdx.x * scan_tile(ITEMS);
    const int nvalid = (int)min((int64_t)scan_tile(ITEMS), n - block_base);
    const unsigned long long row0 = pre[1];
    for (uint32_t q = threadIdx.x; q < block_rows; q += kThreads) {
        int lo = 0, hi = nvalid;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (row_start[mid] <= q)
                lo = mid;
            else
                hi = mid;
        }
        // rows <= instances, so every row index lies below capacity
        row_owner[row0 + q] = (uint32_t)(block_base + lo);
    }
}

// ---------------------------------------------------------------- emission
// One lane per tile row of the sorted Gaussian-views (a grid-stride loop
// over the row count the scan produced): the lane computes the support's
// x-extent over the row and over its rows of pixel slots and writes every
// tile of the box row at its scanned position, as (tile id, id | slot bits)
// when the tile's pixel-centre rectangle meets the support and as the empty
// marker `empty_tile` otherwise.  Instances end up
// grouped by Gaussian-view in depth order, so a stable sort on the tile id
// alone leaves every tile's list in depth order.  The kernel also clears the
// tile ranges and the compositing scheduling words for the stages after the
// tile sort (`clear` holds clear_words uint32 at `clear_a`, then `clear_b`).
// Instantiated per tile shape, so the slot layout of the culling bits is
// constant.
template <int TW, int TH>
__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t *__restrict__ order,
                                                   const uint32_t *__restrict__ offsets,
                                                   const uint32_t *__restrict__ row_offsets,
                                                   const uint32_t *__restrict__ row_owner,
                                                   const uint2 *__restrict__ sorted_boxes,
                                                   const Conic *__restrict__ conics,
                                                   const DevView *__restrict__ views, int64_t n,
                                                   const int64_t *__restrict__ counters, int64_t capacity,
                                                   uint32_t empty_tile, uint32_t *__restrict__ inst_tiles,
                                                   uint32_t *__restrict__ inst_ids, uint32_t *__restrict__ clear_a,
                                                   int64_t clear_a_words, uint32_t *__restrict__ clear_b,
                                                   int64_t clear_b_words)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    for (int64_t i = tid; i < clear_a_words; i += stride) clear_a[i] = 0u;
    for (int64_t i = tid; i < clear_b_words; i += stride) clear_b[i] = 0u;
    if (counters[0] > capacity) return;  // overflow: the instance total reports it
    const int64_t rows = counters[2];
    for (int64_t r = tid; r < rows; r += stride) {
        const uint32_t k = row_owner[r];
        const uint32_t id = order[k];
        const PixelBox pb = unpack_box(sorted_boxes[k]);
        const int v = (int)(id / (uint32_t)n);
        const int row = (int)(r - row_offsets[k]);
        const int ty = pb.y0 / TH + row;
        const int tx0 = pb.x0 / TW, tx1 = pb.x1 / TW;
        int64_t pos = (int64_t)offsets[k] + (int64_t)row * (tx1 - tx0 + 1);
        const Conic C = conics[id];
        const ConicFrame F = conic_frame(C);
        BandRanges B;
        band_ranges(C, F, pb, ty, TW, TH, B);
        const uint32_t row_base = (uint32_t)views[v].tile_base + (uint32_t)(ty * views[v].tiles_x);
        for (int tx = tx0; tx <= tx1; ++tx, ++pos) {
            uint32_t bands;
            const bool listed = tile_listed(C, B, pb, tx, TW, TH, bands);
            inst_tiles[pos] = listed ? row_base + (uint32_t)tx : empty_tile;
            inst_ids[pos] = pack_instance(id, bands, TW, TH);
        }
    }
}

// ------------------------------------------------------------ tile ranges
__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void k_copy_i64(const int64_t *__restrict__ src, int64_t *__restrict__ dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

// Each thread takes four consecutive positions per step (one 16-byte load and
// the two neighbours), so the grid-stride loop keeps four times as many loads
// in flight per step as one position per thread would.
__global__ __launch_bounds__(kThreads) void k_tile_ranges(const uint32_t *__restrict__ inst_tiles,
                                                          const int64_t *__restrict__ counters, int64_t capacity,
                                                          int64_t total_tiles, uint2 *__restrict__ ranges)
{
    const int64_t m = clamp_count(counters, capacity);
    const int64_t groups = (m + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    constexpr uint32_t kNone = 0xffffffffu;  // no neighbour (never a tile id)
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < groups; g += stride) {
        const int64_t p0 = 4 * g;
        uint32_t t[6];  // tiles at positions p0 - 1 .. p0 + 4
        if (p0 + 4 <= m) {
            const uint4 v = *reinterpret_cast<const uint4 *>(inst_tiles + p0);
            t[1] = v.x;
            t[2] = v.y;
            t[3] = v.z;
            t[4] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) t[1 + j] = p0 + j < m ? inst_tiles[p0 + j] : kNone;
        }
        t[0] = p0 > 0 ? inst_tiles[p0 - 1] : kNone;
        t[5] = p0 + 4 < m ? inst_tiles[p0 + 4] : kNone;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t tj = t[1 + j];
            if (tj >= total_tiles) continue;  // also past the end (kNone)
            if (t[j] != tj) ranges[tj].x = (uint32_t)(p0 + j);
            if (t[j + 2] != tj) ranges[tj].y = (uint32_t)(p0 + j + 1);
        }
    }
}

// -------------------------------------------------------- tile scheduling
// Work order of the compositing kernels: work items sorted by decreasing list
// length (coarse buckets of 4 entries, order inside a bucket arbitrary), so
// the longest lists start first and the persistent grid drains evenly.  A
// tile whose list is longer than the average work of a compositing wave
// (listed instances / waves, at least split_min; split_min 0: never split)
// becomes two items, each compositing half of the tile's pixel rows against
// the whole list, which halves the longest chains of dependent work.  Item
// value = tile << 2 | part (0 whole tile, 1 first half, 2 second half).
constexpr int kSchedBuckets = 256;
constexpr int64_t kRangeBlocks = 4096;

__device__ __forceinline__ uint32_t work_bucket(uint32_t len)
{
    return min(len >> 2, (uint32_t)(kSchedBuckets - 1));
}

__device__ __forceinline__ uint32_t split_length(const int64_t *listed, uint32_t split_min, uint32_t waves)
{
    if (split_min == 0u) return 0u;
    const int64_t share = (*listed + waves - 1) / waves;
    return (uint32_t)max((int64_t)split_min, share);
}

__device__ __forceinline__ uint32_t work_parts(uint32_t len, uint32_t split_len)
{
    return (split_len != 0u && len >= split_len) ? 2u : 1u;
}

__global__ __launch_bounds__(kThreads) void k_sched_hist(const uint2 *__restrict__ ranges, int64_t total_tiles,
                                                         const int64_t *__restrict__ listed, uint32_t split_min,
                                                         uint32_t waves, uint32_t *__restrict__ hist)
{
    const uint32_t split_len = split_length(listed, split_min, waves);
    __shared__ uint32_t cnt[kSchedBuckets];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t < total_tiles) {
        const uint2 r = ranges[t];
        atomicAdd(&cnt[work_bucket(r.y - r.x)], work_parts(r.y - r.x, split_len));
    }
    __syncthreads();
    if (cnt[threadIdx.x]) atomicAdd(&hist[threadIdx.x], cnt[threadIdx.x]);
}

__global__ __launch_bounds__(kThreads) void k_sched_scatter(const uint2 *__restrict__ ranges, int64_t total_tiles,
                                                            const int64_t *__restrict__ listed, uint32_t split_min,
                                                            uint32_t waves, const uint32_t *__restrict__ hist,
                                                            uint32_t *__restrict__ cursor,
                                                            uint32_t *__restrict__ n_items,
                                                            uint32_t *__restrict__ work_order)
{
    __shared__ uint32_t smem[kWaves];
    __shared__ uint32_t base[kSchedBuckets];
    __shared__ uint32_t cnt[kSchedBuckets];
    const uint32_t split_len = split_length(listed, split_min, waves);
    // buckets in decreasing order: bucket b starts after all items of buckets > b
    const uint32_t hb = hist[kSchedBuckets - 1 - threadIdx.x];
    uint32_t tot;
    const uint32_t before = block_inclusive_scan(hb, smem, &tot) - hb;
    base[kSchedBuckets - 1 - threadIdx.x] = before;
    cnt[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_items = tot;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t b = 0, rank = 0, parts = 0;
    if (t < total_tiles) {
        const uint2 r = ranges[t];
        b = work_bucket(r.y - r.x);
        parts = work_parts(r.y - r.x, split_len);
        rank = atomicAdd(&cnt[b], parts);
    }
    __syncthreads();
    if (cnt[threadIdx.x]) base[threadIdx.x] += atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (parts == 1u) work_order[base[b] + rank] = (uint32_t)t << 2;
    if (parts == 2u) {
        work_order[base[b] + rank] = (uint32_t)t << 2 | 1u;
        work_order[base[b] + rank + 1] = (uint32_t)t << 2 | 2u;
    }
}

}  // namespace

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

// sized for the smallest tile, so any choice of ITEMS fits
size_t radix_hist_entries(int64_t n_max)
{
    const int64_t tile = radix_tile(kRadixItemsMin);
    return (size_t)kBins * (size_t)((n_max + tile - 1) / tile + 1);
}

namespace {
// Keys per thread by sort size, from timings of the depth and tile sorts of a
// 1080p frame (0.5M and 2.6M keys) and of an 8-view batch (24M and 91M).
int radix_items_for(int64_t n_max) { return n_max <= (int64_t(1) << 20) ? 4 : n_max <= (int64_t(1) << 24) ? 8 : 16; }

template <int ITEMS>
void radix_pass(const uint32_t *ki, const uint32_t *vi, uint32_t *ko, uint32_t *vo, int64_t n_max,
                const int64_t *pn, int shift, int pbits, bool pdrop, uint32_t drop_key, int64_t *kept_out,
                uint32_t *hist, uint32_t *row_total, hipStream_t stream)
{
    const int nblocks = (int)((n_max + radix_tile(ITEMS) - 1) / radix_tile(ITEMS));
    k_radix_hist<ITEMS><<<nblocks, kThreads, 0, stream>>>(ki, n_max, pn, shift, pbits, pdrop, drop_key, hist, nblocks);
    k_radix_scan_rows<<<kBins, kThreads, 0, stream>>>(hist, nblocks, n_max, pn, radix_tile(ITEMS), row_total);
    k_radix_scatter<ITEMS><<<nblocks, kThreads, 0, stream>>>(ki, vi, ko, vo, n_max, pn, shift, pbits, pdrop, drop_key,
                                                             kept_out, hist, row_total, nblocks);
}
}  // namespace

hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n_max,
                      const int64_t *n_dev, int bits, bool drop, uint32_t drop_key, int64_t *kept_out,
                      uint32_t *hist, uint32_t *row_total, hipStream_t stream, bool iota)
{
    const int passes = radix_passes(bits);
    const int items = radix_items_for(n_max);
    if (n_max <= 0 || passes == 0) {
        if (drop) k_fill_u32<<<1, kThreads, 0, stream>>>(reinterpret_cast<uint32_t *>(kept_out), 0u, 2);
        return hipGetLastError();
    }
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        // spread the bits evenly over the passes (each <= 8); the first pass
        // drops, the later ones sort the kept items
        const int pbits = (bits - shift + (passes - p) - 1) / (passes - p);
        const bool pdrop = drop && p == 0;
        const int64_t *pn = drop && p > 0 ? kept_out : n_dev;
        const uint32_t *pvi = iota && p == 0 ? nullptr : vi;
        if (items == 4)
            radix_pass<4>(ki, pvi, ko, vo, n_max, pn, shift, pbits, pdrop, drop_key, kept_out, hist, row_total, stream);
        else if (items == 8)
            radix_pass<8>(ki, pvi, ko, vo, n_max, pn, shift, pbits, pdrop, drop_key, kept_out, hist, row_total, stream);
        else
            radix_pass<16>(ki, pvi, ko, vo, n_max, pn, shift, pbits, pdrop, drop_key, kept_out, hist, row_total, stream);
        shift += pbits;
        uint32_t *t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    return hipGetLastError();
}

// sized for the smallest tile, so either choice of items per thread fits
size_t scan_block_entries(int64_t n)
{
    const int64_t tile = scan_tile(kScanItemsMin);
    return 2 * (size_t)((n + tile - 1) / tile + 1);
}

namespace {
template <int ITEMS>
void scan_launch(const uint32_t *keys, const uint2 *boxes, const uint32_t *order, int64_t n, const int64_t *n_dev,
                 int tile_w, int tile_h, int64_t capacity, uint32_t *offsets, uint32_t *row_offsets,
                 uint32_t *row_owner, uint2 *sorted_boxes, unsigned long long *block_sums, int64_t *counters,
                 hipStream_t stream)
{
    const int nb = (int)((n + scan_tile(ITEMS) - 1) / scan_tile(ITEMS));
    k_scan_reduce<ITEMS><<<nb, kThreads, 0, stream>>>(keys, boxes, order, n, n_dev, tile_w, tile_h, offsets,
                                                      row_offsets, sorted_boxes, block_sums);
    // up to kScanSelfPrefixBlocks blocks, each apply block sums the block
    // pairs before it (at most that many loads) instead of a separate scan
    const bool self_prefix = nb <= kScanSelfPrefixBlocks;
    if (!self_prefix) k_scan_top<<<1, 1024, 0, stream>>>(block_sums, nb, counters);
    k_scan_apply<ITEMS><<<nb, kThreads, 0, stream>>>(n, n_dev, capacity, block_sums, counters, self_prefix,
                                                     nb >= kScanRowOrderBlocks, offsets, row_offsets, row_owner);
}
}  // namespace

hipError_t binning_scan(const uint32_t *keys, const uint2 *boxes, const uint32_t *order, int64_t n,
                        const int64_t *n_dev, int tile_w, int tile_h, int64_t capacity, uint32_t *offsets,
                        uint32_t *row_offsets, uint32_t *row_owner, uint2 *sorted_boxes,
                        unsigned long long *block_sums, int64_t *counters, hipStream_t stream)
{
    if (n <= 0) {
        // counters[0] and counters[2] (int64) = 0, counters[1] (capacity) kept
        k_fill_u32<<<1, kThreads, 0, stream>>>(reinterpret_cast<uint32_t *>(counters), 0u, 2);
        k_fill_u32<<<1, kThreads, 0, stream>>>(reinterpret_cast<uint32_t *>(counters + 2), 0u, 2);
        return hipGetLastError();
    }
    if (n <= (int64_t(1) << 20))
        scan_launch<4>(keys, boxes, order, n, n_dev, tile_w, tile_h, capacity, offsets, row_offsets, row_owner,
                       sorted_boxes, block_sums, counters, stream);
    else
        scan_launch<8>(keys, boxes, order, n, n_dev, tile_w, tile_h, capacity, offsets, row_offsets, row_owner,
                       sorted_boxes, block_sums, counters, stream);
    return hipGetLastError();
}

int emit_grid(int num_cus) { return 8 * num_cus; }

hipError_t launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *row_offsets,
                       const uint32_t *row_owner, const uint2 *sorted_boxes, const Conic *conics, const DevView *views,
                       int64_t n, int n_views, const int64_t *counters, int64_t capacity, int tile_w, int tile_h,
                       uint32_t empty_tile, uint32_t *inst_tiles, uint32_t *inst_ids, uint2 *ranges,
                       int64_t total_tiles, uint32_t *sched, int grid, hipStream_t stream)
{
    // runs even with no Gaussian: it clears the ranges and scheduling words
#define RGS_EMIT(W, H)                                                                                               \
    if (tile_w == W && tile_h == H) {                                                                                \
        k_emit<W, H><<<grid, kThreads, 0, stream>>>(order, offsets, row_offsets, row_owner, sorted_boxes, conics,     \
                                                    views, n > 0 ? n : 1, counters, capacity, empty_tile, inst_tiles, \
                                                    inst_ids, reinterpret_cast<uint32_t *>(ranges), 2 * total_tiles,  \
                                                    sched, (int64_t)sched_words());                                   \
        return hipGetLastError();                                                                                    \
    }
    RGS_EMIT(8, 8)
    RGS_EMIT(8, 16)
    RGS_EMIT(8, 32)
    RGS_EMIT(16, 8)
    RGS_EMIT(16, 16)
    RGS_EMIT(16, 32)
    RGS_EMIT(32, 8)
    RGS_EMIT(32, 16)
    RGS_EMIT(32, 32)
#undef RGS_EMIT
    (void)n_views;
    return hipErrorInvalidValue;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    k_fill_u32<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, stream>>>(p, value, n);
    return hipGetLastError();
}

hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, hipStream_t stream)
{
    k_copy_i64<<<1, 64, 0, stream>>>(src, dst);
    return hipGetLastError();
}

size_t sched_backward_heads() { return (size_t)kQueues * kQueueStride; }
size_t sched_item_count() { return 2 * sched_backward_heads() + 2 * kSchedBuckets; }
size_t sched_words() { return sched_item_count() + 4; }

hipError_t launch_tile_ranges(const uint32_t *inst_tiles, const int64_t *counters, int64_t capacity,
                              int64_t total_tiles, uint32_t split_min, uint32_t waves, uint2 *ranges,
                              uint32_t *sched, uint32_t *work_order, hipStream_t stream)
{
    // the ranges, queue heads and scheduling histograms were cleared by k_emit
    // a grid-stride loop over the listed instances (a grid sized for the whole
    // capacity would mostly launch idle workgroups)
    if (capacity > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>((capacity + 4 * kThreads - 1) / (4 * kThreads), kRangeBlocks);
        k_tile_ranges<<<grid, kThreads, 0, stream>>>(inst_tiles, counters, capacity, total_tiles, ranges);
    }
    const unsigned nb = (unsigned)((total_tiles + kThreads - 1) / kThreads);
    uint32_t *hist = sched + 2 * sched_backward_heads(), *cursor = hist + kSchedBuckets;
    k_sched_hist<<<nb, kThreads, 0, stream>>>(ranges, total_tiles, counters, split_min, waves, hist);
    k_sched_scatter<<<nb, kThreads, 0, stream>>>(ranges, total_tiles, counters, split_min, waves, hist, cursor,
                                                 sched + sched_item_count(), work_order);
    return hipGetLastError();
}

}  // namespace rgs
