// Internal declarations shared by the HIP translation units of the renderer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "binning.h"
#include "raygs.h"

namespace rgs {

// Per-view table, device resident (one entry per camera of the batch).
struct DevView {
    double w2c[12];        // row-major [R | t]
    double fx, fy, cx, cy;
    double ifx, ify;       // 1 / fx, 1 / fy
    double centre[3];      // camera centre in world coordinates, -R^T t
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;     // first global tile id of this view
    int32_t pad;
    float *rgb;            // [3][H][W]
    float *final_T;        // [H][W]
    int32_t *n_contrib;    // [H][W]
    const float *dL_drgb;  // [3][H][W] (backward only)
};

struct DevOptions {
    double p_min, alpha_max, t_eps, near_z, mip_sigma2_px;
    int32_t mip;
    int32_t tile_w, tile_h;
    int32_t tile_wshift, tile_hshift;  // log2 of the tile shape (powers of two)
    int32_t divergence;  // RGS_DIVERGENCE_*
    float bg[3];
};

// Raster record of one Gaussian-view, 16 floats (64 B), written by the
// preprocess kernel and read by the compositing kernels:
//   [0] u_hi, v_hi, lo, rows     projected centre pi(mu) = (u_hi, v_hi) + lo where
//                                lo = (u_lo, v_lo) as an fp16 pair (bits); rows =
//                                first | last << 16 covered pixel row (bits)
//   [1] G00, G01, G10, G11       pixel offset -> quad-plane coordinate (whitened)
//   [2] gx, gy, k0, ic2          den = k0 + g . delta, ic2 = 1 / c^2
//   [3] log2o, r, g, b           log2 of the prior opacity, colour
constexpr int kRecordFloats = 16;

// With exact MIP (mip = 2) the record is 28 floats (seven float4, 112 B): the
// Gaussian in its own axes, for the per-ray widening (layout in blend.hip).
constexpr int kRecordFloatsExactMip = 28;

inline int record_floats(int mip) { return mip == 2 ? kRecordFloatsExactMip : kRecordFloats; }

// Where r, g, b sit in a record: floats first, first + step, first + 2 step
// (13, 14, 15; with exact MIP 15, 19, 23).
struct ColourSlot {
    int first, step;
};
__host__ __device__ constexpr ColourSlot colour_slot(int mip) { return mip == 2 ? ColourSlot{15, 4} : ColourSlot{13, 1}; }

// Gradient of one record as accumulated by the backward compositing kernel,
// as sums over its fragments (13 used):
//   [0, 1]  sum e dx, sum e dy          [2, 3, 4]  sum e dx^2, e dx dy, e dy^2
//   [5, 6]  sum f dx, sum f dy          [7]        sum f
//   [8]     sum ew q^2                  [9]        sum w dL/dw
//   [10..12] dL/d(colour)
// with (dx, dy) the pixel offset from the projected centre, q and den the
// fragment's quadratic and denominator in the test form (q_s = s^2 q, 1 / s^2
// = 2 ln 2 K, K = log2(record opacity / p_min)), ew = w dL/dw / t^2, e = ew
// den^2 and f = ew q_s den (sum w dL/dw is the record opacity times the
// derivative with respect to it).  The per-Gaussian backward turns them into the
// derivatives with respect to the record's u0, v0, M = G^T G, g, k0 and 1/c^2
// (k_preprocess_bwd in backward.hip).
constexpr int kGradFloats = 16;

// With exact MIP (mip = 2) the record gradient is 32 floats (layout at the
// exact MIP backward compositing kernel in blend.hip; 25 used).
constexpr int kGradFloatsExactMip = 32;

__host__ __device__ inline int grad_floats(int mip) { return mip == 2 ? kGradFloatsExactMip : kGradFloats; }

constexpr int kMaxViews = 256;

struct TileShape {
    int w, h;
};

// ---- launchers (each enqueues on `stream`, returns hipError_t) -----------
// Writes per Gaussian-view: the record (its colour for every view, culled or
// not), depth key (0xffffffff when culled), pixel box, binning box (the
// pixels of the pixel box whose centres lie in the support ellipse's bounding
// box; culled when there are none), support conic, and the number of tiles
// of the binning box (0 when culled).  A quad with a vertex at z <= 0 is first
// given the whole view; its parameters go to the crossing list (kCrossingDoubles
// doubles per entry, at most crossing_cap entries, *crossing_count zero on
// entry), and a second kernel bounds its box by the part of the quad inside
// the view frustum.  Entries beyond the cap keep the whole view.
constexpr int kCrossingDoubles = 12;
hipError_t launch_preprocess(const rgs_gaussians &g, const DevView *views, int n_views, const DevOptions &opt,
                             float4 *records, uint32_t *depth_keys, uint2 *boxes, uint2 *bin_boxes, Conic *conics,
                             uint32_t *tile_counts, double *crossing, int64_t *crossing_count,
                             uint32_t crossing_cap, hipStream_t stream);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits), 8-bit digits
// (with `iota` the input values are not read: they are the positions 0, 1,
// 2, ...)
// (radix_passes(bits) passes of a per-workgroup digit histogram, a scan of
// each digit's row over the workgroups, and a stable scatter).  n_dev (may
// be null) holds a device-side element count, clamped to n_max.  With
// `drop`, elements whose key equals drop_key leave the sort in the first
// pass; the kept elements end up sorted in [0, *kept_out) (int64, device,
// written).  Ping-pongs between (keys, vals) and (keys_alt, vals_alt): the
// result lands in the primary buffers when the pass count is even, else in
// the alternates.
int radix_passes(int bits);
hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n_max,
                      const int64_t *n_dev, int bits, bool drop, uint32_t drop_key, int64_t *kept_out,
                      uint32_t *hist, uint32_t *row_total, hipStream_t stream, bool iota = false);
size_t radix_hist_entries(int64_t n_max);

// Binning scan over the depth order (Gaussian-view order[k] at position k,
// sorted key keys[k], 0xffffffff when culled; positions k < *n_dev, at most
// n): offsets[k] = box tiles and
// row_offsets[k] = box tile rows of the positions before k; counters[0] =
// all box tiles (instances), counters[2] = all tile rows (int64);
// row_owner[r] = k for each tile row r of position k, written when the
// instances fit `capacity` (row_owner holds capacity entries);
// sorted_boxes[k] = boxes[order[k]] (n entries).  block_sums holds
// scan_block_entries(n) uint64.
hipError_t binning_scan(const uint32_t *keys, const uint2 *boxes, const uint32_t *order, int64_t n,
                        const int64_t *n_dev, int tile_w, int tile_h, int64_t capacity, uint32_t *offsets,
                        uint32_t *row_offsets, uint32_t *row_owner, uint2 *sorted_boxes,
                        unsigned long long *block_sums, int64_t *counters, hipStream_t stream);
size_t scan_block_entries(int64_t n);

// Instances of every tile row (one lane per row, `grid` workgroups looping
// over counters[2] rows): (tile id, id | slot bits) for listed tiles and
// (empty_tile, id) for the other tiles of the box.  Also zeroes `ranges`
// (total_tiles entries) and `sched` (sched_words()) for the stages after the
// tile sort; always launched, also for an empty scene.
int emit_grid(int num_cus);
hipError_t launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *row_offsets,
                       const uint32_t *row_owner, const uint2 *sorted_boxes, const Conic *conics, const DevView *views,
                       int64_t n, int n_views, const int64_t *counters, int64_t capacity, int tile_w, int tile_h,
                       uint32_t empty_tile, uint32_t *inst_tiles, uint32_t *inst_ids, uint2 *ranges,
                       int64_t total_tiles, uint32_t *sched, int grid, hipStream_t stream);

// Compositing work queues: kQueues heads per pass, kQueueStride words apart
// (separate memory lines, so their atomics do not serialise on one
// address); workgroup b takes queue b % min(grid, kQueues) and queue q hands
// out the work-order slots q, q + nq, q + 2 nq, ...
constexpr int kQueues = 8;
constexpr int kQueueStride = 1024;

// Tile ranges of the `*counters` sorted instances plus the compositing work
// order: work items tile << 2 | part (0 whole tile; 1, 2 the first and
// second half of its pixel rows, for tiles whose list is longer than
// max(split_min, *counters / waves), split_min 0 = never split) by
// decreasing list length, at most 2 * total_tiles of them.
// `ranges` and `sched` must be zero (launch_emit clears them).  `sched` holds
// sched_words() uint32: the forward queue heads from word 0, the backward
// heads from sched_backward_heads(), bucket histograms, and the number of
// work items at sched_item_count().
size_t sched_words();
size_t sched_backward_heads();
size_t sched_item_count();
hipError_t launch_tile_ranges(const uint32_t *inst_tiles, const int64_t *counters, int64_t capacity,
                              int64_t total_tiles, uint32_t split_min, uint32_t waves, uint2 *ranges,
                              uint32_t *sched, uint32_t *work_order, hipStream_t stream);

// Shortest list composited as two half-tile work items (for tile shapes with
// at least two pixel slots per lane).
#ifndef RGS_SPLIT_LEN
#define RGS_SPLIT_LEN 256
#endif

// Compositing of the work items work_order[0, *n_items) (see
// launch_tile_ranges); `queue` holds the kQueues heads (zero).
// item_clock (may be null): per work-order slot, the device wall clock when
// the item finished.
hipError_t launch_blend(TileShape shape, const uint2 *ranges, const uint32_t *work_order, const uint32_t *n_items,
                        const uint32_t *inst_ids, const float4 *records, const DevView *views, int n_views,
                        int64_t total_tiles, int64_t n_records, const DevOptions &opt, unsigned int *queue, int grid,
                        unsigned long long *item_clock, hipStream_t stream);

// Per-view completion clocks: stamps[0] = frame start (written by
// launch_view_clock_start, which also clears stamps[1..n_views]), stamps[1 + v]
// = max item clock over view v's work items (launch_view_clock_max, after the
// compositing kernel).
hipError_t launch_view_clock_start(unsigned long long *stamps, int n_views, hipStream_t stream);
hipError_t launch_view_clock_max(const unsigned long long *item_clock, const uint32_t *work_order,
                                 const uint32_t *n_items, int64_t max_items, const DevView *views, int n_views,
                                 unsigned long long *stamps, hipStream_t stream);
int blend_grid(TileShape shape, bool exact_mip, int num_cus);

// Backward compositing over the same work items (whole tiles and halves).
hipError_t launch_blend_backward(TileShape shape, const uint2 *ranges, const uint32_t *work_order,
                                 const uint32_t *n_items, const uint32_t *inst_ids, const float4 *records,
                                 const DevView *views, int n_views, int64_t total_tiles, int64_t n_records,
                                 const DevOptions &opt, float *record_grads, unsigned int *queue, int grid,
                                 hipStream_t stream);
int blend_backward_grid(TileShape shape, bool exact_mip, int num_cus);

hipError_t launch_preprocess_backward(const rgs_gaussians &g, const DevView *views, int n_views,
                                      const DevOptions &opt, const uint32_t *tile_counts, const float *record_grads,
                                      const rgs_gaussian_grads &grads, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t stream);

// *dst = *src (one int64, device to device), stream-ordered.
hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, hipStream_t stream);

// dst[p][y][x] = mean of src[p][y f + r][x f + c] over r, c < f (src is
// [planes][height f][width f]).
hipError_t launch_downsample_box(const float *src, int width, int height, int factor, int planes, float *dst,
                                 hipStream_t stream);

bool tile_shape_supported(int w, int h);

// Adds `amount` to a global counter once per wave and returns the previous
// value in every lane.  Only the first active lane contributes, selected by
// value rather than by a branch: a lane-0 branch in front of the convergent
// read-first-lane inside a persistent loop is loop invariant, and the
// compiler may thread it into the back edge, leaving lanes 1..63 in a loop
// of their own that re-reads a stale value and never exits.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *counter, uint32_t amount)
{
    const unsigned long long active = __ballot(1);
    const bool first = (threadIdx.x & 63u) == (unsigned)__builtin_ctzll(active);
    return __builtin_amdgcn_readfirstlane(atomicAdd(counter, first ? amount : 0u));
}

}  // namespace rgs
