// Internal declarations shared by the HIP translation units of the renderer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "raygs.h"

namespace rgs {

// Per-view table, device resident (one entry per camera of the batch).
struct DevView {
    double w2c[12];        // row-major [R | t]
    double fx, fy, cx, cy;
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

// Gradient of one record as accumulated by the backward compositing kernel:
//   du0, dv0, dM00, dM01, dM11, dgx, dgy, dk0, dic2, do, dr, dg, db (13 used)
// where M = G^T G (q = delta^T M delta; dM01 is the derivative with respect to
// the single off-diagonal parameter) and do = dL / d(prior opacity).
constexpr int kGradFloats = 16;

constexpr int kMaxViews = 256;

struct TileShape {
    int w, h;
};

// ---- launchers (each enqueues on `stream`, returns hipError_t) -----------
hipError_t launch_preprocess(const rgs_gaussians &g, const DevView *views, int n_views, const DevOptions &opt,
                             float4 *records, uint32_t *depth_keys, uint32_t *order, uint2 *rects,
                             uint32_t *tile_counts, hipStream_t stream);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits).  n_dev (may
// be null) holds a device-side element count, clamped to n_max.  Ping-pongs
// between (keys, vals) and (keys_alt, vals_alt): the result lands in the
// primary buffers when the pass count is even, else in the alternates.
int radix_passes(int bits);
hipError_t radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n_max,
                      const int64_t *n_dev, int bits, uint32_t *hist, uint32_t *row_total, hipStream_t stream);
size_t radix_hist_entries(int64_t n_max);

// offsets[k] = sum_{j<k} counts[gather[k]], counters[0] = total (int64).
hipError_t exclusive_scan_gather(const uint32_t *counts, const uint32_t *gather, uint32_t *offsets, int64_t n,
                                 unsigned long long *block_sums, int64_t *total, hipStream_t stream);
size_t scan_block_entries(int64_t n);

hipError_t launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *tile_counts, const uint2 *rects,
                       const DevView *views, int64_t n, int n_views, int64_t capacity, uint32_t *inst_tiles,
                       uint32_t *inst_ids, hipStream_t stream);

// Tile ranges of the sorted instances plus the compositing work order
// (tile ids by decreasing list length).  `sched` holds sched_words() uint32:
// [0] forward queue head, [1] backward queue head, [4..) bucket histograms.
size_t sched_words();
hipError_t launch_tile_ranges(const uint32_t *inst_tiles, const int64_t *counters, int64_t capacity,
                              int64_t total_tiles, uint2 *ranges, uint32_t *sched, uint32_t *tile_order,
                              hipStream_t stream);

hipError_t launch_blend(TileShape shape, const uint2 *ranges, const uint32_t *tile_order, const uint32_t *inst_ids,
                        const float4 *records,
                        const DevView *views, int n_views, int64_t total_tiles, int64_t n_records,
                        const DevOptions &opt, unsigned int *queue, int grid, hipStream_t stream);
int blend_grid(TileShape shape, int num_cus);

hipError_t launch_blend_backward(TileShape shape, const uint2 *ranges, const uint32_t *tile_order,
                                 const uint32_t *inst_ids,
                                 const float4 *records, const DevView *views, int n_views, int64_t total_tiles,
                                 int64_t n_records, const DevOptions &opt, float *record_grads, unsigned int *queue,
                                 int grid, hipStream_t stream);
int blend_backward_grid(TileShape shape, int num_cus);

hipError_t launch_preprocess_backward(const rgs_gaussians &g, const DevView *views, int n_views,
                                      const DevOptions &opt, const uint32_t *tile_counts, const float *record_grads,
                                      const rgs_gaussian_grads &grads, hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t stream);

bool tile_shape_supported(int w, int h);

}  // namespace rgs
